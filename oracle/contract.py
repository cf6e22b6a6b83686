"""O2: pairwise tensor contraction, written out as a loop nest, and
whole-network contraction along a pairwise path (Sec. 3.1).

Label semantics (einsum-like) for C = contract(A, la, B, lb, lc):
    a label in A and B and not in C is summed;
    a label in one input and in C is free;
    a label in A, B and C is a batch label;
    a label in one input only and not in C is summed out of that input.
A label may appear at most once per tensor.

``contract_pair_loops`` iterates every assignment of the union of labels and
accumulates C[out] += A[a] * B[b] (pure Python, for <= ~2^16 index points).
``contract_pair`` is the same definition handed to ``numpy.einsum``, a
library routine; a test pins the two against each other on small cases.
``contract_pair_mm`` writes the same sum as one batched matrix product
(operands transposed to [batch, free, summed] and [batch, summed, free],
then ``numpy.matmul``), for the large contractions of full-size references;
a test pins it against ``contract_pair`` on every label kind.

Parity pins: loop nest == einsum (tests); whole-network contraction ==
state vector (O1); path invariance; slicing invariance.
"""

from __future__ import annotations

import itertools
from typing import Dict, List, Sequence

import numpy as np

_LETTERS = "abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ"


def _check(la, lb, lc):
    for ls in (la, lb, lc):
        if len(set(ls)) != len(ls):
            raise ValueError("repeated label in one tensor")
    if not set(lc) <= set(la) | set(lb):
        raise ValueError("output label not present in any input")


def contract_pair_loops(A: np.ndarray, la: Sequence[int], B: np.ndarray,
                        lb: Sequence[int], lc: Sequence[int]) -> np.ndarray:
    _check(la, lb, lc)
    ext: Dict[int, int] = {}
    for T, ls in ((A, la), (B, lb)):
        for ax, l in enumerate(ls):
            if l in ext and ext[l] != T.shape[ax]:
                raise ValueError("extent mismatch")
            ext[l] = T.shape[ax]
    allv = list(dict.fromkeys(list(la) + list(lb)))
    C = np.zeros(tuple(ext[l] for l in lc), dtype=np.complex128)
    for vals in itertools.product(*[range(ext[l]) for l in allv]):
        env = dict(zip(allv, vals))
        C[tuple(env[l] for l in lc)] += (complex(A[tuple(env[l] for l in la)])
                                         * complex(B[tuple(env[l] for l in lb)]))
    return C


def contract_pair(A, la, B, lb, lc) -> np.ndarray:
    _check(la, lb, lc)
    labs = list(dict.fromkeys(list(la) + list(lb)))
    if len(labs) > len(_LETTERS):
        raise ValueError("too many labels for einsum")
    m = {l: _LETTERS[i] for i, l in enumerate(labs)}
    spec = "".join(m[l] for l in la) + "," + "".join(m[l] for l in lb) + "->" + "".join(m[l] for l in lc)
    return np.einsum(spec, np.asarray(A, dtype=np.complex128), np.asarray(B, dtype=np.complex128))


def contract_pair_mm(A, la, B, lb, lc) -> np.ndarray:
    """contract_pair as one batched matrix product (library matmul)."""
    _check(la, lb, lc)
    A = np.asarray(A, dtype=np.complex128)
    B = np.asarray(B, dtype=np.complex128)
    la, lb, lc = list(la), list(lb), list(lc)
    # labels in one input only and not in C: summed out of that input first
    for T, ls, other in ((0, la, lb), (1, lb, la)):
        drop = [l for l in ls if l not in other and l not in lc]
        if drop:
            axes = tuple(ls.index(l) for l in drop)
            if T == 0:
                A = A.sum(axis=axes)
                la = [l for l in la if l not in drop]
            else:
                B = B.sum(axis=axes)
                lb = [l for l in lb if l not in drop]
    batch = [l for l in la if l in lb and l in lc]
    summed = [l for l in la if l in lb and l not in lc]
    fa = [l for l in la if l not in lb]
    fb = [l for l in lb if l not in la]
    ext = {l: A.shape[i] for i, l in enumerate(la)}
    ext.update({l: B.shape[i] for i, l in enumerate(lb)})
    size = lambda ls: int(np.prod([ext[l] for l in ls], dtype=np.int64))
    At = np.transpose(A, [la.index(l) for l in batch + fa + summed]).reshape(size(batch), size(fa), size(summed))
    Bt = np.transpose(B, [lb.index(l) for l in batch + summed + fb]).reshape(size(batch), size(summed), size(fb))
    C = np.matmul(At, Bt).reshape([ext[l] for l in batch + fa + fb])
    order = batch + fa + fb
    return np.transpose(C, [order.index(l) for l in lc]) if lc else C.reshape(())


def contract_entries(A, la, B, lb, lc, index_list) -> np.ndarray:
    """Selected entries C[idx] of contract_pair(A, la, B, lb, lc), each
    computed on its own: fix the output labels, then sum the product over
    every remaining label (einsum of the two fixed sub-tensors)."""
    _check(la, lb, lc)
    out = np.empty(len(index_list), dtype=np.complex128)
    for t, idx in enumerate(index_list):
        env = dict(zip(lc, idx))
        sa = tuple(env[l] if l in env else slice(None) for l in la)
        sb = tuple(env[l] if l in env else slice(None) for l in lb)
        ra = [l for l in la if l not in env]
        rb = [l for l in lb if l not in env]
        out[t] = complex(contract_pair(np.asarray(A)[sa], ra, np.asarray(B)[sb], rb, []))
    return out


def result_labels(la, lb, others: List[Sequence[int]], keep: Sequence[int]) -> List[int]:
    """Labels the product of A and B keeps: those still used by another live
    tensor or listed in ``keep`` (open output legs); order = A's then B's."""
    still = set(keep)
    for ls in others:
        still.update(ls)
    out = []
    for l in list(la) + list(lb):
        if l in still and l not in out:
            out.append(l)
    return out


def contract_path(tensors: List[np.ndarray], labels: List[List[int]], path,
                  open_labels: Sequence[int], pair=None) -> np.ndarray:
    """Contract a network along an SSA path (pairs of tensor ids; the result of
    step t gets id len(tensors) + t).  Returns the tensor over
    ``open_labels`` in that order (a scalar array if there are none).

    Components left unconnected at the end are multiplied as outer products in
    id order.  ``pair``: the pairwise contraction (default contract_pair).
    """
    pair = pair or contract_pair
    live = {i: (np.asarray(T, dtype=np.complex128), list(ls)) for i, (T, ls) in enumerate(zip(tensors, labels))}
    nid = len(tensors)
    for (i, j) in path:
        A, la = live.pop(i)
        B, lb = live.pop(j)
        lc = result_labels(la, lb, [ls for _, ls in live.values()], open_labels)
        live[nid] = (pair(A, la, B, lb, lc), lc)
        nid += 1
    while len(live) > 1:
        ids = sorted(live)
        A, la = live.pop(ids[0])
        B, lb = live.pop(ids[1])
        lc = result_labels(la, lb, [ls for _, ls in live.values()], open_labels)
        live[nid] = (pair(A, la, B, lb, lc), lc)
        nid += 1
    (T, ls), = live.values()
    # sum out anything not open (cannot happen for circuit networks)
    extra = [l for l in ls if l not in open_labels]
    if extra:
        T = contract_pair(T, ls, np.ones(()), [], [l for l in ls if l in open_labels])
        ls = [l for l in ls if l in open_labels]
    order = [ls.index(l) for l in open_labels]
    return np.transpose(T, order) if order else T
