"""Circuit -> tensor network (Sec. 3.1, Fig. 1), oracle side.

Qubits are rank-1 tensors, single-qubit gates rank-2 and two-qubit gates
rank-4; the circuit fixes which legs are joined.  The network is simplified
the way the paper describes small gate tensors being absorbed into larger
ones (Sec. 3.1.1):

* the |0> input of a wire and every single-qubit gate before the wire's first
  two-qubit gate are folded into that two-qubit gate's input side (the input
  leg disappears);
* single-qubit gates between two two-qubit gates on a wire are folded into
  the input side of the later one;
* single-qubit gates after the wire's last two-qubit gate are folded into that
  gate's output leg;
* a wire with no two-qubit gate becomes one rank-1 tensor (gates applied to
  |0>) holding the wire's output leg.

Tensor order: two-qubit gates in circuit order, then lone wires in qubit
order.  Index labels are integers handed out in creation order: each
two-qubit gate on (a, b) creates the label of a's output leg, then b's; lone
wires get theirs after all gates, in qubit order.  A tensor's axes are
[out_a, out_b, in_a, in_b] with absent input legs dropped.

Parity pin: contracting the whole network reproduces the state vector (O1)
on small circuits, for any pairwise order (tests).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List

import numpy as np

from .gates import I2, gate_matrix


@dataclass
class Network:
    n_qubits: int
    tensors: List[np.ndarray] = field(default_factory=list)
    labels: List[List[int]] = field(default_factory=list)
    out_label: List[int] = field(default_factory=list)   # per qubit
    n_labels: int = 0

    def extents(self) -> Dict[int, int]:
        ext = {}
        for t, ls in zip(self.tensors, self.labels):
            for ax, l in enumerate(ls):
                ext[l] = t.shape[ax]
        return ext


def build_network(n: int, ops) -> Network:
    pend = [I2.copy() for _ in range(n)]     # single-qubit product waiting on each wire
    wire = [None] * n                         # current label on each wire (None: still |0>)
    owner = [None] * n                        # (tensor id, axis) holding that label
    net = Network(n_qubits=n)
    nxt = 0
    for op in ops:
        if len(op.qubits) == 1:
            q = op.qubits[0]
            pend[q] = gate_matrix(op.name, op.params) @ pend[q]
            continue
        a, b = op.qubits
        U = gate_matrix(op.name, op.params) @ np.kron(pend[a], pend[b])
        T = U.reshape(2, 2, 2, 2)               # [out_a, out_b, in_a, in_b]
        pend[a] = I2.copy()
        pend[b] = I2.copy()
        labs = [nxt, nxt + 1]
        nxt += 2
        # fix fresh input legs to |0>: drop in_b first so in_a's axis stays put
        keep_in = []
        if wire[b] is None:
            T = T[:, :, :, 0]
        else:
            keep_in.append(("b", wire[b]))
        if wire[a] is None:
            T = T[:, :, 0]
        else:
            keep_in.insert(0, ("a", wire[a]))
        labs += [l for _, l in keep_in]
        tid = len(net.tensors)
        net.tensors.append(np.ascontiguousarray(T))
        net.labels.append(labs)
        wire[a], wire[b] = labs[0], labs[1]
        owner[a], owner[b] = (tid, 0), (tid, 1)
    # trailing single-qubit gates: fold into the output leg of the last owner
    for q in range(n):
        if owner[q] is not None and not np.array_equal(pend[q], I2):
            tid, ax = owner[q]
            T = net.tensors[tid]
            T = np.moveaxis(np.tensordot(pend[q], T, axes=([1], [ax])), 0, ax)
            net.tensors[tid] = np.ascontiguousarray(T)
    # lone wires
    for q in range(n):
        if owner[q] is None:
            v = pend[q] @ np.array([1, 0], dtype=np.complex128)
            net.tensors.append(v)
            net.labels.append([nxt])
            wire[q] = nxt
            nxt += 1
    net.out_label = [int(w) for w in wire]
    net.n_labels = nxt
    return net


def fix_outputs(net: Network, bits) -> tuple:
    """Project output legs with bit value 0/1; keep -1 legs open.

    Returns (tensors, labels, open_labels) where fixed legs are removed from
    the tensors by indexing (a projection onto a basis state, Fig. 3), and
    open_labels lists the open output labels by ascending qubit.
    """
    fixed = {}
    open_labels = []
    for q, bval in enumerate(bits):
        if int(bval) < 0:
            open_labels.append(net.out_label[q])
        else:
            fixed[net.out_label[q]] = int(bval)
    tensors, labels = fix_labels(net.tensors, net.labels, fixed)
    return tensors, labels, open_labels


def fix_labels(tensors, labels, fixed: Dict[int, int]):
    """Index every axis whose label is in ``fixed`` at the given value."""
    out_t, out_l = [], []
    for T, ls in zip(tensors, labels):
        idx = tuple(fixed[l] if l in fixed else slice(None) for l in ls)
        out_t.append(np.asarray(T[idx]))
        out_l.append([l for l in ls if l not in fixed])
    return out_t, out_l
