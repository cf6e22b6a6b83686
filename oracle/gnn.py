"""O7: the contraction-order scorer, written out in FP64 numpy.

Nodes of the scored graph are the candidate pairwise contractions of a
path-search state (the line graph of the tensor network: two candidates are
neighbours when they share a tensor).  The paper motivates learning here only
indirectly: its Sec. 4.3 remarks that a better contraction path took longer
to find but ran faster.  Everything below is this project's own reading.

Features of candidate (A, B) -> C, with a = log2|A|, b = log2|B|,
c = log2|C|, u = log2|A u B|, d = |C| - |A| - |B| and
sigma = sign(d) log2(1 + |d|) (the greedy score on a log scale):
    x0 a/32, x1 b/32, x2 c/32, x3 u/32, x4 (a + b - u)/8,
    x5 (c - max(a, b))/8, x6 sigma/32, x7 (sigma - min sigma)/8,
    x8 1 if sigma == min sigma else 0, x9 live tensors / leaves,
    x10 log2(1 + candidates)/16, x11 (u - min u)/8, x12 deg(A)/16,
    x13 deg(B)/16, x14 1 if A and B share no label else 0, x15 1.
deg(T) = number of candidates containing T.

Network (H hidden units, L message-passing layers):
    h0 = relu(X W0 + b0)
    h_l = relu(h_{l-1} Ws_l + (N h_{l-1}) Wn_l + b_l),  N = row-mean over
          line-graph neighbours (a node without neighbours aggregates 0)
    s = relu(h_L Wh + bh) wo + bo
Loss of one state with teacher choice y: logsumexp(s) - s_y.

Parity pins (tests): central finite differences of the loss agree with the
hand-written backward; features agree with the native featurizer; the
forward on a hand-sized example is checked against a direct evaluation.
"""

from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np

from .paths import _State, size_of

N_FEAT = 16


# ------------------------------------------------------------------ features

def candidates_and_features(st: _State, ext, n_leaves: int):
    """Candidates of a state (the greedy's order), their features and the
    line-graph neighbour lists (ascending)."""
    cands = st.candidates()
    deg: Dict[int, int] = {}
    for i, j in cands:
        deg[i] = deg.get(i, 0) + 1
        deg[j] = deg.get(j, 0) + 1
    rows = []
    for i, j in cands:
        A, B = st.sets[i], st.sets[j]
        C = st.result(i, j)
        sa, sb, sc = size_of(A, ext), size_of(B, ext), size_of(C, ext)
        su = size_of(A | B, ext)
        d = sc - sa - sb
        sig = math.copysign(math.log2(1.0 + abs(d)), d)
        rows.append((math.log2(sa), math.log2(sb), math.log2(sc), math.log2(su), sig, i, j, len(A & B)))
    smin = min(r[4] for r in rows)
    umin = min(r[3] for r in rows)
    nc = len(cands)
    X = np.zeros((nc, N_FEAT))
    for k, (a, b, c, u, sig, i, j, shared) in enumerate(rows):
        X[k] = [a / 32, b / 32, c / 32, u / 32, (a + b - u) / 8, (c - max(a, b)) / 8, sig / 32,
                (sig - smin) / 8, 1.0 if sig == smin else 0.0, len(st.sets) / n_leaves,
                math.log2(1 + nc) / 16, (u - umin) / 8, deg[i] / 16, deg[j] / 16,
                1.0 if shared == 0 else 0.0, 1.0]
    by_t: Dict[int, List[int]] = {}
    for k, (i, j) in enumerate(cands):
        by_t.setdefault(i, []).append(k)
        by_t.setdefault(j, []).append(k)
    nbrs = []
    for k, (i, j) in enumerate(cands):
        s = set(by_t[i]) | set(by_t[j])
        s.discard(k)
        nbrs.append(sorted(s))
    return cands, X, nbrs


def teacher_samples(leaves, ext, open_set, path) -> List[Tuple[np.ndarray, list, int]]:
    """(features, neighbours, label) for every step of a teacher path."""
    st = _State(leaves, open_set, ())
    out = []
    for (i, j) in path:
        cands, X, nbrs = candidates_and_features(st, ext, len(leaves))
        out.append((X, nbrs, cands.index((i, j))))
        st.merge(i, j)
    return out


# ------------------------------------------------------------------ network

def param_shapes(H: int, L: int):
    shapes = [("W0", (N_FEAT, H)), ("b0", (H,))]
    for l in range(L):
        shapes += [(f"Ws{l}", (H, H)), (f"Wn{l}", (H, H)), (f"b{l + 1}", (H,))]
    shapes += [("Wh", (H, H)), ("bh", (H,)), ("wo", (H,)), ("bo", (1,))]
    return shapes


def unflatten(theta: np.ndarray, H: int, L: int) -> Dict[str, np.ndarray]:
    P, o = {}, 0
    for name, shp in param_shapes(H, L):
        n = int(np.prod(shp))
        P[name] = theta[o:o + n].reshape(shp)
        o += n
    assert o == theta.size
    return P


def n_params(H: int, L: int) -> int:
    return sum(int(np.prod(s)) for _, s in param_shapes(H, L))


def _mean_agg(h, nbrs):
    out = np.zeros_like(h)
    for k, nb in enumerate(nbrs):
        if nb:
            out[k] = h[nb].sum(axis=0) / len(nb)
    return out


def _mean_agg_T(g, nbrs):
    """Adjoint of _mean_agg: node j receives g_k / deg_k from every k with j in N(k)."""
    out = np.zeros_like(g)
    for k, nb in enumerate(nbrs):
        if nb:
            out[nb] += g[k] / len(nb)
    return out


def forward(theta, H, L, X, nbrs):
    P = unflatten(np.asarray(theta, dtype=np.float64), H, L)
    cache = {"X": X}
    z = X @ P["W0"] + P["b0"]
    h = np.maximum(z, 0)
    cache["z0"], cache["h0"] = z, h
    for l in range(L):
        m = _mean_agg(h, nbrs)
        z = h @ P[f"Ws{l}"] + m @ P[f"Wn{l}"] + P[f"b{l + 1}"]
        cache[f"m{l}"] = m
        h = np.maximum(z, 0)
        cache[f"z{l + 1}"], cache[f"h{l + 1}"] = z, h
    zh = h @ P["Wh"] + P["bh"]
    hh = np.maximum(zh, 0)
    s = hh @ P["wo"] + P["bo"][0]
    cache["zh"], cache["hh"] = zh, hh
    return s, cache


def loss_and_grad(theta, H, L, X, nbrs, label):
    P = unflatten(np.asarray(theta, dtype=np.float64), H, L)
    s, c = forward(theta, H, L, X, nbrs)
    smax = s.max()
    e = np.exp(s - smax)
    lse = smax + math.log(e.sum())
    loss = lse - s[label]
    ds = e / e.sum()
    ds[label] -= 1.0
    G = {}
    G["wo"] = c["hh"].T @ ds
    G["bo"] = np.array([ds.sum()])
    dhh = np.outer(ds, P["wo"])
    dzh = dhh * (c["zh"] > 0)
    G["Wh"] = c[f"h{L}"].T @ dzh
    G["bh"] = dzh.sum(axis=0)
    dh = dzh @ P["Wh"].T
    for l in reversed(range(L)):
        dz = dh * (c[f"z{l + 1}"] > 0)
        hp = c[f"h{l}"]
        G[f"Ws{l}"] = hp.T @ dz
        G[f"Wn{l}"] = c[f"m{l}"].T @ dz
        G[f"b{l + 1}"] = dz.sum(axis=0)
        dh = dz @ P[f"Ws{l}"].T + _mean_agg_T(dz @ P[f"Wn{l}"].T, nbrs)
    dz0 = dh * (c["z0"] > 0)
    G["W0"] = c["X"].T @ dz0
    G["b0"] = dz0.sum(axis=0)
    grad = np.concatenate([G[name].reshape(-1) for name, _ in param_shapes(H, L)])
    return loss, grad


def learned_path(theta, H, L, leaves, ext, open_set=()):
    """Path built by always taking the highest-scoring candidate."""
    st = _State(leaves, open_set, ())
    path = []
    while len(st.sets) > 1:
        cands, X, nbrs = candidates_and_features(st, ext, len(leaves))
        s, _ = forward(theta, H, L, X, nbrs)
        k = int(np.argmax(s))
        path.append(cands[k])
        st.merge(*cands[k])
    return path
