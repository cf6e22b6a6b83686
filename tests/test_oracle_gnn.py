"""Pins of the scorer oracle (O7): finite differences vs the hand-written
backward, and the forward of a tiny network evaluated directly."""

import numpy as np
import pytest

from oracle import gnn
from oracle.network import build_network
from oracle.paths import greedy_path, random_greedy_path
from workloads import grid_random_circuit, scorer_init


def _sample(seed=3):
    n, ops = grid_random_circuit(3, 3, 5, seed)
    net = build_network(n, ops)
    outs = set(net.out_label)
    leaves = [[l for l in ls if l not in outs] for ls in net.labels]
    ext = net.extents()
    path = random_greedy_path(leaves, ext, seed=1, trials=4)
    return gnn.teacher_samples(leaves, ext, set(), path)


def test_finite_differences():
    H, L = 8, 2
    theta = scorer_init(gnn.param_shapes(H, L), 5) + 0.01
    X, nbrs, y = _sample()[6]
    loss, g = gnn.loss_and_grad(theta, H, L, X, nbrs, y)
    rng = np.random.default_rng(0)
    for idx in rng.choice(theta.size, size=40, replace=False):
        e = np.zeros_like(theta)
        h = 1e-6
        e[idx] = h
        lp, _ = gnn.loss_and_grad(theta + e, H, L, X, nbrs, y)
        lm, _ = gnn.loss_and_grad(theta - e, H, L, X, nbrs, y)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, g[idx])


def test_forward_direct_evaluation():
    # H = 1, L = 1: every quantity is a scalar per node; evaluate by hand
    H, L = 1, 1
    names = [n for n, _ in gnn.param_shapes(H, L)]
    theta = np.zeros(gnn.n_params(H, L))
    P = gnn.unflatten(theta, H, L)
    P["W0"][:, 0] = np.arange(gnn.N_FEAT) / 10.0
    P["b0"][0] = 0.1
    P["Ws0"][0, 0] = 0.5
    P["Wn0"][0, 0] = -0.25
    P["b1"][0] = 0.2
    P["Wh"][0, 0] = 2.0
    P["bh"][0] = -0.1
    P["wo"][0] = 3.0
    P["bo"][0] = 0.7
    theta = np.concatenate([P[n].reshape(-1) for n in names])
    X = np.random.default_rng(1).random((3, gnn.N_FEAT))
    nbrs = [[1, 2], [0], []]
    s, _ = gnn.forward(theta, H, L, X, nbrs)
    h0 = np.maximum(X @ (np.arange(gnn.N_FEAT) / 10.0) + 0.1, 0)
    m = np.array([(h0[1] + h0[2]) / 2, h0[0], 0.0])
    h1 = np.maximum(0.5 * h0 - 0.25 * m + 0.2, 0)
    want = np.maximum(2.0 * h1 - 0.1, 0) * 3.0 + 0.7
    assert np.allclose(s, want, atol=1e-14)


def test_teacher_labels_reproduce_teacher_path():
    n, ops = grid_random_circuit(3, 3, 5, 4)
    net = build_network(n, ops)
    outs = set(net.out_label)
    leaves = [[l for l in ls if l not in outs] for ls in net.labels]
    ext = net.extents()
    path = random_greedy_path(leaves, ext, seed=2, trials=4)
    from oracle.paths import _State
    st = _State(leaves, set(), ())
    for (X, nbrs, y), step in zip(gnn.teacher_samples(leaves, ext, set(), path), path):
        cands = st.candidates()
        assert cands[y] == step and X.shape == (len(cands), gnn.N_FEAT)
        st.merge(*step)
