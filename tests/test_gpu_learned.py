"""The learned contraction-order scorer on the GPU: gradients of the
hand-written kernels against the FP64 oracle (O7), training by imitation of
randomised-greedy teacher paths, and what the learned path (with greedy as
fallback) gains over greedy on held-out circuits."""

import math

import numpy as np
import pytest

from oracle import gnn
from oracle.network import build_network
from oracle.paths import random_greedy_path
from workloads import grid_random_circuit, scorer_init

pytestmark = pytest.mark.gpu


def _states(seed, rows=3, cols=4, cyc=8):
    n, ops = grid_random_circuit(rows, cols, cyc, seed)
    net = build_network(n, ops)
    outs = set(net.out_label)
    leaves = [[l for l in ls if l not in outs] for ls in net.labels]
    ext = net.extents()
    path = random_greedy_path(leaves, ext, seed=1, trials=4)
    return gnn.teacher_samples(leaves, ext, set(), path)


@pytest.mark.parametrize("H,L", [(16, 2), (128, 4)])
def test_gradients_match_oracle(gpu, H, L):
    import paper_2104_10523_amd as tn
    m = tn.Model(H, L)
    theta = scorer_init(gnn.param_shapes(H, L), 7)
    theta[theta == 0] = 0.01            # non-zero biases exercise every term
    m.set_params(theta)
    theta32 = m.get_params()            # what the GPU actually holds (FP32)
    for k in (3, 11, 20):
        X, nbrs, y = _states(5)[k]
        loss, g, s = m.loss_grad(X, nbrs, y)
        lo, go = gnn.loss_and_grad(theta32, H, L, X, nbrs, y)
        so, _ = gnn.forward(theta32, H, L, X, nbrs)
        assert abs(loss - lo) <= 1e-4 * max(1, abs(lo))
        assert np.abs(s - so).max() <= 1e-4 * max(1, np.abs(so).max())
        assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)


def _ring_state(nc, seed):
    """A synthetic scorer input with nc candidates: random features and a
    symmetric neighbour relation (ring of radius 2 plus random chords)."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((nc, 16))
    nb = [set() for _ in range(nc)]
    for i in range(nc):
        for d in (1, 2):
            nb[i].add((i + d) % nc)
            nb[(i + d) % nc].add(i)
    for i, j in rng.integers(0, nc, size=(nc // 4, 2)):
        if i != j:
            nb[i].add(int(j))
            nb[j].add(int(i))
    return X, [sorted(x) for x in nb], int(rng.integers(nc))


@pytest.mark.parametrize("H,L,nc", [(16, 1, 6000), (128, 2, 9000)])
def test_split_k_gradients_match_oracle_and_repeat_exactly(gpu, H, L, nc):
    """Thousands of candidates: the weight-gradient products (K = nc) split
    K over blocks and sum the partials in a fixed order, so two calls give
    bit-identical gradients, and both match the FP64 oracle."""
    import paper_2104_10523_amd as tn
    m = tn.Model(H, L)
    theta = scorer_init(gnn.param_shapes(H, L), 5)
    theta[theta == 0] = 0.01
    m.set_params(theta)
    theta32 = m.get_params()
    X, nbrs, y = _ring_state(nc, H + L)
    loss, g, s = m.loss_grad(X, nbrs, y)
    loss2, g2, s2 = m.loss_grad(X, nbrs, y)
    assert loss == loss2 and np.array_equal(g, g2) and np.array_equal(s, s2)
    lo, go = gnn.loss_and_grad(theta32, H, L, X, nbrs, y)
    so, _ = gnn.forward(theta32, H, L, X, nbrs)
    assert abs(loss - lo) <= 1e-4 * max(1, abs(lo))
    assert np.abs(s - so).max() <= 1e-4 * max(1, np.abs(so).max())
    assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)


def test_training_repeats_exactly(gpu):
    """Same teachers, same seed: two trainings end at identical parameters."""
    import paper_2104_10523_amd as tn
    from workloads import path_search_circuit
    H, L = 128, 4
    theta0 = scorer_init(gnn.param_shapes(H, L), 11)
    out = []
    for _ in range(2):
        m = tn.Model(H, L)
        m.set_params(theta0)
        for i in range(12):
            n, ops = path_search_circuit(i)
            net = tn.tn_build_network(n, ops)
            teacher = tn.tn_find_path(net, "random_greedy", trials=8, seed=i, temperature=0.5)
            m.add_teacher(net, teacher.pairs, stride=max(1, len(teacher.pairs) // 16))
        m.train(epochs=2, batch=64, lr=1e-3, seed=3)
        out.append(m.get_params())
    assert np.array_equal(out[0], out[1])


def _corpus_paths(model, ids, rescore_every=1):
    import paper_2104_10523_amd as tn
    from workloads import path_search_circuit
    out = []
    for i in ids:
        n, ops = path_search_circuit(i)
        net = tn.tn_build_network(n, ops)
        g = tn.tn_find_path(net, "greedy")
        lp = tn.tn_find_path_learned(net, model, rescore_every=rescore_every)
        if lp.cost.algo_used == 2:
            # a complete path: re-evaluated from its own pairs, same cost
            again = tn.tn_path_from_pairs(net, lp.pairs)
            assert again.cost.flops_per_slice == lp.cost.flops_per_slice
            assert len(lp.pairs) == net.info().n_tensors - 1
        out.append((g.cost.flops_per_slice, lp.cost.flops_per_slice, lp.cost.algo_used == 2))
    return np.array(out)


@pytest.mark.timeout(600)
def test_training_and_learned_path_gain(gpu):
    """Imitation of the 32-trial randomised-greedy teacher on 400 corpus
    circuits (30-60 qubits, 8-16 CZ cycles, 16 states each), then 40
    held-out circuits: the learned path must be the one kept (it beats the
    greedy fallback) on at least half of them, with a geometric-mean flop
    ratio to greedy below 1/4, and the trained scorer must do strictly better
    than the same network at its initial parameters under the same fallback
    (which on its own only guarantees the greedy cost)."""
    import paper_2104_10523_amd as tn
    from workloads import path_search_circuit
    H, L = 128, 4
    theta0 = scorer_init(gnn.param_shapes(H, L), 11)
    m = tn.Model(H, L)
    m.set_params(theta0)
    m0 = tn.Model(H, L)
    m0.set_params(theta0)
    for i in range(400):
        n, ops = path_search_circuit(i)
        net = tn.tn_build_network(n, ops)
        teacher = tn.tn_find_path(net, "random_greedy", trials=32, seed=i, temperature=0.5)
        m.add_teacher(net, teacher.pairs, stride=max(1, len(teacher.pairs) // 16))
    first, last = m.train(epochs=4, batch=64, lr=1e-3, seed=3)
    print(f"training loss {first:.3f} -> {last:.3f}", flush=True)
    assert last < first
    held = range(5000, 5040)
    tr = _corpus_paths(m, held)
    un = _corpus_paths(m0, held)
    assert np.all(tr[:, 1] <= tr[:, 0]) and np.all(un[:, 1] <= un[:, 0])     # greedy is the fallback
    chosen = float(np.mean(tr[:, 2]))
    ratio = float(2 ** np.mean(np.log2(tr[:, 1] / tr[:, 0])))
    ratio0 = float(2 ** np.mean(np.log2(un[:, 1] / un[:, 0])))
    print(f"held-out: learned path kept on {chosen:.0%} of circuits, geometric-mean flops / greedy "
          f"{ratio:.3g} (untrained: kept {np.mean(un[:, 2]):.0%}, {ratio0:.3g})", flush=True)
    assert chosen >= 0.5
    assert ratio < 0.25
    assert ratio < ratio0
    # re-scoring after every 8 merges (the best 8 disjoint pairs per scoring)
    r8 = _corpus_paths(m, held, rescore_every=8)
    assert np.all(r8[:, 1] <= r8[:, 0])
    ratio8 = float(2 ** np.mean(np.log2(r8[:, 1] / r8[:, 0])))
    print(f"rescore_every=8: kept {np.mean(r8[:, 2]):.0%}, geometric-mean flops / greedy {ratio8:.3g}",
          flush=True)
    assert ratio8 < ratio0
