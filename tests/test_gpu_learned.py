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


def test_training_and_learned_path_gain(gpu):
    import paper_2104_10523_amd as tn
    H, L = 64, 3
    m = tn.Model(H, L)
    m.set_params(scorer_init(gnn.param_shapes(H, L), 11))
    shapes = [(4, 5), (4, 6), (5, 5)]
    for i in range(36):
        r, c = shapes[i % 3]
        n, ops = grid_random_circuit(r, c, 8 + i % 5, 1000 + i)
        net = tn.tn_build_network(n, ops)
        teacher = tn.tn_find_path(net, "random_greedy", trials=8, seed=i, temperature=0.5)
        m.add_teacher(net, teacher.pairs, stride=2)
    first, last = m.train(epochs=8, batch=16, lr=2e-3, seed=3)
    print(f"training loss {first:.3f} -> {last:.3f}")
    assert last < first
    gains, wins = [], 0
    for i in range(10):
        r, c = shapes[i % 3]
        n, ops = grid_random_circuit(r, c, 8 + i % 5, 5000 + i)
        net = tn.tn_build_network(n, ops)
        g = tn.tn_find_path(net, "greedy")
        lp = tn.tn_find_path_learned(net, m)
        assert lp.cost.flops_per_slice <= g.cost.flops_per_slice      # greedy is the fallback
        gain = math.log2(g.cost.flops_per_slice / lp.cost.flops_per_slice)
        gains.append(gain)
        wins += lp.cost.algo_used == 2
    print(f"held-out: learned path chosen on {wins}/10 circuits, mean log2 flop gain over greedy "
          f"{np.mean(gains):.2f}")
    assert np.mean(gains) >= 0.0
