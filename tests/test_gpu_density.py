"""Exact noisy expectation values from the density-matrix network on the GPU
(Sec. 3.3, Eq. 3) against the density-matrix oracle (O3), and the exact
check of the Kraus trajectories (Sec. 3.3) it makes possible.

Values lie in [-1, 1]; the bar is an absolute error of 1e-5 (complex64
contraction, FP64 accumulation)."""

import math

import numpy as np
import pytest

from oracle import observables as ob
from workloads import (grid_random_circuit, noisy_ops, trajectory_uniforms, count_channel_events,
                       chain_random_circuit)

pytestmark = pytest.mark.gpu
TOL = 1e-5


def dm_value(n, ops, codes, precision="fp32"):
    import paper_2104_10523_amd as tn
    net, kept = tn.tn_build_density_network(n, ops, codes)
    path = tn.tn_find_path(net, "random_greedy", trials=16, seed=1)
    out, rep = tn.tn_amplitudes(net, path, np.zeros((1, 0), np.int8), precision=precision)
    assert rep.nonfinite == 0
    return complex(out.cpu().numpy()[0, 0]), kept


def random_pauli(n, weight, rng):
    codes = [0] * n
    for q in rng.choice(n, size=weight, replace=False):
        codes[int(q)] = int(rng.integers(1, 4))
    return codes


@pytest.mark.parametrize("precision", ["fp32", "f16x3"])
@pytest.mark.parametrize("seed", range(3))
def test_density_network_matches_oracle(gpu, workspace, precision, seed):
    rng = np.random.default_rng(20 + seed)
    n, ops = grid_random_circuit(3, 3, 3 + seed, 950 + seed)
    ops = noisy_ops(ops, 0.01, 0.03, 0.05)
    codes = random_pauli(n, 1 + seed, rng)
    got, kept = dm_value(n, ops, codes, precision)
    ref = ob.dm_expectation(n, ops, codes)
    assert abs(got - ref) <= TOL, (got, ref)


def test_density_network_noiseless_and_trace(gpu, workspace):
    rng = np.random.default_rng(3)
    n, ops = grid_random_circuit(3, 4, 5, 31)
    codes = random_pauli(n, 2, rng)
    got, _ = dm_value(n, ops, codes)
    assert abs(got - ob.expectation(n, ops, codes)) <= TOL
    nops = noisy_ops(ops, 0.01, 0.02, 0.03)
    tr, kept = dm_value(n, nops, [0] * n)
    assert kept == 0 and abs(tr - 1) <= TOL


def test_density_network_chain_light_cone(gpu, workspace):
    """16-qubit noisy chain (a 2^32-entry density matrix): one <Z> keeps its
    light cone only and matches the oracle run on that cone's qubits."""
    n, ops = chain_random_circuit(16, 3, 12)
    ops = noisy_ops(ops, 0.01, 0.02, 0.04)
    codes = [0] * n
    codes[0] = 3
    got, kept = dm_value(n, ops, codes)
    cone = ob.light_cone(n, ops, codes)
    qs = sorted({q for k in cone for q in ops[k].qubits} | {0})
    remap = {q: i for i, q in enumerate(qs)}
    sub = [type(ops[k])(ops[k].name, tuple(remap[q] for q in ops[k].qubits), ops[k].params) for k in cone]
    assert len(qs) <= 10
    ref = ob.dm_expectation(len(qs), sub, [3] + [0] * (len(qs) - 1))
    assert kept == len(cone)
    assert abs(got - ref) <= TOL, (got, ref)


def test_trajectories_against_exact_density_network(gpu, workspace):
    """The stochastic trajectories (a10) against the exact density-matrix
    network: every <Z_q> mean within 4 standard errors."""
    import paper_2104_10523_amd as tn
    n, ops = grid_random_circuit(2, 3, 5, 77)
    ops = noisy_ops(ops, 0.02, 0.05, 0.1)
    T = 3000
    U = trajectory_uniforms(T, count_channel_events(ops), 21)
    z, _ = tn.tn_run_trajectories([(n, ops)], T, U)
    for q in range(n):
        codes = [0] * n
        codes[q] = 3
        exact, _ = dm_value(n, ops, codes)
        se = z[:, q].std() / math.sqrt(T)
        assert abs(z[:, q].mean() - exact.real) <= 4 * se + 1e-9, (q, z[:, q].mean(), exact)
