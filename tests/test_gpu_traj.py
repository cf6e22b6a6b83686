"""tn_run_trajectories on the GPU against the trajectory oracle (O4) driven
by the same uniforms, and against the density-matrix oracle (O3)."""

import math

import numpy as np
import pytest

from oracle import noise
from workloads import (Op, grid_random_circuit, noisy_ops, trajectory_uniforms, count_channel_events,
                       hh_circuit)

pytestmark = pytest.mark.gpu


def run_gpu(circuits, tpc, U):
    import paper_2104_10523_amd as tn
    return tn.tn_run_trajectories(circuits, tpc, U)


def test_trajectories_match_oracle_per_trajectory(gpu):
    circuits = []
    for c in range(3):
        n, ops = grid_random_circuit(2, 3, 3 + 2 * c, 30 + c)
        circuits.append((n, noisy_ops(ops, 0.05, 0.1, 0.08)))
    tpc = 8
    ev = max(count_channel_events(o) for _, o in circuits)
    U = trajectory_uniforms(len(circuits) * tpc, ev, 9)
    z, rep = run_gpu(circuits, tpc, U)
    zo = noise.trajectories_expect_z(circuits, tpc, U)
    assert z.shape == zo.shape
    assert np.abs(z - zo).max() <= 2e-5
    assert rep.seconds > 0


def test_trajectory_mean_matches_density_matrix(gpu):
    n, ops = grid_random_circuit(2, 3, 4, 21)
    ops = noisy_ops(ops, 0.05, 0.1, 0.08)
    zdm = noise.dm_expect_z(noise.dm_simulate(n, ops), n)
    T = 2000
    U = trajectory_uniforms(T, count_channel_events(ops), 6)
    z, _ = run_gpu([(n, ops)], T, U)
    se = z.std(axis=0) / math.sqrt(T)
    assert np.all(np.abs(z.mean(axis=0) - zdm) <= 4 * se + 1e-9)


def test_noisy_hh_on_gpu_matches_closed_form(gpu):
    """Depolarising H-H chain on qubit 0 of a 4-qubit register: every
    trajectory is a Pauli sequence, the mean over many trajectories
    approaches (1 - 4p/3)^(2n)."""
    p, cyc = 0.02, 10
    _, ops = hh_circuit(cyc)
    ops = noisy_ops(ops, p, 0.0, 0.0)
    T = 4000
    U = trajectory_uniforms(T, count_channel_events(ops), 8)
    z, _ = run_gpu([(4, ops)], T, U)
    want = (1 - 4 * p / 3) ** (2 * cyc)
    se = z[:, 0].std() / math.sqrt(T)
    assert abs(z[:, 0].mean() - want) <= 4 * se
    assert np.all(np.abs(z[:, 1:] - 1) <= 1e-6)


def test_uneven_depth_batch(gpu):
    circuits = []
    for c, depth in enumerate((2, 9, 5, 1)):
        n, ops = grid_random_circuit(2, 2, depth, 50 + c)
        circuits.append((n, noisy_ops(ops, 1e-2, 5e-2, 5e-2)))
    tpc = 4
    ev = max(count_channel_events(o) for _, o in circuits)
    U = trajectory_uniforms(len(circuits) * tpc, ev, 3)
    z, _ = run_gpu(circuits, tpc, U)
    zo = noise.trajectories_expect_z(circuits, tpc, U)
    assert np.abs(z - zo).max() <= 2e-5


@pytest.mark.parametrize("rows,cols,depth", [(3, 4, 6), (4, 4, 5)])
def test_trajectories_wide_registers(gpu, rows, cols, depth):
    """12 and 16 qubits: many 16-amplitude groups per block and several
    blocks per trajectory, damping on every gate."""
    circuits = []
    for c in range(2):
        n, ops = grid_random_circuit(rows, cols, depth + c, 70 + c)
        circuits.append((n, noisy_ops(ops, 0.02, 0.05, 0.1)))
    tpc = 3
    ev = max(count_channel_events(o) for _, o in circuits)
    U = trajectory_uniforms(len(circuits) * tpc, ev, 11)
    z, _ = run_gpu(circuits, tpc, U)
    zo = noise.trajectories_expect_z(circuits, tpc, U)
    assert np.abs(z - zo).max() <= 5e-5


def _c41_ensemble():
    """The trajectory row's ensemble: 32 circuits on a 4x5 grid (CZ) of
    depth 10 + round(20 c / 31), depolarising 1e-3 / 1e-2 and damping 5e-3
    after every gate, 32 trajectories each, uniforms from seed 4."""
    circuits = []
    for c in range(32):
        n, ops = grid_random_circuit(4, 5, 10 + round(20 * c / 31), 40 + c)
        circuits.append((n, noisy_ops(ops, 1e-3, 1e-2, 5e-3)))
    ev = max(count_channel_events(o) for _, o in circuits)
    return circuits, 32, trajectory_uniforms(32 * 32, ev, 4)


@pytest.fixture(scope="module")
def c41_run(gpu):
    circuits, tpc, U = _c41_ensemble()
    z, rep = run_gpu(circuits, tpc, U)
    assert z.shape == (1024, 20)
    return circuits, tpc, U, z


@pytest.mark.timeout(400)
@pytest.mark.parametrize("circ", [0, 31], ids=["depth10", "depth30"])
def test_c41_full_size_trajectories_match_oracle(c41_run, circ):
    """Full-size ensemble (1024 trajectories of 20 qubits in one call): the
    first 4 trajectories of the depth-10 and of the depth-30 circuit against
    the trajectory oracle on the same uniform rows.  A trajectory whose
    uniforms all sit more than 1e-8 from a branch boundary must take the
    oracle's branches (complex64 state, FP64 branch probabilities); its <Z_q>
    then agrees to 1e-5 (the state carries ~1e-7 of complex64 rounding per
    pass over ~10^3 passes, renormalised in FP64)."""
    circuits, tpc, U, z = c41_run
    n, ops = circuits[circ]
    compared = 0
    for j in range(4):
        row = circ * tpc + j
        margins = []
        psi, _ = noise.trajectory(n, ops, U[row], margins)
        zo = sv_expect_z(psi)
        err = float(np.abs(z[row] - zo).max())
        print(f"circuit {circ} trajectory {j}: min margin {min(margins):.2e} max |dZ| {err:.2e}", flush=True)
        if min(margins) > 1e-8:
            assert err <= 1e-5, (circ, j, err)
            compared += 1
    assert compared >= 3


def sv_expect_z(psi):
    from oracle.statevector import expect_z
    return expect_z(psi)
