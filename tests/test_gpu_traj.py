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
