"""Pins of the noise oracles (O3 density matrix, O4 trajectories)."""

import json
import math
from pathlib import Path

import numpy as np
import pytest

from oracle import noise
from oracle import statevector as sv
from workloads import Op, hh_circuit, noisy_ops, grid_random_circuit, trajectory_uniforms, count_channel_events

GOLDEN = Path(__file__).parent / "golden"


def _hh_z(cycles, p):
    n, ops = hh_circuit(cycles)
    rho = noise.dm_simulate(n, noisy_ops(ops, p, 0.0, 0.0))
    return noise.dm_expect_z(rho, n)[0]


@pytest.mark.parametrize("p", [1e-3, 0.05])
def test_depolarising_hh_closed_form(p):
    for cycles in (1, 3, 10):
        assert abs(_hh_z(cycles, p) - (1 - 4 * p / 3) ** (2 * cycles)) <= 1e-13


def test_paper_noisy_hh_curves():
    """Sec. 4.2, Fig. h_gate_chart: each printed curve is matched, to its
    printed 6 digits, by a depolarising channel after every H with one
    probability p (fitted on the first and last points)."""
    g = json.loads((GOLDEN / "hh_noise.json").read_text())
    for q in ("Q0", "Q1"):
        pts = [(x, y) for x, y in g[q] if x > 0]
        (x0, y0), (x1, y1) = pts[0], pts[-1]
        f = math.exp((math.log(y1) - math.log(y0)) / (x1 - x0))   # per-cycle factor
        p = 3 * (1 - math.sqrt(f)) / 4
        worst = max(abs(_hh_z(x, p) - y) for x, y in pts)
        assert worst <= 1.0e-6, (q, p, worst)


def test_amplitude_damping_closed_form():
    gamma = 0.03
    for m in (1, 5, 20):
        ops = [Op("x", (0,))] + [Op("amp_damp", (0,), (gamma,))] * m
        rho = noise.dm_simulate(1, ops)
        assert abs(noise.dm_expect_z(rho, 1)[0] - (1 - 2 * (1 - gamma) ** m)) <= 1e-14


def test_trajectory_branch_rule():
    # depolarising with p = 1: the branch is X, Y or Z by the uniform's third
    ops = [Op("depol1", (0,), (1.0,))]
    for u, want in ((0.1, 1), (0.5, 2), (0.9, 3)):
        _, br = noise.trajectory(1, ops, [u])
        assert br == [want]
    # damping of |1> with g = 0.25: branch 1 (decay) iff u >= 0.75
    ops = [Op("x", (0,)), Op("amp_damp", (0,), (0.25,))]
    for u, want in ((0.7, 0), (0.8, 1)):
        psi, br = noise.trajectory(1, ops, [u])
        assert br == [want]
        assert abs(np.sum(np.abs(psi) ** 2) - 1) <= 1e-15


def test_trajectory_mean_matches_density_matrix():
    n, ops = grid_random_circuit(2, 3, 4, 21)
    ops = noisy_ops(ops, 0.05, 0.1, 0.08)
    rho = noise.dm_simulate(n, ops)
    zdm = noise.dm_expect_z(rho, n)
    T = 400
    U = trajectory_uniforms(T, count_channel_events(ops), 5)
    z = noise.trajectories_expect_z([(n, ops)], T, U)
    se = z.std(axis=0) / math.sqrt(T)
    assert np.all(np.abs(z.mean(axis=0) - zdm) <= 4 * se + 1e-12)
