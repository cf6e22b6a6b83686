"""Pins of the slice-sampling oracle (Sec. 4.4, Table 1)."""

import math

import numpy as np

from oracle.sampling import cumulative, sample_indices


def test_point_mass():
    psi = np.zeros(37, complex)
    psi[11] = 0.3 - 0.4j
    u = np.random.default_rng(0).random(100)
    assert np.all(sample_indices(psi, u) == 11)


def test_two_outcomes_boundary():
    a = 0.3
    psi = np.array([math.sqrt(a), 1j * math.sqrt(1 - a)])
    u = np.array([0.0, 0.1, 0.2999, 0.3001, 0.9, 0.999999])
    got = sample_indices(psi, u)
    assert list(got) == [0, 0, 0, 1, 1, 1]


def test_uniform_slice_dyadic():
    k = 6
    psi = np.full(1 << k, 1 / 8.0, complex)
    u = (np.arange(1 << k) + 0.5) / (1 << k)
    assert np.all(sample_indices(psi, u) == np.arange(1 << k))


def test_frequencies_chi_square():
    rng = np.random.default_rng(3)
    psi = rng.standard_normal(16) + 1j * rng.standard_normal(16)
    p = np.abs(psi) ** 2 / np.sum(np.abs(psi) ** 2)
    N = 200000
    counts = np.bincount(sample_indices(psi, rng.random(N)), minlength=16)
    chi2 = np.sum((counts - N * p) ** 2 / (N * p))
    assert chi2 < 50          # 15 degrees of freedom: p-value ~ 1e-5 at 50
    assert abs(cumulative(psi)[-1] - np.sum(np.abs(psi) ** 2)) < 1e-12
