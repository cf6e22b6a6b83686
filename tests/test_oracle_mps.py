"""Pins of the MPS oracle (O5): no truncation reproduces the state vector;
one truncated two-qubit update obeys Eckart-Young; the norm stays 1."""

import numpy as np
import pytest

from oracle import statevector as sv
from oracle.gates import gate_matrix
from oracle.mps import MPS, run_circuit
from workloads import chain_random_circuit


@pytest.mark.parametrize("n,cyc", [(6, 4), (10, 8), (12, 6)])
def test_untruncated_mps_equals_state_vector(n, cyc):
    _, ops = chain_random_circuit(n, cyc, 11 + n)
    m, disc = run_circuit(n, ops, chi_max=1 << (n // 2), cutoff=0.0)
    psi = sv.simulate(n, ops)
    assert np.abs(m.to_statevector() - psi).max() <= 1e-12
    assert disc <= 1e-20
    assert np.abs(m.expect_z() - sv.expect_z(psi)).max() <= 1e-12


def test_single_truncation_eckart_young():
    n, ops = chain_random_circuit(8, 6, 3)
    m, _ = run_circuit(n, ops, chi_max=64, cutoff=0.0)
    m.move_center(3)
    A, B = m.sites[3], m.sites[4]
    U = gate_matrix("fsim", (0.9, 0.4))
    theta = np.einsum("abst,lsm,mtr->labr", U.reshape(2, 2, 2, 2), A, B)
    l, r = A.shape[0], B.shape[2]
    s = np.linalg.svd(theta.reshape(2 * l, 2 * r), compute_uv=False)
    chi = 3
    before = m.to_statevector()
    disc = m.apply_gate2(3, U, chi_max=chi, cutoff=0.0)
    # discarded weight = sum of the dropped squared singular values
    assert abs(disc - np.sum(s[chi:] ** 2) / np.sum(s ** 2)) <= 1e-13
    # the kept state is the Eckart-Young projection, renormalised
    exact = sv.apply_gate(before, U, (3, 4))
    after = m.to_statevector()
    overlap = abs(np.vdot(after, exact)) ** 2
    assert abs(overlap - (1 - disc)) <= 1e-12
    assert abs(np.linalg.norm(after) - 1) <= 1e-12
    assert m.bond_dims()[3] == chi


@pytest.mark.parametrize("n,cyc", [(8, 5), (10, 6)])
def test_untruncated_bond_spectra_are_schmidt_coefficients(n, cyc):
    """Without truncation the recorded spectrum of every bond is the list of
    Schmidt coefficients of the final state across that cut (gates on other
    bonds act unitarily on one side and leave them unchanged), found here by
    an SVD of the state vector reshaped to 2^(b+1) x 2^(n-b-1)."""
    _, ops = chain_random_circuit(n, cyc, 40 + n)
    m, _ = run_circuit(n, ops, chi_max=1 << (n // 2), cutoff=1e-13)
    psi = sv.simulate(n, ops)
    for b in range(n - 1):
        s = np.linalg.svd(psi.reshape(2 ** (b + 1), -1), compute_uv=False)
        s = s[s > 1e-13 * s[0]]
        assert m.spectra[b].shape == s.shape, (b, m.spectra[b].shape, s.shape)
        assert np.abs(m.spectra[b] - s).max() <= 1e-12
    assert all(g == np.inf or g > 0 for g in m.cut_gaps)
