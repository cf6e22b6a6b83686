"""Pins of the locally-purified MPS oracle (O8, Sec. 3.4) against the
density-matrix oracle (O3), the state vector (O1) and the rank bound of the
Kraus compression."""

import numpy as np
import pytest

from oracle import noise
from oracle import statevector as sv
from oracle.gates import kraus_ops
from oracle.pmps import PMPS, run_circuit
from workloads import chain_random_circuit, noisy_ops


def _rho_matrix(rho, n):
    return rho.reshape(2 ** n, 2 ** n)


@pytest.mark.parametrize("n,cyc,seed", [(4, 3, 1), (5, 3, 2), (6, 3, 3)])
def test_untruncated_pmps_equals_density_matrix(n, cyc, seed):
    """Depolarising (1- and 2-qubit) and amplitude damping after every gate,
    nothing truncated: rho equals the density-matrix oracle, Tr rho = 1 and
    <Z_i> equals Tr(rho Z_i)."""
    _, ops = chain_random_circuit(n, cyc, seed)
    ops = noisy_ops(ops, 0.05, 0.1, 0.08)
    # cutoff 1e-14 drops only singular values that are zero to rounding
    m, db, dk = run_circuit(n, ops, d_max=1 << n, k_max=1 << (2 * n), cutoff=1e-14)
    ref = noise.dm_simulate(n, ops)
    rho = m.to_density_matrix()
    assert np.abs(_rho_matrix(rho, n) - _rho_matrix(ref, n)).max() <= 1e-12
    assert abs(m.trace() - 1) <= 1e-12
    assert db <= 1e-14 and dk <= 1e-14     # (total - kept) / total: rounding only
    assert np.abs(m.expect_z() - noise.dm_expect_z(ref, n)).max() <= 1e-12


def test_noiseless_pmps_is_the_pure_state():
    n, ops = chain_random_circuit(6, 5, 4)
    m, _, _ = run_circuit(n, ops, d_max=64, k_max=8, cutoff=0.0)
    psi = sv.simulate(n, ops).reshape(-1)
    assert m.kraus_dims() == [1] * n
    assert np.abs(_rho_matrix(m.to_density_matrix(), n) - np.outer(psi, psi.conj())).max() <= 1e-12


def test_kraus_compression_is_exact_and_rank_bounded():
    """A channel multiplies K by its number of operators; compressing with
    every non-zero singular value kept changes nothing in rho, and the kept
    Kraus dimension never exceeds rows of the SVD, 2 D_l D_r."""
    n, ops = chain_random_circuit(5, 3, 6)
    m, _, _ = run_circuit(n, ops, d_max=32, k_max=1, cutoff=0.0)
    for step in range(6):
        site = step % n
        before = m.to_density_matrix()
        m.move_center(site)
        disc = m.apply_channel1(site, kraus_ops("depol1", (0.2,)), k_max=10 ** 6, cutoff=1e-14)
        after = m.to_density_matrix()
        # the channel itself, applied to the dense rho
        K = kraus_ops("depol1", (0.2,))
        want = sum(_apply1(before, A, site, n) for A in K)
        assert np.abs(after - want).max() <= 1e-12
        assert disc <= 1e-14
        l, _, k, r = m.sites[site].shape
        assert k <= 2 * l * r


def _apply1(rho, A, q, n):
    out = sv.apply_gate(rho, A, [q])
    return sv.apply_gate(out, A.conj(), [n + q])


def test_truncation_keeps_unit_trace_and_reports_weight():
    n, ops = chain_random_circuit(8, 6, 7)
    ops = noisy_ops(ops, 0.02, 0.05, 0.05)
    m, db, dk = run_circuit(n, ops, d_max=4, k_max=2)
    assert abs(m.trace() - 1) <= 1e-12
    assert max(m.bond_dims()) <= 4 and max(m.kraus_dims()) <= 2
    assert db > 0 and dk > 0


def test_asymmetric_two_qubit_gates_and_channels():
    """CX in both orientations (not symmetric under exchanging the qubits,
    unlike fSim and the depolarising pairs) with amplitude damping on one
    qubit of each pair: still equal to the density-matrix oracle."""
    from workloads import Op
    n = 4
    ops = [Op("h", (0,)), Op("sqrt_y", (2,)), Op("cx", (0, 1)), Op("amp_damp", (1,), (0.3,)),
           Op("sqrt_w", (1,)), Op("cx", (2, 1)), Op("amp_damp", (2,), (0.2,)), Op("cx", (2, 3)),
           Op("depol1", (3,), (0.1,)), Op("sqrt_x", (3,)), Op("cx", (3, 2)), Op("cx", (1, 2))]
    # (2, 1) and (3, 2) act on neighbours in descending order: the oracle
    # takes pairs (a, a+1), so express them with the gate's qubits swapped
    fixed = []
    for op in ops:
        if op.name == "cx" and op.qubits[0] > op.qubits[1]:
            a, b = op.qubits[1], op.qubits[0]
            fixed += [Op("h", (a,)), Op("h", (b,)), Op("cx", (a, b)), Op("h", (a,)), Op("h", (b,))]
        else:
            fixed.append(op)
    m, _, _ = run_circuit(n, fixed, d_max=64, k_max=256, cutoff=1e-14)
    ref = noise.dm_simulate(n, ops)
    assert np.abs(_rho_matrix(m.to_density_matrix(), n) - _rho_matrix(ref, n)).max() <= 1e-12


def test_channel_with_complex_kraus_operators():
    """A channel from a random 6 x 2 isometry (three complex Kraus operators,
    sum A^dagger A = 1) applied to one site equals sum_a A rho A^dagger on
    the dense density matrix."""
    rng = np.random.default_rng(9)
    V, _ = np.linalg.qr(rng.standard_normal((6, 2)) + 1j * rng.standard_normal((6, 2)))
    K = [V[2 * a:2 * a + 2] for a in range(3)]
    assert np.abs(sum(A.conj().T @ A for A in K) - np.eye(2)).max() <= 1e-14
    n, ops = chain_random_circuit(4, 3, 10)
    m, _, _ = run_circuit(n, ops, d_max=16, k_max=1, cutoff=0.0)
    for site in (1, 3, 0):
        before = m.to_density_matrix()
        m.apply_channel1(site, K, k_max=10 ** 6, cutoff=1e-14)
        want = sum(_apply1(before, A, site, n) for A in K)
        assert np.abs(m.to_density_matrix() - want).max() <= 1e-12
