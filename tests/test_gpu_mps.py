"""tn_mps_* on the GPU against the complex128 MPS oracle (O5) and the state
vector (O1).  Site tensors are complex64 and theta comes from the FP32 MFMA
GEMM, so amplitudes agree to ~1e-6; the SVD and QR run in FP64."""

import numpy as np
import pytest

from oracle import statevector as sv
from oracle.gates import gate_matrix
from oracle.mps import run_circuit
from workloads import chain_random_circuit

pytestmark = pytest.mark.gpu


def gpu_run(n, ops, chi_max, cutoff=1e-12):
    import paper_2104_10523_amd as tn
    m = tn.tn_mps_create(n, chi_max)
    disc = 0.0
    for op in ops:
        U = gate_matrix(op.name, op.params)
        if len(op.qubits) == 1:
            m.apply_gate1(op.qubits[0], U)
        else:
            disc += tn.tn_mps_apply_gate(m, op.qubits[0], U, chi_max, cutoff)
    return m, disc


@pytest.mark.parametrize("n,cyc", [(6, 4), (10, 6)])
def test_mps_untruncated_matches_state_vector(gpu, n, cyc):
    _, ops = chain_random_circuit(n, cyc, 11 + n)
    m, disc = gpu_run(n, ops, chi_max=1 << (n // 2), cutoff=0.0)
    psi = sv.simulate(n, ops)
    rng = np.random.default_rng(1)
    bits = rng.integers(0, 2, size=(32, n)).astype(np.int8)
    got = m.amplitudes(bits)
    ref = np.array([psi[tuple(b)] for b in bits])
    assert np.abs(got - ref).max() <= 2e-6
    assert np.abs(m.expect_z() - sv.expect_z(psi)).max() <= 2e-6
    assert disc <= 1e-10


def test_mps_truncated_matches_oracle(gpu):
    n, ops = chain_random_circuit(12, 8, 4)
    chi = 8
    ref, dref = run_circuit(n, ops, chi_max=chi)
    m, d = gpu_run(n, ops, chi_max=chi)
    assert m.bond_dims() == ref.bond_dims()
    assert abs(d - dref) <= 1e-4 * max(1.0, dref)
    rng = np.random.default_rng(2)
    bits = rng.integers(0, 2, size=(16, n)).astype(np.int8)
    got = m.amplitudes(bits)
    want = np.array([ref.amplitude(b) for b in bits])
    assert np.abs(got - want).max() <= 1e-4 * np.abs(want).max() + 1e-6
    assert np.abs(m.expect_z() - ref.expect_z()).max() <= 1e-4


def test_mps_errors(gpu):
    import paper_2104_10523_amd as tn
    m = tn.tn_mps_create(4, 4)
    with pytest.raises(tn.TnError, match="SITE"):
        tn.tn_mps_apply_gate(m, 3, np.eye(4), 4)
    with pytest.raises(tn.TnError, match="ARG"):
        tn.tn_mps_apply_gate(m, 0, np.eye(4), 0)
    with pytest.raises(tn.TnError, match="ARG"):
        tn.tn_mps_create(1, 4)
