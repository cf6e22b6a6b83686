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


@pytest.mark.timeout(400)
def test_c42_full_size_matches_oracle(gpu):
    """The MPS row's workload at full size: 40-site chain, 20 cycles of
    fSim(pi/2, pi/6) on alternating bonds, chi_max 256, cutoff 1e-12, against
    the complex128 MPS oracle (O5) gate by gate.  Compared: bond dimensions,
    the cumulative discarded weight, the last spectrum of every bond, <Z_i>
    and 16 amplitudes.  Truncated cuts whose singular values are degenerate
    (relative gap below 1e-10) would make the kept subspace ambiguous; the
    oracle reports their gaps, and none occurs here."""
    n, ops = chain_random_circuit(40, 20, 5)
    chi = 256
    ref, dref = run_circuit(n, ops, chi_max=chi)
    gaps = np.array(ref.cut_gaps)
    print(f"oracle: {len(gaps)} gates, smallest cut gap {gaps.min():.2e}, discarded {dref:.6f}", flush=True)
    assert gaps.min() > 1e-10
    m, d = gpu_run(n, ops, chi_max=chi)
    assert m.bond_dims() == ref.bond_dims()
    assert max(m.bond_dims()) == chi
    ed = abs(d - dref) / dref
    es = max(float(np.abs(m.bond_spectrum(b) - ref.spectra[b]).max()) for b in range(n - 1))
    ez = float(np.abs(m.expect_z() - ref.expect_z()).max())
    rng = np.random.default_rng(6)
    bits = rng.integers(0, 2, size=(16, n)).astype(np.int8)
    got = m.amplitudes(bits)
    want = np.array([ref.amplitude(b) for b in bits])
    ea = float(np.abs(got - want).max() / np.sqrt(np.mean(np.abs(want) ** 2)))
    print(f"discarded rel {ed:.2e}, spectra {es:.2e}, <Z> {ez:.2e}, amplitudes (rel to rms) {ea:.2e}", flush=True)
    # complex64 sites and FP32 theta perturb each gate by ~1e-7; the kept
    # singular vectors at a cut with relative gap g rotate by ~1e-7 / g
    # (smallest gap here 5e-4), which individual amplitudes feel most
    assert ed <= 1e-6 and es <= 1e-5 and ez <= 1e-5 and ea <= 2e-3


def test_mps_bond_spectrum_matches_oracle(gpu):
    n, ops = chain_random_circuit(12, 8, 4)
    ref, _ = run_circuit(n, ops, chi_max=8)
    m, _ = gpu_run(n, ops, chi_max=8)
    for b in range(n - 1):
        s = m.bond_spectrum(b)
        assert s.shape == ref.spectra[b].shape
        assert np.abs(s - ref.spectra[b]).max() <= 1e-5
        assert abs(np.sum(s ** 2) - 1) <= 1e-12


def test_mps_errors(gpu):
    import paper_2104_10523_amd as tn
    m = tn.tn_mps_create(4, 4)
    with pytest.raises(tn.TnError, match="SITE"):
        tn.tn_mps_apply_gate(m, 3, np.eye(4), 4)
    with pytest.raises(tn.TnError, match="ARG"):
        tn.tn_mps_apply_gate(m, 0, np.eye(4), 0)
    with pytest.raises(tn.TnError, match="ARG"):
        tn.tn_mps_create(1, 4)
    with pytest.raises(tn.TnError, match="SITE"):
        m.bond_spectrum(3)
