"""Pauli expectation values on the GPU (Sec. 3.1, Eq. 2, Table 1) against the
oracle's direct definition <Psi|P|Psi>.

Both methods of the paper: the conjugate (double-depth) network, contracted
as one all-zero amplitude, and wave-function slicing, reduced on the device.
<P> lies in [-1, 1]; the bar is an absolute error of 1e-5 (complex64
contraction, FP64 accumulation), and the imaginary part of a Hermitian
string's value within the same bound of zero.
"""

import itertools

import numpy as np
import pytest

from oracle import observables as ob
from workloads import Op, chain_random_circuit, ghz_circuit, grid_random_circuit

pytestmark = pytest.mark.gpu
TOL = 1e-5


def random_pauli(n, weight, rng, allowed=None):
    codes = [0] * n
    pool = list(range(n)) if allowed is None else list(allowed)
    for q in rng.choice(pool, size=weight, replace=False):
        codes[int(q)] = int(rng.integers(1, 4))
    return codes


def conjugate_value(n, ops, codes, precision="fp32", algo="greedy"):
    import paper_2104_10523_amd as tn
    net, kept = tn.tn_build_expectation_network(n, ops, codes)
    path = tn.tn_find_path(net, algo, trials=16, seed=1)
    out, rep = tn.tn_amplitudes(net, path, np.zeros((1, n), np.int8), precision=precision)
    return complex(out.cpu().numpy()[0, 0]), kept, rep


def sliced_value(n, ops, codes, open_q, precision="fp32"):
    import paper_2104_10523_amd as tn
    proj = [q for q in range(n) if q not in open_q]
    bits = np.full((1 << len(proj), n), -1, np.int8)
    for s, vals in enumerate(itertools.product((0, 1), repeat=len(proj))):
        bits[s, proj] = vals
    net = tn.tn_build_network(n, ops)
    open_mask = (bits[0] < 0).astype(np.int8)
    path = tn.tn_find_path(net, "greedy", open_mask=open_mask)
    psi, _ = tn.tn_amplitudes(net, path, bits, precision=precision)
    return tn.tn_pauli_expectation(psi, bits, codes)


@pytest.mark.parametrize("precision", ["fp32", "f16x3"])
@pytest.mark.parametrize("seed", range(3))
def test_conjugate_network_matches_oracle(gpu, workspace, precision, seed):
    rng = np.random.default_rng(seed)
    n, ops = grid_random_circuit(3, 4, 5 + seed, 700 + seed)
    codes = random_pauli(n, 1 + seed, rng)
    got, kept, rep = conjugate_value(n, ops, codes, precision)
    ref = ob.expectation(n, ops, codes)
    assert abs(got - ref) <= TOL, (got, ref)
    assert kept == len(ob.light_cone(n, ops, codes))
    assert rep.nonfinite == 0


def test_conjugate_network_chain_light_cone(gpu, workspace):
    """A 20-qubit chain: a Z on an end qubit keeps only its light cone, so
    the double-depth network stays small although the state has 2^20
    entries."""
    n, ops = chain_random_circuit(20, 4, 3)
    codes = [0] * n
    codes[0] = 3
    got, kept, _ = conjugate_value(n, ops, codes)
    assert kept < len(ops) // 2
    ref = ob.conjugate_network_value(n, ops, codes, collapse=True)
    assert abs(got - ref) <= TOL


def test_ghz_closed_forms_on_gpu(gpu, workspace):
    n, ops = ghz_circuit(5)
    for s, want in [("ZZIII", 1.0), ("XXXXX", 1.0), ("YYXXX", -1.0), ("ZIIII", 0.0), ("IIIII", 1.0)]:
        got, _, _ = conjugate_value(n, ops, s)
        assert abs(got - want) <= TOL, (s, got)
        got2 = sliced_value(n, ops, [ob.CODES[c] for c in s], [0, 1, 2, 3, 4])
        assert abs(got2 - want) <= TOL, (s, got2)


@pytest.mark.parametrize("seed", range(3))
def test_sliced_matches_oracle(gpu, workspace, seed):
    rng = np.random.default_rng(10 + seed)
    n, ops = grid_random_circuit(3, 4, 6, 800 + seed)
    open_q = sorted(int(q) for q in rng.choice(n, size=7, replace=False))
    codes = random_pauli(n, 2, rng, allowed=open_q)
    # a Z on a projected qubit is a per-slice sign
    proj = [q for q in range(n) if q not in open_q]
    codes[proj[seed]] = 3
    got = sliced_value(n, ops, codes, open_q)
    ref = ob.expectation(n, ops, codes)
    assert abs(got - ref) <= TOL, (got, ref)
    assert abs(got - ob.sliced_expectation(n, ops, codes, open_q)) <= TOL


@pytest.mark.parametrize("n_open,n_slices", [(0, 1), (0, 5), (1, 3), (5, 1), (7, 37), (12, 3)])
def test_reduction_kernel_on_random_slices(gpu, n_open, n_slices):
    """tn_pauli_expectation against a numpy evaluation on arbitrary (not
    normalised) slices: ragged slice counts, every Pauli on the open bits,
    Z signs on projected bits."""
    import torch
    import paper_2104_10523_amd as tn
    rng = np.random.default_rng(n_open * 100 + n_slices)
    n = n_open + 4
    psi = rng.standard_normal((n_slices, 1 << n_open)) + 1j * rng.standard_normal((n_slices, 1 << n_open))
    open_q = sorted(int(q) for q in rng.choice(n, size=n_open, replace=False))
    proj = [q for q in range(n) if q not in open_q]
    bits = np.full((n_slices, n), -1, np.int8)
    bits[:, proj] = rng.integers(0, 2, size=(n_slices, len(proj)))
    codes = [0] * n
    for q in open_q:
        codes[q] = int(rng.integers(0, 4))
    codes[proj[0]] = 3
    got = tn.tn_pauli_expectation(torch.from_numpy(psi).to("cuda"), bits, codes)
    want = 0j
    for s in range(n_slices):
        v = psi[s].reshape((2,) * n_open) if n_open else psi[s].reshape(())
        pv = ob.apply_pauli(v, [codes[q] for q in open_q]) if n_open else v
        sign = -1.0 if bits[s, proj[0]] == 1 else 1.0
        want += sign * np.vdot(v.reshape(-1), np.asarray(pv).reshape(-1))
    assert abs(got - want) <= 1e-10 * max(1.0, abs(want)) * (1 << n_open), (got, want)


def test_expectation_errors(gpu, workspace):
    import torch
    import paper_2104_10523_amd as tn
    n, ops = ghz_circuit(3)
    bits = np.array([[-1, 0, -1], [-1, 1, -1]], np.int8)
    psi = torch.zeros((2, 4), dtype=torch.complex128, device="cuda")
    with pytest.raises(tn.TnError, match="TN_ERR_ARG"):
        tn.tn_pauli_expectation(psi, bits, "IXI")          # X on a projected qubit
    with pytest.raises(tn.TnError, match="TN_ERR_BITS"):
        tn.tn_pauli_expectation(psi, np.array([[-1, 0, -1], [-1, -1, 0]], np.int8), "ZII")
    with pytest.raises(tn.TnError, match="TN_ERR_GATE"):
        tn.tn_build_expectation_network(n, ops + [Op("amp_damp", (0,), (0.1,))], "ZII")
