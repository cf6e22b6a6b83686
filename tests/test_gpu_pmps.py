"""tn_pmps_* (locally-purified MPS, Sec. 3.4) on the GPU against the
complex128 PMPS oracle (O8) and the density-matrix oracle (O3).

Sites are complex64 and the merged pair comes from the FP32 GEMM, so the
density matrix agrees to ~1e-6; the SVDs and QRs run in FP64.  rho is
assembled on the host from the GPU's site tensors with the oracle's own
contraction (Kraus legs summed against their conjugates)."""

import numpy as np
import pytest

from oracle import noise
from oracle.gates import gate_matrix, is_channel, kraus_ops
from oracle.pmps import PMPS, run_circuit
from workloads import Op, chain_random_circuit, noisy_ops

pytestmark = pytest.mark.gpu


def gpu_run(n, ops, d_max, k_max, cutoff=1e-12):
    import paper_2104_10523_amd as tn
    m = tn.tn_pmps_create(n, d_max, k_max)
    db = dk = 0.0
    for op in ops:
        q = op.qubits
        if is_channel(op.name):
            b, k = m.apply_channel(q[0], kraus_ops(op.name, op.params), cutoff)
            db += b
            dk += k
        elif len(q) == 1:
            m.apply_gate1(q[0], gate_matrix(op.name, op.params))
        else:
            db += m.apply_gate(q[0], gate_matrix(op.name, op.params), cutoff)
    return m, db, dk


def gpu_rho(m, n):
    """rho of the GPU's sites, contracted by the oracle's own routine."""
    host = PMPS(n)
    host.sites = [m.site(i) for i in range(n)]
    return host.to_density_matrix().reshape(2 ** n, 2 ** n)


@pytest.mark.parametrize("n,cyc,seed,p2,d_max,k_max", [(6, 2, 3, 0.0, 64, 16), (4, 2, 1, 0.1, 16, 32)])
def test_pmps_untruncated_equals_density_matrix(gpu, n, cyc, seed, p2, d_max, k_max):
    """Depolarising (one-qubit, and two-qubit with p2 > 0) and damping after
    every gate, limits above what the exact state needs (bonds <= 4, Kraus
    <= 16 / 32): the GPU's rho equals O3's."""
    _, ops = chain_random_circuit(n, cyc, seed)
    ops = noisy_ops(ops, 0.05, p2, 0.08)
    m, db, dk = gpu_run(n, ops, d_max=d_max, k_max=k_max, cutoff=1e-9)
    ref = noise.dm_simulate(n, ops).reshape(2 ** n, 2 ** n)
    rho = gpu_rho(m, n)
    err = np.abs(rho - ref).max()
    print(f"pmps n={n}: |rho - rho_O3| max {err:.2e}, trace {np.trace(rho).real:.8f}, dims {m.dims()}", flush=True)
    assert err <= 1e-6
    assert abs(np.trace(rho) - 1) <= 1e-6
    assert np.abs(m.expect_z() - noise.dm_expect_z(noise.dm_simulate(n, ops), n)).max() <= 1e-6


def test_pmps_truncated_matches_oracle(gpu):
    """10-site noisy chain (depolarising 0.005 / 0.01, damping 0.01) with
    d_max = 16 and k_max = 4: the same truncations as the PMPS oracle --
    bond and Kraus dimensions, discarded weights, <Z_i> and rho."""
    n, ops = chain_random_circuit(10, 6, 21)
    ops = noisy_ops(ops, 0.005, 0.01, 0.01)
    ref, rdb, rdk = run_circuit(n, ops, d_max=16, k_max=4)
    m, db, dk = gpu_run(n, ops, d_max=16, k_max=4)
    bonds, kdims = m.dims()
    assert bonds == ref.bond_dims() and kdims == ref.kraus_dims()
    ez = np.abs(m.expect_z() - ref.expect_z()).max()
    erho = np.abs(gpu_rho(m, n) - ref.to_density_matrix().reshape(2 ** n, 2 ** n)).max()
    print(f"truncated: disc bond {db:.6f} vs {rdb:.6f}, kraus {dk:.6f} vs {rdk:.6f}, <Z> {ez:.2e}, rho {erho:.2e}",
          flush=True)
    assert abs(db - rdb) <= 1e-5 * max(1.0, rdb) and abs(dk - rdk) <= 1e-5 * max(1.0, rdk)
    assert ez <= 1e-5 and erho <= 1e-6


def test_pmps_asymmetric_gates(gpu):
    n = 4
    ops = [Op("h", (0,)), Op("sqrt_y", (2,)), Op("cx", (0, 1)), Op("amp_damp", (1,), (0.3,)),
           Op("sqrt_w", (1,)), Op("cx", (1, 2)), Op("amp_damp", (2,), (0.2,)), Op("cx", (2, 3)),
           Op("depol2", (2, 3), (0.1,)), Op("sqrt_x", (3,))]
    m, _, _ = gpu_run(n, ops, d_max=16, k_max=16, cutoff=1e-9)
    ref = noise.dm_simulate(n, ops).reshape(2 ** n, 2 ** n)
    assert np.abs(gpu_rho(m, n) - ref).max() <= 1e-6


def test_pmps_errors(gpu):
    import paper_2104_10523_amd as tn
    with pytest.raises(tn.TnError, match="ARG"):
        tn.tn_pmps_create(4, 0, 4)
    with pytest.raises(tn.TnError, match="ARG"):
        tn.tn_pmps_create(4, 8, 65)
    with pytest.raises(tn.TnError, match="UNSUPPORTED"):
        tn.tn_pmps_create(4, 256, 64)
    m = tn.tn_pmps_create(4, 8, 4)
    with pytest.raises(tn.TnError, match="SITE"):
        m.apply_gate(3, np.eye(4))
    with pytest.raises(tn.TnError, match="SITE"):
        m.apply_channel(3, kraus_ops("depol2", (0.1,)))
