"""tn_contract_pair on the GPU against the complex128 einsum oracle (O2).

Label sets are drawn at random: batch, contracted (K), free (M, N) and
summed-out labels in shuffled orders, so every kernel path is exercised:
bit-addressed small-operand apply, permute + MFMA GEMM (FP32, BF16x3,
BF16x6, scaled FP16x3), split-K, dot, outer product, scalar output, pure
permutation and ragged tiles.

Tolerances (relative L2 over C): FP32 and BF16x6 2e-6; BF16x3 2e-5 (a
bfloat16 hi + lo split keeps 16 significant bits, products within 2^-17);
FP16x3 3e-6 (fp16 hi + lo keeps 22 bits, products within 2^-21).
"""

import zlib

import numpy as np
import pytest

from oracle.contract import contract_pair as oracle_pair
from workloads import random_complex
from tests.helpers import l2_rel, floored_rel

pytestmark = pytest.mark.gpu

TOL = {"fp32": 2e-6, "bf16x6": 2e-6, "bf16x3": 2e-5, "f16x3": 3e-6}


def make_case(seed, nb=0, nm=0, nk=0, nn=0, da=0, db=0, wide=None, shuffle=True):
    rng = np.random.default_rng(seed)
    labels = list(range(100, 100 + nb + nm + nk + nn + da + db))
    rng.shuffle(labels)
    it = iter(labels)
    L = {k: [next(it) for _ in range(c)] for k, c in
         (("b", nb), ("m", nm), ("k", nk), ("n", nn), ("da", da), ("db", db))}
    ext = {l: 2 for l in labels}
    if wide:
        for l in L["k"][:1] + L["m"][:1]:
            ext[l] = wide
    la = L["b"] + L["m"] + L["k"] + L["da"]
    lb = L["b"] + L["k"] + L["n"] + L["db"]
    lc = L["b"] + L["m"] + L["n"]
    if shuffle:
        la = list(rng.permutation(la)) if la else la
        lb = list(rng.permutation(lb)) if lb else lb
        lc = list(rng.permutation(lc)) if lc else lc
    la, lb, lc = [int(x) for x in la], [int(x) for x in lb], [int(x) for x in lc]
    A = random_complex([ext[l] for l in la], seed + 1, dtype=np.complex64)
    B = random_complex([ext[l] for l in lb], seed + 2, dtype=np.complex64)
    return A, la, B, lb, lc, [ext[l] for l in lc]


def run(A, la, B, lb, lc, shape_c, precision):
    import torch
    import paper_2104_10523_amd as tn
    dA = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    dB = torch.from_numpy(np.ascontiguousarray(B)).cuda()
    dC = torch.full(shape_c, complex(float("nan"), 0), dtype=torch.complex64, device="cuda")
    tn.tn_contract_pair(dA, la, dB, lb, dC, lc, precision)
    torch.cuda.synchronize()
    return dC.cpu().numpy()


CASES = [
    # (name, kwargs)
    ("apply_k1", dict(nm=14, nk=1, nn=2)),
    ("apply_k2_n2", dict(nm=16, nk=2, nn=2)),
    ("apply_k4_n4", dict(nm=12, nk=4, nn=4)),
    ("apply_k6_n0", dict(nm=10, nk=6, nn=0)),
    # 16 outputs per row: the matrix-core apply (32-row groups, KK = 2 .. 64)
    ("apply_k1_n4", dict(nm=16, nk=1, nn=4)),
    ("apply_k3_n4_many_groups", dict(nm=20, nk=3, nn=4)),
    ("apply_k6_n4", dict(nm=5, nk=6, nn=4)),
    # 32 and 64 outputs per row: the matrix-core apply with 2 or 4 column blocks
    ("apply_k6_n6", dict(nm=10, nk=6, nn=6)),
    ("apply_k5_n5", dict(nm=12, nk=5, nn=5)),
    ("apply_k6_n6_64_rows", dict(nm=6, nk=6, nn=6)),
    ("apply_k2_n5_b_summed", dict(nm=9, nk=2, nn=5, db=1)),
    ("gemm_square", dict(nm=9, nk=7, nn=8)),
    ("gemm_ragged_small_mn", dict(nm=5, nk=6, nn=5)),
    ("gemm_n16", dict(nm=11, nk=7, nn=4 + 1)),
    ("gemm_n32", dict(nm=10, nk=8, nn=5)),
    ("gemm_splitk", dict(nm=6, nk=14, nn=6)),
    ("gemm_splitk_ragged", dict(nm=5, nk=15, nn=3)),      # 32 x 8 outputs, K = 2^15 split over blocks
    ("gemm_k_beyond_packed_panels", dict(nm=2, nk=21, nn=2)),   # K = 2^21: packed planes would overflow
    ("dot_small_mn", dict(nm=2, nk=17, nn=2)),          # 4 x 4 outputs, K = 2^17: dot per (m, n) pair
    ("dot_small_mn_batch", dict(nb=2, nm=1, nk=16, nn=3)),
    ("skinny_8x8", dict(nm=3, nk=18, nn=3)),            # 8 x 8 outputs over K = 2^18: skinny kernel
    ("skinny_16x4", dict(nm=4, nk=17, nn=2)),
    ("skinny_2x1", dict(nm=1, nk=16, nn=0)),
    ("gemm_batch", dict(nb=3, nm=7, nk=6, nn=6)),
    ("gemm_wide_extents", dict(nm=5, nk=3, nn=6, wide=8)),
    ("outer_product", dict(nm=8, nk=0, nn=6)),
    ("dot", dict(nk=16)),
    ("dot_batch", dict(nb=2, nk=12)),
    ("scalar_times_tensor", dict(nm=10)),
    ("sum_out_a", dict(nm=8, nk=3, nn=6, da=2)),
    ("sum_out_b_apply", dict(nm=12, nk=2, nn=2, db=1)),
    ("rank0_all", dict()),
]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "bf16x6", "f16x3"])
@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
def test_contract_pair(gpu, workspace, name, kw, precision):
    seed = zlib.crc32(f"{name}/{precision}".encode()) % 10000
    A, la, B, lb, lc, shape_c = make_case(seed, **kw)
    print(f"case {name} prec {precision} A{A.shape} B{B.shape} la={la} lb={lb} lc={lc}", flush=True)
    got = run(A, la, B, lb, lc, shape_c, precision)
    ref = oracle_pair(A.astype(np.complex128), la, B.astype(np.complex128), lb, lc)
    assert np.all(np.isfinite(got))
    err = l2_rel(got, ref)
    tol = TOL[precision]
    if name == "gemm_k_beyond_packed_panels":
        # K = 2^21 runs on the FP32 kernel at every precision: 4096-long FP32
        # chains plus 512 chunk additions, 2^-24 * sqrt(4096 + 512) ~ 4e-6
        tol = max(tol, 4e-6)
    assert err <= tol, (name, precision, err)


@pytest.mark.parametrize("nk,nn", [(1, 0), (2, 2), (3, 3), (4, 4), (4, 2)])
def test_contract_pair_apply_low_k_bits(gpu, workspace, nk, nn):
    """A small operand contracted over A's lowest labels (the K bits sit
    below every M bit): the LDS-tiled apply kernel reads each block's rows as
    one contiguous run."""
    A, la, B, lb, lc, shape_c = make_case(60 + 7 * nk + nn, nm=12, nk=nk, nn=nn, shuffle=False)
    got = run(A, la, B, lb, lc, shape_c, "fp32")
    ref = oracle_pair(A.astype(np.complex128), la, B.astype(np.complex128), lb, lc)
    assert l2_rel(got, ref) <= 2e-6


def test_contract_pair_unshuffled_orders(gpu, workspace):
    """Operands already in GEMM order (no permutation kernels)."""
    A, la, B, lb, lc, shape_c = make_case(7, nm=8, nk=6, nn=7, shuffle=False)
    got = run(A, la, B, lb, lc, shape_c, "fp32")
    ref = oracle_pair(A.astype(np.complex128), la, B.astype(np.complex128), lb, lc)
    assert l2_rel(got, ref) <= 2e-6


def test_contract_pair_large_mfma(gpu, workspace):
    """A contraction spanning many MFMA tiles (M = 2^12, N = 2^11, K = 2^9),
    all precisions, on 2048 sampled output entries that the oracle computes
    one by one."""
    from oracle.contract import contract_entries
    A, la, B, lb, lc, shape_c = make_case(11, nm=12, nk=9, nn=11)
    rng = np.random.default_rng(5)
    idx = [tuple(int(rng.integers(0, e)) for e in shape_c) for _ in range(2048)]
    ref = contract_entries(A.astype(np.complex128), la, B.astype(np.complex128), lb, lc, idx)
    rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    for prec in ("fp32", "bf16x3", "bf16x6", "f16x3"):
        got = run(A, la, B, lb, lc, shape_c, prec)
        g = np.array([got[i] for i in idx])
        e2 = l2_rel(g, ref)
        ef = floored_rel(g, ref, 0.1 * rms)
        print(f"large {prec}: l2 {e2:.2e} floored {ef:.2e}", flush=True)
        assert e2 <= TOL[prec], (prec, e2)
        assert ef <= 20 * TOL[prec], (prec, ef)


@pytest.mark.parametrize("precision,scale", [("bf16x3", 1.0), ("f16x3", 1.0), ("f16x3", 2.0 ** -25)])
def test_contract_pair_dma_chunk_flush(gpu, workspace, precision, scale):
    """M = 2^13, N = 2^12, K = 2^13 in shuffled label orders: whole 256 x 128
    tiles and K % 16 = 0 select the direct-to-LDS split kernel, 1024 block
    tiles need no split-K, and K > 4096 makes every block flush its FP32
    accumulators into C once mid-K (with the exact power-of-two rescale of
    scaled FP16 operands; scale 2^-25 is the benchmark's amplitude scale).
    4096 sampled entries against the oracle, computed one by one."""
    from oracle.contract import contract_entries
    A, la, B, lb, lc, shape_c = make_case(13, nm=13, nk=13, nn=12)
    if scale != 1.0:
        A = (A * np.float32(scale)).astype(np.complex64)
    rng = np.random.default_rng(17)
    idx = [tuple(int(rng.integers(0, e)) for e in shape_c) for _ in range(4096)]
    ref = contract_entries(A.astype(np.complex128), la, B.astype(np.complex128), lb, lc, idx)
    import torch
    import paper_2104_10523_amd as tn
    big = torch.empty(3 << 30, dtype=torch.uint8, device=gpu)   # 2 packed operands + C
    tn.tn_set_workspace(big)
    try:
        got = run(A, la, B, lb, lc, shape_c, precision)
    finally:
        tn.tn_set_workspace(workspace)
        del big
    g = np.array([got[i] for i in idx])
    rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    e2 = l2_rel(g, ref)
    ef = floored_rel(g, ref, 0.1 * rms)
    print(f"dma flush {precision} x{scale:g}: l2 {e2:.2e} floored {ef:.2e}", flush=True)
    assert np.all(np.isfinite(g))
    assert e2 <= TOL[precision], e2
    assert ef <= 20 * TOL[precision], ef


@pytest.mark.parametrize("sa,sb", [(1e-25, 1e20), (1e30, 1e-30), (3e-7, 5e4)])
def test_contract_pair_f16_operand_scaling(gpu, workspace, sa, sb):
    """Split-FP16 scales each operand by a power of two from its largest
    entry, so magnitudes far outside fp16's range (6e-8 .. 65504) keep their
    accuracy; the product's scale is undone exactly."""
    A, la, B, lb, lc, shape_c = make_case(31, nm=9, nk=7, nn=8)
    A = (A * np.float32(sa)).astype(np.complex64)
    B = (B * np.float32(sb)).astype(np.complex64)
    got = run(A, la, B, lb, lc, shape_c, "f16x3")
    ref = oracle_pair(A.astype(np.complex128), la, B.astype(np.complex128), lb, lc)
    assert np.all(np.isfinite(got))
    assert l2_rel(got, ref) <= TOL["f16x3"], l2_rel(got, ref)


def test_contract_pair_f16_wide_range_and_zero(gpu, workspace):
    """Entries spanning eight decades within one operand stay accurate in
    the L2 sense; an all-zero operand gives exact zeros."""
    A, la, B, lb, lc, shape_c = make_case(32, nm=8, nk=8, nn=8)
    rng = np.random.default_rng(3)
    A = (A * (10.0 ** rng.uniform(-8, 0, A.shape))).astype(np.complex64)
    got = run(A, la, B, lb, lc, shape_c, "f16x3")
    ref = oracle_pair(A.astype(np.complex128), la, B.astype(np.complex128), lb, lc)
    assert l2_rel(got, ref) <= TOL["f16x3"], l2_rel(got, ref)
    got0 = run(np.zeros_like(A), la, B, lb, lc, shape_c, "f16x3")
    assert np.all(got0 == 0)


def test_contract_pair_errors(gpu, workspace):
    import torch
    import paper_2104_10523_amd as tn
    a = torch.zeros((2, 2), dtype=torch.complex64, device="cuda")
    b = torch.zeros((2, 2), dtype=torch.complex64, device="cuda")
    c = torch.zeros((2, 2), dtype=torch.complex64, device="cuda")
    with pytest.raises(tn.TnError, match="MODES"):
        tn.tn_contract_pair(a, [1, 1], b, [1, 2], c, [1, 2])
    with pytest.raises(tn.TnError, match="MODES"):
        tn.tn_contract_pair(a, [1, 2], b, [2, 3], c, [1, 9])
    c3 = torch.zeros((3, 2), dtype=torch.complex64, device="cuda")
    with pytest.raises(tn.TnError, match="EXTENT"):
        tn.tn_contract_pair(a, [1, 2], b, [2, 3], c3, [1, 3])
