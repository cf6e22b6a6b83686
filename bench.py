"""Benchmark: amplitudes of the 49-qubit 7x7 random grid circuit (14 cycles,
fSim(pi/2, pi/6)) on one MI355X.

Workload: 64 seeded uniform bit-strings; the contraction path is the best of
greedy and 1024 recursive-bisection trees (run on host threads), each sliced
so that the live set of one slice fits the memory budget.  One *step* is one job of the hot
path: one bit-string x one slice, from the leaf gather through every
pairwise contraction to the FP64 accumulation of the amplitude.  The whole
job (64 bit-strings x 2^k slices) cannot run in minutes, so `value` is the
whole-job amplitude rate extrapolated from the timed steps (every slice has
the same shapes): amplitudes/s = 1 / (2^k x seconds per step).

The timed region replays the job's captured hipGraph (the production path).
A profiled pass after it times every op with HIP events; the kernel with the
largest share of a step is the roofline entry (HBM-bound unless it is a GEMM
whose intensity reaches the balance point of its own arithmetic).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

PEAKS = {"bf16x3": 2.5e15, "bf16x6": 2.5e15, "f16x3": 2.5e15, "fp32": 157.3e12}
HBM_PEAK = 8.0e12


# tile id -> (BM, BN, BK, WGM, WGN) of the kernels in csrc/kernels.hip
PACKED_TILES = {2: {0: (256, 16, 32, 4, 1), 1: (128, 32, 32, 4, 1), 2: (128, 64, 32, 2, 2),
                    3: (256, 128, 16, 4, 2), 4: (128, 128, 16, 2, 2), 5: (256, 128, 16, 4, 2)},
                3: {0: (256, 16, 16, 4, 1), 1: (128, 32, 16, 4, 1), 2: (128, 64, 16, 2, 2),
                    4: (128, 128, 16, 2, 2)}}
UNPACKED_TILES = {0: (256, 16), 1: (128, 32), 2: (128, 64), 3: (64, 64)}


def kernel_name(precision, tile, packed):
    if precision == "auto":       # packed GEMMs run split FP16x3, the others FP32
        precision = "f16x3" if packed else "fp32"
    if packed:
        np_ = 3 if precision == "bf16x6" else 2
        bm, bn, bk, wm, wn = PACKED_TILES[np_][tile]
        kern = "gemm_packed_dma_kernel" if tile == 5 else "gemm_packed_kernel"
        f16 = "true" if precision == "f16x3" else "false"
        return f"{kern}<{bm}, {bn}, {bk}, {wm}, {wn}, {np_}, {f16}>"
    bm, bn = UNPACKED_TILES[tile]
    if precision == "f16x3":
        precision = "fp32"        # split FP16 exists only on packed planes
    bk = 8 if precision == "fp32" else 16
    wm, wn = (2, 2) if bn >= 64 else (4, 1)
    prec_id = {"fp32": 0, "bf16x3": 1, "bf16x6": 2}[precision]      # TN_PREC_* template argument
    return f"gemm_mfma_kernel<{bm}, {bn}, {bk}, {wm}, {wn}, {prec_id}>"


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` on this workload from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, calibrated against a
    1 GiB copy).  None when no summary covers the kernel or the kernel
    source has changed since the counters were taken."""
    import hashlib
    src = hashlib.sha256((ROOT / "paper_2104_10523_amd" / "csrc" / "kernels.hip").read_bytes()).hexdigest()
    for f in sorted((ROOT / "profiles").glob("*__hbm_traffic.txt")):
        kv = dict(l.split(": ", 1) for l in f.read_text().splitlines() if ": " in l and not l.startswith(" "))
        if kv.get("kernel") == kernel and kv.get("kernels_hip_sha256") == src:
            return float(kv["traffic_bytes_per_launch"]), f.name
    return None, None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="auto", choices=["bf16x3", "bf16x6", "f16x3", "fp32", "auto"],
                    help="auto: scaled split-FP16x3 for GEMMs with K >= 64, M >= 1024, N >= 64, FP32 otherwise")
    ap.add_argument("--compare-fp32", type=int, default=1, help="also time FP32 steps")
    ap.add_argument("--budget-gib", type=float, default=160.0)
    ap.add_argument("--trials", type=int, default=1024, help="path search trials")
    ap.add_argument("--path", default="partition", choices=["partition", "random_greedy"],
                    help="path search for the 7x7 workload")
    ap.add_argument("--rank", default="time", choices=["time", "flops"],
                    help="partition search: re-rank the best candidates by modelled kernel time (default) "
                         "or keep the flop-minimal tree")
    ap.add_argument("--validate", type=int, default=4,
                    help="(bit-string, slice) jobs also run at the FP64 validation precision; the line reports "
                         "the benchmark precision's and FP32's error against them")
    ap.add_argument("--profile-steps", type=int, default=1,
                    help="jobs run once more with HIP events around every kernel, after the timed region")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--rows", type=int, default=7)
    ap.add_argument("--cols", type=int, default=7)
    ap.add_argument("--cycles", type=int, default=14)
    ap.add_argument("--autotune", type=int, default=1,
                    help="run the GEMM tile autotuner before the warmup (its trial launches appear in kernel traces)")
    ap.add_argument("--workload", default="c2", choices=["c2", "c1", "c3", "traj", "mps", "pmps", "learned", "expval", "dm"],
                    help="c2 (default) is the benchmark line; the others measure the remaining rows")
    ap.add_argument("--learned-train", type=int, default=5000, help="learned row: training circuits")
    ap.add_argument("--learned-test", type=int, default=200, help="learned row: held-out circuits")
    ap.add_argument("--learned-epochs", type=int, default=6)
    ap.add_argument("--learned-batch", type=int, default=64)
    ap.add_argument("--learned-lr", type=float, default=1e-3)
    ap.add_argument("--learned-rescore", type=int, default=8, help="merges per scoring of the second learned search")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run one 1 GiB device-to-device copy (a counter calibration kernel)")
    return ap.parse_args()


def make_workload(a):
    import paper_2104_10523_amd as tn
    from workloads import grid_random_circuit, random_bitstrings
    n, ops = grid_random_circuit(a.rows, a.cols, a.cycles, 2, two_qubit="fsim")
    bits = random_bitstrings(64, n, 12345)
    net = tn.tn_build_network(n, ops)
    t0 = time.time()
    if a.path == "partition":
        path = tn.tn_find_path(net, "partition", trials=a.trials, seed=1, mem_budget_bytes=a.budget_gib * 2 ** 30,
                               rank=a.rank, rank_precision=a.precision)
    else:
        path = tn.tn_find_path(net, "random_greedy", trials=a.trials, seed=1, temperature=0.5,
                               mem_budget_bytes=a.budget_gib * 2 ** 30)
    t_path = time.time() - t0
    return n, ops, bits, net, path, t_path


def plan_ops(net, path, precision):
    import ctypes as C
    import paper_2104_10523_amd as tn
    from paper_2104_10523_amd._native import TnPlanInfo, PREC
    info = TnPlanInfo()
    tn._native.check(tn.lib().tn_amplitudes_plan_info(net.h, path.h, PREC[precision], C.byref(info)))
    N = info.n_ops
    kind = (C.c_int32 * N)()
    fl = (C.c_double * N)()
    by = (C.c_double * N)()
    shape = (C.c_int64 * (8 * N))()
    tn._native.check(tn.lib().tn_amplitudes_plan_ops(net.h, path.h, PREC[precision], kind, fl, by, shape))
    return info, np.array(kind), np.array(fl), np.array(by), np.array(shape).reshape(N, 8)


def time_steps(net, path, bits, precision, jobs, stream):
    """Run each (bit-string, slice) job once with per-op events; returns the
    wall time of every job (device events) and the per-op seconds summed."""
    import ctypes as C
    import torch
    import paper_2104_10523_amd as tn
    from paper_2104_10523_amd._native import TnExecOpts, TnReport, PREC
    info, kind, fl, by, shape = plan_ops(net, path, precision)
    op_sec = np.zeros(info.n_ops)
    per_job = []
    amps = []
    out = torch.zeros((1, 1), dtype=torch.complex128, device="cuda")
    for (b, s) in jobs:
        buf = np.zeros(info.n_ops)
        o = TnExecOpts(PREC[precision], 0, int(s), 1, 0, 1,
                       buf.ctypes.data_as(C.POINTER(C.c_double)))
        rep = TnReport()
        bb = np.ascontiguousarray(bits[b:b + 1])
        tn._native.check(tn.lib().tn_amplitudes(net.h, path.h, bb.ctypes.data_as(C.POINTER(C.c_int8)), 1,
                                                C.byref(o), C.c_void_p(out.data_ptr()), C.byref(rep),
                                                C.c_void_p(stream.cuda_stream)))
        per_job.append(rep.seconds)
        op_sec += buf
        amps.append(complex(out.cpu().numpy()[0, 0]))
        if rep.nonfinite:
            raise RuntimeError("non-finite amplitude")
    return np.array(per_job), op_sec, (info, kind, fl, by, shape), np.array(amps)


def blas_threads():
    """Threads of the BLAS library numpy calls (what the matmul oracle uses)."""
    try:
        from threadpoolctl import threadpool_info
        return max([p.get("num_threads", 1) for p in threadpool_info() if p.get("user_api") == "blas"] or [1])
    except Exception:
        return 1


def cpu_baseline(path_pairs, net_py, budget_s):
    """The oracle (complex128; each pairwise step one batched matrix
    product, oracle.contract.contract_pair_mm, on all BLAS threads) timed on
    the workload's own pairwise contractions, largest first among those
    whose tensors fit in 2^25 entries and whose cost is at most 2e10 flops
    (a few seconds each), cycling through them until budget_s of wall time;
    returns flops/s."""
    from oracle.contract import contract_pair_mm
    from oracle.paths import path_stats
    from workloads import random_complex
    leaves, ext, open_l, sliced = net_py
    st = path_stats(leaves, ext, path_pairs, open_l, sliced)
    steps = []
    for (a, b, c) in st["steps"]:
        f = 8.0 * 2 ** len(a | b)
        if max(len(a), len(b), len(c)) <= 25 and f <= 2e10:
            steps.append((f, sorted(a), sorted(b), sorted(c)))
    steps.sort(key=lambda x: -x[0])
    # operands: leading parts of two seeded random pools (drawn once)
    top = max([max(len(s[1]), len(s[2])) for s in steps], default=0)
    pools = [random_complex([1 << top], 1), random_complex([1 << top], 2)]
    done_f, done_t, k = 0.0, 0.0, 0
    while done_t < budget_s and steps:
        f, la, lb, lc = steps[k % len(steps)]
        A = pools[0][:1 << len(la)].reshape([2] * len(la))
        B = pools[1][:1 << len(lb)].reshape([2] * len(lb))
        t0 = time.perf_counter()
        contract_pair_mm(A, la, B, lb, lc)
        done_t += time.perf_counter() - t0
        done_f += f
        k += 1
    return done_f / done_t, done_t, done_f


# --------------------------------------------------------------------------
# Other rows of the hot path (non-default `--workload`): one JSON line each,
# with the roofline entry of the dominant kernel where one applies and the
# oracle timed beside it.  The default run (C2) above is the benchmark line.

def _timed(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def bench_c1(a):
    """3x4 grid, 8 cycles, CZ: all 4096 amplitudes (all legs open) and the
    all-zeros amplitude; launch/latency-bound (< 1e8 flops)."""
    import paper_2104_10523_amd as tn
    from workloads import grid_random_circuit
    from oracle import statevector as sv
    import torch
    n, ops = grid_random_circuit(3, 4, 8, 1)
    net = tn.tn_build_network(n, ops)
    ws = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    tn.tn_set_workspace(ws)
    res = {}
    for name, bits in (("all_open", [-1] * n), ("all_zeros", [0] * n)):
        bits = np.array([bits], dtype=np.int8)
        path = tn.tn_find_path(net, "greedy", open_mask=(bits[0] < 0).astype(np.int8))
        out = {}
        for g in (0, 1):
            T = _timed(lambda: tn.tn_amplitudes(net, path, bits, precision="fp32", use_graph=bool(g)), 20)
            out["graph" if g else "eager"] = T
        _, rep = tn.tn_amplitudes(net, path, bits, precision="fp32")
        res[name] = {"seconds": out, "flops": rep.flops, "bytes": rep.bytes,
                     "amplitudes": int(2 ** (bits[0] < 0).sum())}
    T = min(res["all_open"]["seconds"].values())
    t0 = time.perf_counter()
    for _ in range(5):
        sv.simulate(n, ops)
    t_cpu = (time.perf_counter() - t0) / 5
    return {"metric": "amplitudes/s, 12-qubit 3x4 grid depth 8 (all 4096 amplitudes)",
            "value": 4096 / T, "unit": "amplitudes/s", "dtype": "c64 fp32",
            "config": {"workload": "3x4 grid random circuit, 8 cycles, CZ, seed 1, greedy path", "runs": res},
            "roofline": {"bound": "hbm", "achieved": res["all_open"]["bytes"] / T / 1e9, "peak": HBM_PEAK / 1e9,
                         "unit": "GB/s", "frac": res["all_open"]["bytes"] / T / HBM_PEAK, "traffic": None,
                         "note": "launch/latency-bound: ~1e5 flops per kernel"},
            "cpu_baseline": {"value": 4096 / t_cpu, "unit": "amplitudes/s", "cores": 1, "kind": "oracle",
                             "sample": "oracle state-vector simulation of the whole circuit (complex128), 5 runs"}}


def bench_c3(a):
    """Pairwise contractions with C1's structure (extents 2, random mode
    orders), output ranks 24-30, contracted ranks 2-15, per precision:
    TFLOP/s and error on 4096 sampled entries against the oracle."""
    import torch
    import paper_2104_10523_amd as tn
    from oracle.contract import contract_entries, contract_pair
    shapes = [(16, 16, 2), (20, 20, 8), (26, 26, 12), (30, 30, 15)]   # (rank A, rank B, k)
    ws = torch.empty(40 << 30, dtype=torch.uint8, device="cuda")
    tn.tn_set_workspace(ws)
    rows, best = [], None
    for ra, rb, k in shapes:
        rng = np.random.default_rng(3 + ra)
        kl = list(range(1000, 1000 + k))
        la = list(range(ra - k)) + kl
        lb = kl + list(range(2000, 2000 + rb - k))
        rng.shuffle(la)
        rng.shuffle(lb)
        lc = list(range(ra - k)) + list(range(2000, 2000 + rb - k))
        rng.shuffle(lc)
        g = torch.Generator(device="cuda")
        g.manual_seed(ra * 100 + k)
        A = torch.randn([2] * ra, dtype=torch.complex64, device="cuda", generator=g)
        B = torch.randn([2] * rb, dtype=torch.complex64, device="cuda", generator=g)
        C = torch.empty([2] * len(lc), dtype=torch.complex64, device="cuda")
        fl = 8.0 * 2.0 ** (ra + rb - k)
        # error reference for every shape: 4096 sampled output entries, each
        # a complex128 sum over its own slices of A and B (the oracle's
        # per-entry evaluation on host copies of the operands)
        Ah = A.cpu().numpy()
        Bh = B.cpu().numpy()
        idx = [tuple(int(x) for x in rng.integers(0, 2, len(lc))) for _ in range(4096)]
        ref = contract_entries(Ah, la, Bh, lb, lc, idx)
        del Ah, Bh
        check = True
        for prec in ("fp32", "bf16x3", "f16x3", "bf16x6"):
            T = _timed(lambda: tn.tn_contract_pair(A, la, B, lb, C, lc, prec), 2 if fl > 1e14 else 3)
            row = {"ranks": [ra, rb, k], "precision": prec, "seconds": T, "tflops": fl / T / 1e12}
            if check:
                Cc = C.cpu().numpy()
                got = np.array([Cc[i] for i in idx])
                rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
                row["l2_rel_err"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
                row["max_floored_err"] = float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 0.1 * rms)))
                del Cc
            rows.append(row)
            print(f"# c3 {row}", file=sys.stderr, flush=True)
            if prec == "f16x3" and (best is None or fl > best[0]):
                best = (fl, T)
        del A, B, C
        torch.cuda.empty_cache()
    tn.tn_set_workspace(None)
    # oracle: einsum (complex128) on a rank-18 pair with k = 8
    rng = np.random.default_rng(5)
    A = rng.standard_normal([2] * 18) + 1j * rng.standard_normal([2] * 18)
    B = rng.standard_normal([2] * 18) + 1j * rng.standard_normal([2] * 18)
    la = list(range(10)) + list(range(100, 108))
    lb = list(range(100, 108)) + list(range(200, 210))
    t0 = time.perf_counter()
    contract_pair(A, la, B, lb, list(range(10)) + list(range(200, 210)))
    t_cpu = time.perf_counter() - t0
    fl_cpu = 8.0 * 2.0 ** 28
    fl, T = best
    return {"metric": "complex TFLOP/s of pairwise contractions (output 2^24-2^30), per precision",
            "value": fl / T / 1e12, "unit": "TFLOP/s (f16x3, largest shape)", "dtype": "c64",
            "config": {"workload": "random pairs, extents 2, shuffled modes, seed 3", "results": rows},
            "roofline": {"bound": "mfma", "achieved": fl / T / 1e12, "peak": PEAKS["f16x3"] / 1e12,
                         "unit": "TFLOP/s", "frac": fl / T / PEAKS["f16x3"], "traffic": None},
            "cpu_baseline": {"value": fl_cpu / t_cpu / 1e12, "unit": "TFLOP/s", "cores": 1, "kind": "oracle",
                             "sample": "oracle einsum complex128, rank-18 x rank-18 pair, k = 8"}}


def bench_traj(a):
    """32 noisy 4x5-grid circuits of depths 10-30 x 32 trajectories each."""
    import paper_2104_10523_amd as tn
    from oracle import noise
    from workloads import grid_random_circuit, noisy_ops, trajectory_uniforms, count_channel_events
    circuits = []
    for c in range(32):
        n, ops = grid_random_circuit(4, 5, 10 + round(20 * c / 31), 40 + c)
        circuits.append((n, noisy_ops(ops, 1e-3, 1e-2, 5e-3)))
    tpc = 32
    ev = max(count_channel_events(o) for _, o in circuits)
    U = trajectory_uniforms(len(circuits) * tpc, ev, 4)
    tn.tn_run_trajectories(circuits, tpc, U)     # warm
    z, rep = tn.tn_run_trajectories(circuits, tpc, U)
    T = rep.seconds
    nt = len(circuits) * tpc
    # oracle: one trajectory of the shallowest (depth-10) circuit, scaled
    # by the ensemble's mean depth
    t0 = time.perf_counter()
    noise.trajectories_expect_z([circuits[0]], 1, U[:1])
    depth = [10 + round(20 * c / 31) for c in range(32)]
    t_cpu = (time.perf_counter() - t0) * np.mean(depth) / 10
    return {"metric": "noisy trajectories/s, 20 qubits, depths 10-30", "value": nt / T,
            "unit": "trajectories/s", "dtype": "c64 state, fp64 norms",
            "config": {"workload": "32 circuits (4x5 grid, CZ, depth 10..30) x 32 trajectories, "
                                   "depolarising 1e-3/1e-2, damping 5e-3", "seconds": T, "bytes": rep.bytes},
            "roofline": {"bound": "hbm", "achieved": rep.bytes / T / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                         "frac": rep.bytes / T / HBM_PEAK, "traffic": None},
            "cpu_baseline": {"value": 1.0 / t_cpu, "unit": "trajectories/s", "cores": 1, "kind": "oracle",
                             "sample": "oracle trajectory (state vector, complex128): one trajectory of the "
                                       "depth-10 circuit, scaled to the ensemble's mean depth 20"}}


def bench_pmps(a):
    """Locally-purified MPS (Sec. 3.4): 24-site noisy chain, 8 cycles of
    fSim(pi/2, pi/6) on alternating bonds, depolarising 1e-3 / 1e-2 and
    damping 5e-3 after every gate, d_max 32, k_max 8."""
    import paper_2104_10523_amd as tn
    from oracle.gates import gate_matrix, is_channel, kraus_ops
    from oracle.pmps import run_circuit as pmps_oracle
    from workloads import chain_random_circuit, noisy_ops
    n, ops = chain_random_circuit(24, 8, 9)
    ops = noisy_ops(ops, 1e-3, 1e-2, 5e-3)
    d_max, k_max = 32, 8

    def run():
        m = tn.tn_pmps_create(n, d_max, k_max)
        db = dk = 0.0
        for op in ops:
            q = op.qubits
            if is_channel(op.name):
                b, k = m.apply_channel(q[0], kraus_ops(op.name, op.params))
                db, dk = db + b, dk + k
            elif len(q) == 1:
                m.apply_gate1(q[0], gate_matrix(op.name, op.params))
            else:
                db += m.apply_gate(q[0], gate_matrix(op.name, op.params))
        return m, db, dk
    run()                                   # warm (graph captures per shape)
    t0 = time.perf_counter()
    m, db, dk = run()
    T = time.perf_counter() - t0
    z = m.expect_z()
    n_ops = sum(1 for op in ops if len(op.qubits) == 2 or is_channel(op.name))
    t1 = time.perf_counter()
    ref, rdb, rdk = pmps_oracle(n, ops, d_max=d_max, k_max=k_max)
    t_cpu = time.perf_counter() - t1
    zerr = float(np.abs(z - ref.expect_z()).max())
    return {"metric": "locally-purified MPS: two-qubit gates + channels per second, 24-site noisy chain",
            "value": n_ops / T, "unit": "ops/s", "dtype": "c64 sites, fp64 SVD/QR",
            "config": {"workload": "24-site chain, 8 cycles fSim(pi/2,pi/6), depolarising 1e-3/1e-2 + damping 5e-3, "
                                   "d_max 32, k_max 8", "seconds": T, "ops": n_ops,
                       "discarded_bond": db, "discarded_kraus": dk, "oracle_discarded_bond": rdb,
                       "oracle_discarded_kraus": rdk, "z_max_abs_diff_vs_oracle": zerr,
                       "dims": m.dims()},
            "roofline": {"bound": "latency", "achieved": None, "peak": None, "unit": None, "frac": None,
                         "traffic": None, "note": "per op: a pivoted QR to the numerical rank (<= 128) and an FP64 Jacobi SVD of R^dagger, plus QR moves"},
            "cpu_baseline": {"value": n_ops / t_cpu, "unit": "ops/s", "cores": os.cpu_count(), "kind": "oracle",
                             "sample": "PMPS oracle (numpy complex128 + LAPACK SVD/QR), the same circuit"}}


def bench_mps(a):
    """40-site chain, 20 cycles, chi_max 256: two-qubit gates per second."""
    import torch
    import paper_2104_10523_amd as tn
    from oracle.gates import gate_matrix
    from oracle.mps import MPS
    from workloads import chain_random_circuit
    n, ops = chain_random_circuit(40, 20, 5)
    chi = 256
    m = tn.tn_mps_create(n, chi)
    g2 = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for op in ops:
        U = gate_matrix(op.name, op.params)
        if len(op.qubits) == 1:
            m.apply_gate1(op.qubits[0], U)
        else:
            tn.tn_mps_apply_gate(m, op.qubits[0], U, chi, 1e-12)
            g2 += 1
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    dims = m.bond_dims()
    # oracle: the same circuit (numpy + LAPACK SVD), stopped after ~40 s
    from threadpoolctl import threadpool_info
    ref = MPS(n)
    k = 0
    t0 = time.perf_counter()
    for op in ops:
        U = gate_matrix(op.name, op.params)
        if len(op.qubits) == 1:
            ref.apply_gate1(op.qubits[0], U)
        else:
            ref.apply_gate2(op.qubits[0], U, chi)
            k += 1
            if time.perf_counter() - t0 > 40.0:
                break
    t_cpu = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    return {"metric": "MPS two-qubit gates/s, 40 sites, chi_max 256", "value": g2 / T, "unit": "gates/s",
            "dtype": "c64 sites, fp64 SVD/QR",
            "config": {"workload": "40-site chain, 20 cycles, fSim(pi/2,pi/6), chi_max 256, cutoff 1e-12",
                       "seconds": T, "two_qubit_gates": g2, "max_bond": max(dims)},
            "roofline": {"bound": "alu", "achieved": None, "peak": 78.6, "unit": "TFLOP/s",
                         "frac": None, "traffic": None,
                         "note": "latency-bound: per gate one FP64 Jacobi SVD of at most 512 x 512"},
            "cpu_baseline": {"value": k / t_cpu, "unit": "gates/s", "cores": threads, "kind": "oracle",
                             "sample": f"oracle MPS (numpy, LAPACK SVD) on the same circuit: {k} of {g2} two-qubit "
                                       f"gates in {t_cpu:.1f} s (BLAS/LAPACK threads: {threads})"}}


def _learned_corpus_teachers(m, ids, trials, states_per_circuit):
    """Teacher paths (best of `trials` randomised-greedy paths) of corpus
    circuits `ids`, sampled at about `states_per_circuit` states each into the
    model's training set; returns the number of states added."""
    import paper_2104_10523_amd as tn
    from workloads import path_search_circuit
    added = 0
    for i in ids:
        n, ops = path_search_circuit(i)
        net = tn.tn_build_network(n, ops)
        teacher = tn.tn_find_path(net, "random_greedy", trials=trials, seed=i, temperature=0.5)
        steps = len(teacher.pairs)
        stride = max(1, steps // states_per_circuit)
        m.add_teacher(net, teacher.pairs, stride=stride)
        added += len(range(0, steps - 1, stride))   # states with more than two live tensors
    return added


def _geomean_ratio(a, b):
    return float(2.0 ** np.mean(np.log2(np.asarray(a)) - np.log2(np.asarray(b))))


def bench_learned(a):
    """Learned contraction-order proposer at the path-search corpus scale:
    a.learned_train training circuits (30-60 qubits, 8-16 CZ cycles), each
    labelled by the best of 32 randomised-greedy paths and sampled at ~16
    states; a.learned_test held-out circuits searched by greedy, the learned
    scorer (greedy fallback) re-scoring after every merge and after every
    a.learned_rescore merges, the same scorer untrained, the 32-trial teacher
    and randomised greedy given the learned search's wall time.  End-to-end
    time of one amplitude (search + plan + contraction, auto precision) on
    held-out circuits whose learned and equal-time paths both stay within 2^40
    flops."""
    import torch
    import paper_2104_10523_amd as tn
    from oracle import gnn
    from workloads import path_search_circuit, random_bitstrings, scorer_init
    H, L = 128, 4
    theta0 = scorer_init(gnn.param_shapes(H, L), 11)
    m = tn.Model(H, L)
    m.set_params(theta0)
    m0 = tn.Model(H, L)
    m0.set_params(theta0)
    t0 = time.perf_counter()
    n_states = 0
    for c0 in range(0, a.learned_train, 500):
        n_states += _learned_corpus_teachers(m, range(c0, min(a.learned_train, c0 + 500)), 32, 16)
        print(f"# learned: {min(a.learned_train, c0 + 500)} teacher paths, {n_states} states, "
              f"{time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
    t_label = time.perf_counter() - t0
    t0 = time.perf_counter()
    first, last = m.train(epochs=a.learned_epochs, batch=a.learned_batch, lr=a.learned_lr, seed=3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    steps = a.learned_epochs * -(-n_states // a.learned_batch)
    print(f"# learned: trained {steps} steps in {t_train:.1f} s, loss {first:.3f} -> {last:.3f}",
          file=sys.stderr, flush=True)

    def timed_path(fn):
        t = time.perf_counter()
        p = fn()
        return p, time.perf_counter() - t

    rows = []
    for i in range(5000, 5000 + a.learned_test):
        n, ops = path_search_circuit(i)
        net = tn.tn_build_network(n, ops)
        g, tg = timed_path(lambda: tn.tn_find_path(net, "greedy"))
        lp, tl = timed_path(lambda: tn.tn_find_path_learned(net, m))
        l0 = tn.tn_find_path_learned(net, m0)
        lr, tlr = timed_path(lambda: tn.tn_find_path_learned(net, m, rescore_every=a.learned_rescore))
        r32, tr = timed_path(lambda: tn.tn_find_path(net, "random_greedy", trials=32, seed=i, temperature=0.5))
        eq = max(1, int(round(32 * tl / tr)))
        req, te = timed_path(lambda: tn.tn_find_path(net, "random_greedy", trials=eq, seed=i, temperature=0.5))
        rows.append(dict(i=i, n=n, greedy=g.cost.flops_per_slice, learned=lp.cost.flops_per_slice,
                         untrained=l0.cost.flops_per_slice, teacher=r32.cost.flops_per_slice,
                         learned_r=lr.cost.flops_per_slice, t_learned_r=tlr,
                         equal_time=req.cost.flops_per_slice, chosen=lp.cost.algo_used == 2,
                         t_greedy=tg, t_learned=tl, t_teacher=tr, t_equal=te, eq_trials=eq,
                         pairs_learned=lp.pairs, pairs_equal=req.pairs))
        if len(rows) % 50 == 0:
            print(f"# learned: {len(rows)} held-out circuits searched", file=sys.stderr, flush=True)
    col = {k: np.array([r[k] for r in rows]) for k in rows[0] if not k.startswith("pairs")}

    # end-to-end amplitude time: search + plan + contraction of one amplitude
    ws = torch.empty(64 << 30, dtype=torch.uint8, device="cuda")
    tn.tn_set_workspace(ws)
    e2e = []
    for r in rows:
        if max(r["learned"], r["equal_time"]) > 2.0 ** 40:
            continue
        n, ops = path_search_circuit(r["i"])
        net = tn.tn_build_network(n, ops)
        bits = random_bitstrings(1, n, r["i"])
        rec = {"i": r["i"], "n": n}
        for name, pairs, ts in (("learned", r["pairs_learned"], r["t_learned"]),
                                ("equal_time", r["pairs_equal"], r["t_equal"])):
            t = time.perf_counter()
            p = tn.tn_path_from_pairs(net, pairs, mem_budget_bytes=16.0 * 2 ** 30)
            if tn.tn_amplitudes_workspace(net, p, 1, "auto") > ws.numel():
                rec = None
                break
            out, rep = tn.tn_amplitudes(net, p, bits, precision="auto")
            rec[name] = ts + time.perf_counter() - t
            rec[name + "_amp"] = complex(out.cpu().numpy()[0, 0])
        if rec is not None:
            e2e.append(rec)
    del ws
    torch.cuda.empty_cache()
    amp_diff = max((abs(x["learned_amp"] - x["equal_time_amp"]) / max(abs(x["equal_time_amp"]), 2.0 ** (-x["n"] / 2))
                    for x in e2e), default=None)
    gains = np.log2(col["greedy"] / col["learned"])
    res = {
        "metric": "learned path: mean log2 flop gain over greedy on held-out circuits",
        "value": float(np.mean(gains)), "unit": "log2", "higher_is_better": True, "dtype": "fp32 training",
        "config": {"workload": f"path-search corpus: {a.learned_train} training / {a.learned_test} held-out "
                               f"circuits, 30-60 qubits, 8-16 CZ cycles",
                   "scorer": f"H={H}, L={L}, {m.n_params} parameters", "states": n_states,
                   "teacher_seconds": t_label, "train_seconds": t_train, "train_steps": steps,
                   "train_steps_per_s": steps / t_train, "epochs": a.learned_epochs, "batch": a.learned_batch,
                   "loss_first": first, "loss_last": last},
        "held_out": {
            "learned_chosen_fraction": float(np.mean(col["chosen"])),
            "geomean_flops_learned_over_greedy": _geomean_ratio(col["learned"], col["greedy"]),
            "geomean_flops_untrained_over_greedy": _geomean_ratio(col["untrained"], col["greedy"]),
            "geomean_flops_learned_over_teacher32": _geomean_ratio(col["learned"], col["teacher"]),
            "geomean_flops_learned_over_equal_time": _geomean_ratio(col["learned"], col["equal_time"]),
            "learned_beats_equal_time_fraction": float(np.mean(col["learned"] < col["equal_time"])),
            "median_search_seconds": {k: float(np.median(col["t_" + k]))
                                      for k in ("greedy", "learned", "learned_r", "teacher", "equal")},
            "rescore_every": a.learned_rescore,
            "geomean_flops_learned_r_over_greedy": _geomean_ratio(col["learned_r"], col["greedy"]),
            "geomean_flops_learned_r_over_learned": _geomean_ratio(col["learned_r"], col["learned"]),
            "median_equal_time_trials": float(np.median(col["eq_trials"])),
            "log2_gain_over_greedy_quartiles": [float(x) for x in np.percentile(gains, [25, 50, 75])]},
        "end_to_end": {
            "circuits": len(e2e),
            "median_seconds_learned": float(np.median([x["learned"] for x in e2e])) if e2e else None,
            "median_seconds_equal_time": float(np.median([x["equal_time"] for x in e2e])) if e2e else None,
            "total_seconds_learned": float(sum(x["learned"] for x in e2e)),
            "total_seconds_equal_time": float(sum(x["equal_time"] for x in e2e)),
            "max_floored_amplitude_difference": amp_diff},
        "roofline": None, "cpu_baseline": None}
    return res


def bench_expval(a):
    """Pauli expectation values (Eq. 2, Table 1).  Conjugate network: <Z Z>
    on two central qubits of a 7x7 grid, 10 fSim cycles, after the light-cone
    collapse, every slice of the double-depth network timed with per-op
    events; FP32 beside it for the error.  Wave-function slicing: the same
    observable on a 5x5 grid, 10 cycles, 20 open qubits (32 slices),
    checked against the conjugate method on that circuit."""
    import itertools
    import torch
    import paper_2104_10523_amd as tn
    from workloads import grid_random_circuit
    stream = torch.cuda.current_stream()
    n, ops = grid_random_circuit(7, 7, 10, 2, two_qubit="fsim")
    codes = [0] * n
    codes[24] = codes[25] = 3
    net, kept = tn.tn_build_expectation_network(n, ops, codes)
    t0 = time.time()
    path = tn.tn_find_path(net, "partition", trials=1024, seed=1, mem_budget_bytes=160 * 2 ** 30)
    t_path = time.time() - t0
    ns = int(path.cost.n_slices)
    need = max(tn.tn_amplitudes_workspace(net, path, 1, p) for p in ("fp32", a.precision))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    tn.tn_set_workspace(ws)
    zeros = np.zeros((1, n), np.int8)
    print(f"# expval: kept {kept} of {len(ops)} gates, 2^{path.cost.n_sliced} slices, total flops "
          f"2^{math.log2(path.cost.total_flops):.2f}, path {t_path:.1f}s", file=sys.stderr, flush=True)
    time_steps(net, path, zeros, a.precision, [(0, 0)], stream)          # warm-up: one slice
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per_job, op_sec, (info, kind, fl, by, shape), parts = time_steps(net, path, zeros, a.precision,
                                                                      [(0, s) for s in range(ns)], stream)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    value = complex(parts.sum())
    _, _, _, parts32 = time_steps(net, path, zeros, "fp32", [(0, s) for s in range(ns)], stream)
    v32 = complex(parts32.sum())
    names = {}
    for k in np.nonzero(kind == 2)[0]:
        names.setdefault(kernel_name(a.precision, int(shape[k, 4]), int(shape[k, 5])), []).append(k)
    dom = max(names, key=lambda nm: op_sec[names[nm]].sum())
    sel = np.array(names[dom])
    g_flops = float(fl[sel].sum()) * ns
    g_time = float(op_sec[sel].sum())
    n_launch = int(shape[sel, 6].sum()) * ns
    peak = PEAKS[a.precision] if a.precision in PEAKS else PEAKS["bf16x3"]
    flops_total = float(fl.sum()) * ns
    # wave-function slicing on a 5x5 grid
    n5, ops5 = grid_random_circuit(5, 5, 10, 3, two_qubit="fsim")
    c5 = [0] * n5
    c5[12] = c5[13] = 3
    proj = list(range(5))
    bits = np.full((32, n5), -1, np.int8)
    for sidx, vals in enumerate(itertools.product((0, 1), repeat=5)):
        bits[sidx, proj] = vals
    net5 = tn.tn_build_network(n5, ops5)
    path5 = tn.tn_find_path(net5, "random_greedy", trials=64, seed=1, open_mask=(bits[0] < 0).astype(np.int8))
    tn.tn_set_workspace(None)
    del ws
    torch.cuda.empty_cache()
    ws5 = torch.empty(tn.tn_amplitudes_workspace(net5, path5, 32, a.precision), dtype=torch.uint8, device="cuda")
    tn.tn_set_workspace(ws5)

    def sliced():
        psi, _ = tn.tn_amplitudes(net5, path5, bits, precision=a.precision)
        return tn.tn_pauli_expectation(psi, bits, c5)
    v5 = sliced()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    v5 = sliced()
    t5 = time.perf_counter() - t0
    netc5, kept5 = tn.tn_build_expectation_network(n5, ops5, c5)
    pc5 = tn.tn_find_path(netc5, "random_greedy", trials=64, seed=1)
    tn.tn_set_workspace(torch.empty(tn.tn_amplitudes_workspace(netc5, pc5, 1, "fp32"), dtype=torch.uint8,
                                    device="cuda"))
    vc5 = complex(tn.tn_amplitudes(netc5, pc5, np.zeros((1, n5), np.int8), precision="fp32")[0].cpu().numpy()[0, 0])
    cpu = None
    if not a.no_cpu:
        leaves = []
        outs = set(net.output_labels())
        for i in range(net.info().n_tensors):
            _, ls = net.tensor(i)
            leaves.append([l for l in ls if l not in outs])
        rate, secs, f = cpu_baseline(path.pairs, (leaves, [2] * net.info().n_labels, set(), path.sliced),
                                     a.cpu_seconds)
        cpu = {"value": rate / flops_total, "unit": "expectation values/s", "cores": blas_threads(), "kind": "oracle",
               "sample": f"oracle complex128 pairwise contractions (batched matmul, all BLAS threads) on the "
                         f"double-depth network's largest pairwise contractions "
                         f"with <= 2^25-entry tensors ({f:.3g} flops in {secs:.1f}s, {rate / 1e9:.2f} GFLOP/s), "
                         f"extrapolated to {flops_total:.3g} flops"}
    return {"metric": "Pauli expectation values/s, <Z24 Z25> on a 49-qubit depth-10 grid (conjugate network)",
            "value": 1.0 / T, "unit": "expectation values/s", "dtype": f"{a.precision} c64, fp64 slice sum",
            "config": {"workload": "7x7 grid, 10 cycles, fSim(pi/2,pi/6), seed 2; double-depth network after "
                                   "light-cone collapse; recursive-bisection path (1024 trials), 160 GiB budget",
                       "path_search_seconds": t_path,
                       "kept_gates": kept, "gates": len(ops), "slices": ns, "seconds": T,
                       "flops": flops_total, "complex_tflops": flops_total / T / 1e12,
                       "value": [value.real, value.imag], "fp32_value": [v32.real, v32.imag],
                       "abs_diff_vs_fp32": abs(value - v32),
                       "sliced_method": {"workload": "5x5 grid, 10 cycles, fSim, seed 3, <Z12 Z13>, 20 open qubits, "
                                                     "32 slices", "seconds": t5, "value": [v5.real, v5.imag],
                                         "conjugate_fp32_value": [vc5.real, vc5.imag],
                                         "abs_diff": abs(v5 - vc5)}},
            "roofline": {"bound": "mfma", "achieved": g_flops / g_time / 1e12, "peak": peak / 1e12,
                         "unit": "TFLOP/s", "frac": g_flops / g_time / peak, "traffic": None, "kernel": dom,
                         "launches": n_launch, "avg_launch_ms": 1e3 * g_time / max(1, n_launch)},
            "cpu_baseline": cpu}


def bench_dm(a):
    """Exact noisy <Z_q> from density-matrix networks (Sec. 3.3, Eq. 3): the
    depth-10 circuit of the trajectory ensemble (4x5 grid, CZ, depolarising
    1e-3/1e-2, damping 5e-3), all 20 qubits, each its own network after
    light-cone pruning; 1024 trajectories of the same circuit beside them."""
    import torch
    import paper_2104_10523_amd as tn
    from oracle import noise
    from workloads import grid_random_circuit, noisy_ops, trajectory_uniforms, count_channel_events
    n, ops = grid_random_circuit(4, 5, 10, 40)
    ops = noisy_ops(ops, 1e-3, 1e-2, 5e-3)
    plans = []
    t0 = time.time()
    for q in range(n):
        codes = [0] * n
        codes[q] = 3
        net, kept = tn.tn_build_density_network(n, ops, codes)
        path = tn.tn_find_path(net, "random_greedy", trials=64, seed=1, mem_budget_bytes=160 * 2 ** 30)
        plans.append((net, path, kept))
    t_plan = time.time() - t0
    need = max(tn.tn_amplitudes_workspace(net, path, 1, "fp32") for net, path, _ in plans)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    tn.tn_set_workspace(ws)
    empty = np.zeros((1, 0), np.int8)

    def run():
        vals, flops = [], 0.0
        for net, path, _ in plans:
            out, rep = tn.tn_amplitudes(net, path, empty, precision="fp32")
            vals.append(out.cpu().numpy()[0, 0].real)
            flops += rep.flops
        return np.array(vals), flops
    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    z_exact, flops = run()
    T = time.perf_counter() - t0
    U = trajectory_uniforms(1024, count_channel_events(ops), 4)
    z_traj, _ = tn.tn_run_trajectories([(n, ops)], 1024, U)
    se = z_traj.std(axis=0) / math.sqrt(1024)
    dev = np.abs(z_traj.mean(axis=0) - z_exact) / np.maximum(se, 1e-12)
    cpu = None
    if not a.no_cpu:
        # the 20-qubit density matrix (2^40 entries) is out of the oracle's
        # reach: it is timed on a 3x3 grid of the same family, per value
        n9, ops9 = grid_random_circuit(3, 3, 10, 40)
        ops9 = noisy_ops(ops9, 1e-3, 1e-2, 5e-3)
        t0 = time.perf_counter()
        rho = noise.dm_simulate(n9, ops9)
        noise.dm_expect_z(rho, n9)
        t9 = time.perf_counter() - t0
        cpu = {"value": n9 / t9, "unit": "expectation values/s", "cores": 1, "kind": "oracle",
               "sample": f"density-matrix oracle (complex128, 4^9 entries) on a 3x3 grid, depth 10, same noise: "
                         f"all 9 <Z_q> in {t9:.1f} s; the 20-qubit rho (2^40 entries) is out of its reach"}
    return {"metric": "exact noisy <Z_q> per second, 20-qubit depth-10 grid (density-matrix networks)",
            "value": n / T, "unit": "expectation values/s", "dtype": "c64 fp32, fp64 accumulate",
            "config": {"workload": "4x5 grid, 10 cycles, CZ, seed 40, depolarising 1e-3/1e-2, damping 5e-3; "
                                   "one density-matrix network per qubit after light-cone pruning; "
                                   "randomised-greedy paths (64 trials)",
                       "seconds": T, "flops": flops, "plan_seconds": t_plan,
                       "kept_ops": [k for _, _, k in plans], "ops": len(ops),
                       "z_exact": z_exact.tolist(),
                       "trajectories_1024_max_dev_in_se": float(dev.max())},
            "roofline": {"bound": "latency", "achieved": None, "peak": None, "unit": None, "frac": None,
                         "traffic": None, "note": f"{flops / T / 1e12:.3f} complex TFLOP/s; ~100 small "
                                                  f"contractions per value"},
            "cpu_baseline": cpu}


def run_graph(net, path, bits, slice_id, precision):
    """All rows of `bits` at one slice in one tn_amplitudes call: the job's
    kernel sequence is captured once as a hipGraph and replayed per job.
    Returns (amplitudes, device seconds)."""
    import torch
    import paper_2104_10523_amd as tn
    bits = np.ascontiguousarray(bits)
    out = torch.zeros((len(bits), 1), dtype=torch.complex128, device="cuda")
    _, rep = tn.tn_amplitudes(net, path, bits, out=out, precision=precision, use_graph=True,
                              slice_begin=slice_id, slice_count=1, sync=True)
    if rep.nonfinite:
        raise RuntimeError("non-finite amplitude")
    return out.cpu().numpy()[:, 0], rep.seconds


def op_kernel_name(precision, k, sh):
    """The kernel an op of the plan launches (rocprofv3's name, without
    arguments)."""
    if k == 2:
        return kernel_name(precision, int(sh[4]), int(sh[5]))
    if k == 0:
        if int(sh[3]) == 2:
            return f"apply16_mfma_kernel<{int(sh[2])}, {max(1, int(sh[1]) // 16)}>"
        return f"{'apply_tile_kernel' if sh[3] else 'apply_small_kernel'}<{int(sh[1])}>"
    if k == 3:
        return f"skinny_partial_kernel<{int(sh[0])}, {int(sh[1])}>" if sh[5] else "dot_partial_kernel"
    np_ = 4 if sh[2] else int(sh[1])
    return {0: "device copy", 1: f"permute_simple_kernel<{np_}>", 2: f"permute_tiled_kernel<{np_}>",
            3: "maxabs_kernel", 4: f"permute_pipe_kernel<{np_}>"}[int(sh[3])]


def kernel_table(precision, kind, fl, by, shape, op_sec, jobs):
    """Per kernel: seconds, launches, algorithmic flops and bytes over `jobs`
    profiled jobs."""
    out = {}
    for k in range(len(kind)):
        nm = op_kernel_name(precision, int(kind[k]), shape[k])
        e = out.setdefault(nm, {"seconds": 0.0, "launches": 0, "flops": 0.0, "bytes": 0.0})
        e["seconds"] += float(op_sec[k])
        e["launches"] += int(shape[k, 6]) * jobs
        e["flops"] += float(fl[k]) * jobs
        e["bytes"] += float(by[k]) * jobs
    return out


def roofline_entry(kernel, flops, bytes_, seconds, precision):
    """Roofline of one launch: a GEMM whose algorithmic intensity reaches the
    balance point of its own arithmetic (split products: 3 or 6 MFMA
    products per multiply-add, so the ridge sits at peak / 3 or / 6 over HBM
    bandwidth) is priced against its dtype's MFMA peak; everything else
    against HBM bandwidth."""
    if kernel.startswith("gemm"):
        if kernel.startswith("gemm_mfma_kernel") and kernel.endswith(", 0>"):      # FP32 MFMA
            peak, eff = PEAKS["fp32"], PEAKS["fp32"]
        elif kernel.startswith("gemm_mfma_kernel"):                              # split in LDS
            peak = 2.5e15
            eff = peak / (6 if kernel.endswith(", 2>") else 3)
        else:                                                                    # packed planes
            np_ = 3 if kernel.endswith(", 3, false>") else 2
            peak = 2.5e15
            eff = peak / (6 if np_ == 3 else 3)
        if bytes_ > 0 and flops / bytes_ >= eff / HBM_PEAK:
            return {"bound": "mfma", "achieved": flops / seconds / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                    "frac": flops / seconds / peak, "algorithmic_peak": eff / 1e12,
                    "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": bytes_}
    return {"bound": "hbm", "achieved": bytes_ / seconds / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": bytes_ / seconds / HBM_PEAK, "algorithmic_flops_per_launch": flops,
            "algorithmic_bytes_per_launch": bytes_}


ROWS = {"c1": bench_c1, "c3": bench_c3, "traj": bench_traj, "mps": bench_mps, "pmps": bench_pmps,
        "learned": bench_learned,
        "expval": bench_expval, "dm": bench_dm}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (one slice job at a time on its HBM); --gpus must be 1"}))
        sys.exit(2)
    import torch
    import paper_2104_10523_amd as tn
    torch.cuda.set_device(0)
    if a.workload != "c2":
        print(json.dumps(ROWS[a.workload](a)), flush=True)
        return
    stream = torch.cuda.current_stream()
    if a.calib_copy:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    n, ops, bits, net, path, t_path = make_workload(a)
    ns = path.cost.n_slices
    need = max(tn.tn_amplitudes_workspace(net, path, max(a.steps, a.warmup, 1), p) for p in ("fp32", a.precision))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    tn.tn_set_workspace(ws)
    t0 = time.time()
    if a.autotune:
        for p in {a.precision, "fp32"}:
            tn.tn_amplitudes_autotune(net, path, p, reps=2)
    t_tune = time.time() - t0
    rng = np.random.default_rng(7)
    slice_warm, slice_timed, slice_prof = (int(x) for x in rng.integers(0, int(ns), 3))
    rows = rng.permutation(64)
    print(f"# workload {a.rows}x{a.cols}x{a.cycles} fSim: slices 2^{path.cost.n_sliced}, per-slice flops "
          f"2^{math.log2(path.cost.flops_per_slice):.2f}, workspace {need / 2**30:.1f} GiB, path search "
          f"{t_path:.1f}s, autotune {t_tune:.1f}s", file=sys.stderr, flush=True)
    # warmup, then the timed region: one tn_amplitudes call per region whose
    # (bit-string, slice) jobs replay one captured hipGraph of the job's
    # kernel sequence (the production path)
    if a.warmup:
        run_graph(net, path, bits[rows[:a.warmup]], slice_warm, a.precision)
    print("# warmup done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    amps, dev_s = run_graph(net, path, bits[rows[a.warmup:a.warmup + a.steps]], slice_timed, a.precision)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    T = wall / a.steps
    amps_per_s = 1.0 / (ns * T)
    # profiled pass (after the timed region): HIP events around every op
    prof_jobs = [(int(rows[(a.warmup + a.steps + j) % 64]), slice_prof) for j in range(a.profile_steps)]
    _, op_sec, (info, kind, fl, by, shape), _ = time_steps(net, path, bits, a.precision, prof_jobs, stream)
    P = max(1, a.profile_steps)
    flops_job = float(fl.sum())
    kern = kernel_table(a.precision, kind, fl, by, shape, op_sec, P)
    dom = max(kern, key=lambda k: kern[k]["seconds"])
    d = kern[dom]
    step_kernel_s = sum(v["seconds"] for v in kern.values()) / P
    traffic, traffic_src = recorded_traffic(dom)
    avg_s = d["seconds"] / d["launches"]
    fl_launch, by_launch = d["flops"] / d["launches"], d["bytes"] / d["launches"]
    roof = roofline_entry(dom, fl_launch, by_launch, avg_s, a.precision)
    t_by_kind = {k: float(op_sec[kind == i].sum()) / P for i, k in enumerate(("apply", "permute", "gemm", "dot"))}
    print(f"# per step {T:.3f}s (graph replays; device {dev_s / a.steps:.3f}s); profiled step {step_kernel_s:.3f}s "
          f"by kind {t_by_kind}; dominant {dom} {100 * d['seconds'] / P / step_kernel_s:.1f}%",
          file=sys.stderr, flush=True)
    fp32 = None
    if a.compare_fp32 and a.precision != "fp32":
        k32 = 2
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        a32, _ = run_graph(net, path, bits[rows[a.warmup:a.warmup + k32]], slice_timed, "fp32")
        torch.cuda.synchronize()
        T32 = (time.perf_counter() - t1) / k32
        fp32 = {"seconds_per_step": T32, "amplitudes_per_s": 1.0 / (ns * T32), "speedup_of_split": T32 / T,
                # same (bit-string, slice) jobs as the first timed ones
                "slice_amplitude_rel_diff": float(np.max(np.abs(amps[:k32] - a32) / np.maximum(np.abs(a32), 1e-300))),
                # floor: the RMS amplitude of one slice of a normalised state
                "slice_amplitude_floored_diff": float(np.max(np.abs(amps[:k32] - a32) /
                                                             np.maximum(np.abs(a32), 2.0 ** (-(n + path.cost.n_sliced) / 2)))),
                "slice_amplitude_over_floor": float(np.min(np.abs(a32)) / 2.0 ** (-(n + path.cost.n_sliced) / 2))}
        print(f"# fp32 step {T32:.3f}s", file=sys.stderr, flush=True)
    val = None
    if a.validate > 0:
        # jobs on distinct random slices: benchmark precision and FP32 first,
        # then the timing workspace is released for the FP64 one (2x larger)
        vjobs = [(int(rows[j % 64]), int(x)) for j, x in
                 enumerate(rng.choice(int(ns), size=min(a.validate, int(ns)), replace=False))]
        va = np.array([run_graph(net, path, bits[[b]], sl, a.precision)[0][0] for b, sl in vjobs])
        v32 = np.array([run_graph(net, path, bits[[b]], sl, "fp32")[0][0] for b, sl in vjobs])
        tn.tn_set_workspace(None)
        del ws
        torch.cuda.empty_cache()
        # FP64 needs twice the workspace; where that does not fit, the same
        # pairs sliced to a smaller budget (sliced labels a superset of the
        # benchmark's) and the slice summed over the finer slices that agree
        # with it on the benchmark's sliced labels (first label = most
        # significant bit of a slice index)
        free = torch.cuda.mem_get_info()[0]
        vpath, budget = path, a.budget_gib * 2 ** 30
        while tn.tn_amplitudes_workspace(net, vpath, 1, "fp64") > 0.9 * free:
            budget /= 2
            vpath = tn.tn_path_from_pairs(net, path.pairs, mem_budget_bytes=budget)
            if not set(path.sliced) <= set(vpath.sliced):
                raise RuntimeError("finer slicing for the FP64 validation does not refine the benchmark's")
        S, S2 = list(path.sliced), list(vpath.sliced)

        def fine_slices(sl):
            want = {l: (sl >> (len(S) - 1 - i)) & 1 for i, l in enumerate(S)}
            return [t for t in range(1 << len(S2))
                    if all(((t >> (len(S2) - 1 - i)) & 1) == want[l] for i, l in enumerate(S2) if l in want)]

        need64 = tn.tn_amplitudes_workspace(net, vpath, 1, "fp64")
        ws = torch.empty(need64, dtype=torch.uint8, device="cuda")
        tn.tn_set_workspace(ws)
        t64 = time.perf_counter()
        v64 = []
        for b, sl in vjobs:
            v64.append(sum(run_graph(net, vpath, bits[[b]], t, "fp64")[0][0] for t in fine_slices(sl)))
            print(f"# fp64 job (bit-string {b}, slice {sl}) done", file=sys.stderr, flush=True)
        v64 = np.array(v64)
        t64 = (time.perf_counter() - t64) / len(vjobs)
        floor = 2.0 ** (-(n + path.cost.n_sliced) / 2)
        den = np.maximum(np.abs(v64), floor)
        val = {"jobs": [[b, sl] for b, sl in vjobs], "floor": floor,
               "amplitude_over_floor": [float(x) for x in np.abs(v64) / floor],
               f"{a.precision}_floored_err": [float(x) for x in np.abs(va - v64) / den],
               "fp32_floored_err": [float(x) for x in np.abs(v32 - v64) / den],
               f"{a.precision}_max": float(np.max(np.abs(va - v64) / den)),
               "fp32_max": float(np.max(np.abs(v32 - v64) / den)),
               "fp64_seconds_per_job": t64, "fp64_workspace_gib": need64 / 2 ** 30,
               "fp64_slices_per_job": 2 ** (len(S2) - len(S))}
        print(f"# fp64 validation: {a.precision} max {val[a.precision + '_max']:.2e}, fp32 max {val['fp32_max']:.2e} "
              f"({t64:.2f} s per fp64 job)", file=sys.stderr, flush=True)
    cpu = None
    if not a.no_cpu:
        from oracle.network import build_network
        onet = build_network(n, ops)
        outs = set(onet.out_label)
        leaves = [[l for l in ls if l not in outs] for ls in onet.labels]
        rate, secs, f = cpu_baseline(path.pairs, (leaves, onet.extents(), set(), path.sliced), a.cpu_seconds)
        cpu = {"value": 1.0 / (ns * flops_job / rate), "unit": "amplitudes/s", "cores": blas_threads(), "kind": "oracle",
               "sample": f"oracle complex128 pairwise contractions (batched matmul, all BLAS threads) on this "
                         f"workload's largest pairwise contractions with "
                         f"<= 2^25-entry tensors ({f:.3g} flops in {secs:.1f}s, {rate / 1e9:.2f} GFLOP/s), "
                         f"extrapolated to {flops_job:.3g} flops per step x 2^{path.cost.n_sliced} slices"}
    line = {
        "metric": "amplitudes/s + complex TFLOP/s, 49q depth-14 grid; split-BF16 vs FP32 @1e-5 err",
        "value": amps_per_s,
        "unit": "amplitudes/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": T * 1e3,
        "device_ms_per_step": dev_s / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16x3": "bf16x3-split c64, fp32 accumulate", "bf16x6": "bf16x6-split c64, fp32 accumulate",
                  "f16x3": "scaled f16x3-split c64, fp32 accumulate",
                  "fp32": "c64 fp32",
                  "auto": "c64: scaled f16x3-split MFMA for large GEMMs, fp32 MFMA otherwise, "
                          "fp32 accumulate"}[a.precision],
        "data": "synthetic",
        "config": {"workload": f"{a.rows}x{a.cols} grid random circuit, {a.cycles} cycles, fSim(pi/2,pi/6), "
                               f"64 bit-strings, {'recursive-bisection' if a.path == 'partition' else 'randomised-greedy'} "
                               f"path ({a.trials} trials, ranked by {a.rank if a.path == 'partition' else 'flops'}), "
                               f"2^{path.cost.n_sliced} slices ({a.budget_gib:g} GiB budget); value extrapolated "
                               f"from timed (bit-string, slice) jobs",
                   "qubits": n, "bitstrings": 64, "slices": ns, "path_search_seconds": t_path,
                   "autotune_seconds": t_tune,
                   "flops_per_step": flops_job, "flops_per_amplitude": flops_job * ns,
                   "bytes_per_step": float(by.sum()),
                   "complex_tflops": flops_job / T / 1e12, "hbm_tbs": float(by.sum()) / T / 1e12,
                   "precision": a.precision},
        "roofline": {**roof, "traffic": traffic,
                     "traffic_unit": "bytes/launch", "traffic_source": traffic_src,
                     "kernel": dom,
                     "launches": d["launches"],
                     "avg_launch_ms": 1e3 * avg_s,
                     "share_of_step": d["seconds"] / P / step_kernel_s,
                     "step_seconds_by_kind": t_by_kind,
                     "kernels": {k: {"share": v["seconds"] / P / step_kernel_s,
                                     "avg_launch_ms": 1e3 * v["seconds"] / v["launches"],
                                     "gbs": v["bytes"] / v["seconds"] / 1e9 if v["seconds"] > 0 else 0.0}
                                 for k, v in sorted(kern.items(), key=lambda kv: -kv[1]["seconds"])[:8]},
                     "note": "kernel = the kernel with the largest share of a step (HIP events around every "
                             "op of the profiled jobs that follow the timed graph replays)"},
        "fp32_comparison": fp32,
        "fp64_validation": val,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
