"""Writes tests/golden/c2_slices.json: slices of the 49-qubit 7x7 grid
circuit of 14 fSim(pi/2, pi/6) cycles (seed 2), each contracted by the
oracle alone (complex128, pairwise along a path, each pair one batched
matrix product: oracle.contract.contract_pair_mm), as the reference for the
GPU's full-circuit slice amplitudes.

Definition of a slice (Eq. 1 with the sliced labels fixed, Sec. 3.1): the
output legs are projected onto a bit-string, the sliced labels are fixed to
the bits of the slice index (the first sliced label is the most significant
bit) and the rest of the network is contracted.  The path and the sliced
labels come from the oracle's own planner: the best of greedy and 16
reconfigured recursive-bisection trees (seed 1) by flops, sliced to a 4 GiB
complex64 live set (18 labels, 2^38.8 flops per slice).

Run from the repository root (about 6 minutes on 8 host cores, 8 GB of memory):
    python tests/golden/make_c2_slices.py
"""

import hashlib
import json
import math
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

from oracle.contract import contract_pair_mm, contract_path  # noqa: E402
from oracle.network import build_network, fix_labels, fix_outputs  # noqa: E402
from oracle.paths import partition_search, path_stats, slice_path  # noqa: E402
from workloads import grid_random_circuit, random_bitstrings  # noqa: E402

BUDGET_GIB = 4.0
TRIALS, SEED = 16, 1
# (bit-string index among the 64 benchmark bit-strings, slice index)
JOBS = [(0, 91233), (21, 5), (58, 262143)]


def pairs_sha256(pairs) -> str:
    return hashlib.sha256(json.dumps([list(map(int, p)) for p in pairs]).encode()).hexdigest()


def main():
    n, ops = grid_random_circuit(7, 7, 14, 2, two_qubit="fsim")
    net = build_network(n, ops)
    outs = set(net.out_label)
    leaves = [[l for l in ls if l not in outs] for ls in net.labels]
    ext = net.extents()
    t0 = time.time()
    pairs = partition_search(leaves, ext, (), seed=SEED, trials=TRIALS, budget_bytes=0.0)
    sliced = slice_path(leaves, ext, pairs, (), BUDGET_GIB * 2.0 ** 30)
    st = path_stats(leaves, ext, pairs, (), sliced)
    print(f"path: {time.time() - t0:.0f} s, {len(sliced)} sliced labels, 2^{math.log2(st['flops']):.2f} flops "
          f"per slice", flush=True)
    bits_all = random_bitstrings(64, n, 12345)
    jobs = []
    for b, s in JOBS:
        t = time.time()
        bits = [int(x) for x in bits_all[b]]
        tensors, labels, open_labels = fix_outputs(net, bits)
        fixed = {l: (s >> (len(sliced) - 1 - i)) & 1 for i, l in enumerate(sliced)}
        tensors, labels = fix_labels(tensors, labels, fixed)
        val = complex(contract_path(tensors, labels, pairs, open_labels, pair=contract_pair_mm))
        print(f"bit-string {b}, slice {s}: {val:.10e} ({time.time() - t:.0f} s)", flush=True)
        jobs.append({"bitstring_index": b, "bits": bits, "slice": s, "value": [val.real, val.imag]})
    out = {
        "circuit": "7x7 grid, 14 cycles, fSim(pi/2, pi/6) couplers, seed 2 (workloads.grid_random_circuit)",
        "bitstrings": "workloads.random_bitstrings(64, 49, 12345)",
        "path": {"algorithm": "partition", "trials": TRIALS, "seed": SEED, "mem_budget_bytes": 0.0,
                 "pairs_sha256": pairs_sha256(pairs)},
        "slice_budget_bytes": BUDGET_GIB * 2.0 ** 30,
        "sliced": [int(l) for l in sliced],
        "log2_flops_per_slice": math.log2(st["flops"]),
        "jobs": jobs,
        "written_by": "python tests/golden/make_c2_slices.py (oracle only, complex128)",
    }
    (ROOT / "tests" / "golden" / "c2_slices.json").write_text(json.dumps(out, indent=1) + "\n")
    print("wrote tests/golden/c2_slices.json")


if __name__ == "__main__":
    main()
