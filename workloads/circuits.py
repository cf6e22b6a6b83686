"""Seeded circuit generators.

A circuit is ``(n_qubits, ops)`` where each op is ``Op(name, qubits,
params)``.  Names, not matrices, are generated here; each side (oracle and
native library) builds the matrix of a name on its own.

Gate names
    one qubit : sqrt_x, sqrt_y, sqrt_w, h, x, y, z, s, t, rz(phi)
    two qubit : cz, cx (control = first qubit), fsim(theta, phi),
                cphase(phi) (phase on |11>), swap
Channel names (noise, inserted by :func:`noisy_ops`)
    depol1(p), depol2(p), amp_damp(gamma)

Grid conventions (random circuits of the kind used for the paper's
single-amplitude benchmark, Sec. 4.3):

* qubit ``q = r * cols + c`` on an R x C grid; qubit 0 is the most
  significant bit of a flat amplitude index;
* a cycle is one layer of single-qubit gates on every qubit followed by one
  layer of two-qubit gates; there is no trailing single-qubit layer;
* single-qubit gates come from {sqrt_x, sqrt_y, sqrt_w}; in cycle 0 one of
  the three is drawn uniformly, later one of the two that differ from the
  qubit's previous gate;
* coupler patterns A, B, C, D are used in cycle t as [A, B, C, D][t % 4]:
  A = horizontal pairs (r,c)-(r,c+1) with c even, B = horizontal with c odd,
  C = vertical pairs (r,c)-(r+1,c) with r even, D = vertical with r odd.
"""

from __future__ import annotations

import math
from typing import List, NamedTuple, Sequence, Tuple

import numpy as np

ONE_QUBIT_SET = ("sqrt_x", "sqrt_y", "sqrt_w")


class Op(NamedTuple):
    name: str
    qubits: Tuple[int, ...]
    params: Tuple[float, ...] = ()


def _single_layer(rng: np.random.Generator, n: int, prev: List[int], first: bool) -> List[Op]:
    ops = []
    for q in range(n):
        if first:
            g = int(rng.integers(0, 3))
        else:
            choices = [i for i in range(3) if i != prev[q]]
            g = choices[int(rng.integers(0, 2))]
        prev[q] = g
        ops.append(Op(ONE_QUBIT_SET[g], (q,)))
    return ops


def grid_couplers(rows: int, cols: int, pattern: int) -> List[Tuple[int, int]]:
    """Qubit pairs of coupler pattern 0..3 (A..D) on a rows x cols grid."""
    pairs = []
    if pattern in (0, 1):
        for r in range(rows):
            for c in range(pattern, cols - 1, 2):
                pairs.append((r * cols + c, r * cols + c + 1))
    else:
        for r in range(pattern - 2, rows - 1, 2):
            for c in range(cols):
                pairs.append((r * cols + c, (r + 1) * cols + c))
    return pairs


def grid_random_circuit(rows: int, cols: int, cycles: int, seed: int,
                        two_qubit: str = "cz",
                        fsim_params: Tuple[float, float] = (math.pi / 2, math.pi / 6),
                        n_qubits: int | None = None) -> Tuple[int, List[Op]]:
    """Random grid circuit; ``two_qubit`` is "cz" or "fsim".

    ``n_qubits`` (optional) keeps only the first n sites of the grid; couplers
    touching a dropped site are skipped.
    """
    n_full = rows * cols
    n = n_full if n_qubits is None else int(n_qubits)
    rng = np.random.default_rng(seed)
    prev = [-1] * n
    ops: List[Op] = []
    for t in range(cycles):
        ops.extend(_single_layer(rng, n, prev, t == 0))
        for a, b in grid_couplers(rows, cols, t % 4):
            if a >= n or b >= n:
                continue
            if two_qubit == "cz":
                ops.append(Op("cz", (a, b)))
            elif two_qubit == "fsim":
                ops.append(Op("fsim", (a, b), tuple(float(x) for x in fsim_params)))
            else:
                raise ValueError(two_qubit)
    return n, ops


def path_search_circuit(i: int) -> Tuple[int, List[Op]]:
    """Circuit i of the path-search corpus: n in [30, 60] qubits on the first
    n sites of a floor(sqrt(n)) x ceil(n / floor(sqrt(n))) grid, 8-16
    cycles of the CZ grid family, all drawn from seed 100000 + i
    (training set: i < 5000; held-out set: i >= 5000)."""
    rng = np.random.default_rng(100000 + i)
    n = int(rng.integers(30, 61))
    cycles = int(rng.integers(8, 17))
    rows = int(math.isqrt(n))
    cols = -(-n // rows)
    return grid_random_circuit(rows, cols, cycles, 100000 + i, n_qubits=n)


def chain_random_circuit(n: int, cycles: int, seed: int,
                         fsim_params: Tuple[float, float] = (math.pi / 2, math.pi / 6)
                         ) -> Tuple[int, List[Op]]:
    """1D chain: single-qubit layer, then fSim on even bonds (even cycles) or
    odd bonds (odd cycles)."""
    rng = np.random.default_rng(seed)
    prev = [-1] * n
    ops: List[Op] = []
    for t in range(cycles):
        ops.extend(_single_layer(rng, n, prev, t == 0))
        for a in range(t % 2, n - 1, 2):
            ops.append(Op("fsim", (a, a + 1), tuple(float(x) for x in fsim_params)))
    return n, ops


def cat_circuit(n: int) -> Tuple[int, List[Op]]:
    """H on qubit 0, then CX(0, i) for i = 1..n-1 (the paper's Sec. 4.4 state)."""
    ops = [Op("h", (0,))]
    ops += [Op("cx", (0, i)) for i in range(1, n)]
    return n, ops


def ghz_circuit(n: int) -> Tuple[int, List[Op]]:
    """H then a CX ladder (i, i+1)."""
    ops = [Op("h", (0,))]
    ops += [Op("cx", (i, i + 1)) for i in range(n - 1)]
    return n, ops


def bell_circuit() -> Tuple[int, List[Op]]:
    return 2, [Op("h", (0,)), Op("cx", (0, 1))]


def qft_circuit(n: int, x: int) -> Tuple[int, List[Op]]:
    """Prepare basis state |x> (qubit 0 = MSB) with X gates, then the textbook
    quantum Fourier transform: H and controlled phases, then qubit reversal."""
    ops = []
    for q in range(n):
        if (x >> (n - 1 - q)) & 1:
            ops.append(Op("x", (q,)))
    for j in range(n):
        ops.append(Op("h", (j,)))
        for k in range(j + 1, n):
            ops.append(Op("cphase", (k, j), (2.0 * math.pi / float(1 << (k - j + 1)),)))
    for i in range(n // 2):
        ops.append(Op("swap", (i, n - 1 - i)))
    return n, ops


def hh_circuit(cycles: int) -> Tuple[int, List[Op]]:
    """Back-to-back Hadamard pairs on one qubit (the paper's noisy H-H test)."""
    ops = []
    for _ in range(cycles):
        ops.append(Op("h", (0,)))
        ops.append(Op("h", (0,)))
    return 1, ops


def noisy_ops(ops: Sequence[Op], p1: float, p2: float, gamma: float) -> List[Op]:
    """Insert channels after every gate: depolarising on the gate's qubits
    (depol1(p1) or depol2(p2)), then amplitude damping(gamma) on each qubit
    the gate touches.  Zero rates insert nothing."""
    out: List[Op] = []
    for op in ops:
        out.append(op)
        if len(op.qubits) == 1 and p1 > 0:
            out.append(Op("depol1", op.qubits, (float(p1),)))
        if len(op.qubits) == 2 and p2 > 0:
            out.append(Op("depol2", op.qubits, (float(p2),)))
        if gamma > 0:
            for q in op.qubits:
                out.append(Op("amp_damp", (q,), (float(gamma),)))
    return out


def count_channel_events(ops: Sequence[Op]) -> int:
    return sum(1 for op in ops if op.name in ("depol1", "depol2", "amp_damp"))
