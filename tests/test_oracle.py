"""Pins of the CPU oracle against facts that do not come from the oracle:
closed forms, the paper's worked example, library routines on special cases,
hand-computed costs and brute force on tiny inputs."""

import itertools
import json
import math
from pathlib import Path

import numpy as np
import pytest

from oracle import gates, statevector as sv
from oracle.contract import contract_pair, contract_pair_loops, contract_pair_mm, contract_path
from oracle.network import build_network, fix_outputs, fix_labels
from oracle.paths import (greedy_path, path_stats, random_greedy_path, slice_path, SplitMix64)
from workloads import (grid_random_circuit, cat_circuit, ghz_circuit, bell_circuit, qft_circuit,
                       random_complex)

GOLDEN = Path(__file__).parent / "golden"

ONE_Q = ["sqrt_x", "sqrt_y", "sqrt_w", "h", "x", "y", "z", "s", "t"]


# ------------------------------------------------------------------ gates

@pytest.mark.parametrize("name,params", [(g, ()) for g in ONE_Q] + [
    ("rz", (0.3,)), ("cz", ()), ("cx", ()), ("swap", ()), ("cphase", (0.7,)),
    ("fsim", (math.pi / 2, math.pi / 6)), ("fsim", (0.3, 1.1))])
def test_gates_unitary(name, params):
    U = gates.gate_matrix(name, params)
    assert np.abs(U.conj().T @ U - np.eye(U.shape[0])).max() <= 1e-15


def test_sqrt_gates_square_to_paulis():
    # R_P(pi/2)^2 = R_P(pi) = -i P for a Pauli-like P (P^2 = 1)
    W = (gates.X + gates.Y) / math.sqrt(2)
    for name, P in (("sqrt_x", gates.X), ("sqrt_y", gates.Y), ("sqrt_w", W)):
        U = gates.gate_matrix(name)
        assert np.allclose(U @ U, -1j * P, atol=1e-15)


def test_fsim_special_cases():
    # fsim(0, phi) is a controlled phase exp(-i phi) on |11>; fsim(pi/2, 0)
    # swaps |01> and |10> with a -i phase (iSWAP^dagger)
    assert np.allclose(gates.gate_matrix("fsim", (0.0, 0.4)), gates.gate_matrix("cphase", (-0.4,)))
    F = gates.gate_matrix("fsim", (math.pi / 2, 0.0))
    assert np.allclose(F @ np.array([0, 1, 0, 0]), [0, 0, -1j, 0])


@pytest.mark.parametrize("name,params", [("depol1", (0.1,)), ("depol2", (0.3,)), ("amp_damp", (0.2,))])
def test_kraus_completeness(name, params):
    ks = gates.kraus_ops(name, params)
    S = sum(K.conj().T @ K for K in ks)
    assert np.abs(S - np.eye(S.shape[0])).max() <= 1e-15
    assert len(ks) == {"depol1": 4, "depol2": 16, "amp_damp": 2}[name]


# ------------------------------------------------------------ state vector

def test_bell_closed_form():
    n, ops = bell_circuit()
    psi = sv.simulate(n, ops).reshape(-1)
    r = 1 / math.sqrt(2)
    assert np.allclose(psi, [r, 0, 0, r], atol=1e-15)


@pytest.mark.parametrize("n", [3, 7, 12])
def test_ghz_closed_form(n):
    _, ops = ghz_circuit(n)
    psi = sv.simulate(n, ops).reshape(-1)
    ref = np.zeros(1 << n)
    ref[0] = ref[-1] = 1 / math.sqrt(2)
    assert np.abs(psi - ref).max() <= 1e-15


@pytest.mark.parametrize("n,x", [(3, 5), (6, 0), (8, 77), (10, 1023)])
def test_qft_basis_state(n, x):
    _, ops = qft_circuit(n, x)
    psi = sv.simulate(n, ops).reshape(-1)
    y = np.arange(1 << n)
    ref = np.exp(2j * np.pi * x * y / (1 << n)) / math.sqrt(1 << n)
    assert np.abs(psi - ref).max() <= 1e-12


def test_identity_circuit_returns_zero_state():
    from workloads import Op
    ops = [Op("h", (0,)), Op("cx", (0, 1)), Op("sqrt_x", (2,)), Op("cx", (0, 1)), Op("h", (0,))]
    ops += [Op("sqrt_x", (2,))] * 3        # sqrt_x^4 = (-i X)^2 = -I
    psi = sv.simulate(3, ops).reshape(-1)
    assert abs(psi[0] + 1) <= 1e-15 and np.abs(psi[1:]).max() <= 1e-15


def test_norm_and_porter_thomas_c1():
    n, ops = grid_random_circuit(3, 4, 8, 1)
    p = np.abs(sv.simulate(n, ops).reshape(-1)) ** 2
    assert abs(p.sum() - 1) <= 1e-12
    N = p.size
    x = np.sort(N * p)
    ks = np.max(np.abs(np.arange(1, N + 1) / N - (1 - np.exp(-x))))
    assert ks < 1.63 / math.sqrt(N)                 # KS critical value, alpha = 0.01
    assert abs((x ** 2).mean() - 2 * N / (N + 1)) < 0.21  # 3 sigma of the second moment


def test_marginal_slice_order():
    n, ops = grid_random_circuit(2, 3, 4, 9)
    psi = sv.simulate(n, ops)
    bits = [1, -1, 0, -1, -1, 1]
    got = sv.slice_of(psi, bits)
    flat = psi.reshape(-1)
    ref = []
    for a, b, c in itertools.product(range(2), repeat=3):   # open qubits 1, 3, 4: q1 is the MSB
        ref.append(flat[int("".join(map(str, [1, a, 0, b, c, 1])), 2)])
    assert np.array_equal(got, ref)


# ---------------------------------------------------------- contraction (O2)

def test_loops_hand_example():
    # C[i,k] = sum_j A[i,j] B[j,k]: a 2x2 product done by hand
    A = np.array([[1, 2j], [3, 4]])
    B = np.array([[5, 6], [7j, 8]])
    C = contract_pair_loops(A, [0, 1], B, [1, 2], [0, 2])
    assert np.array_equal(C, [[1 * 5 + 2j * 7j, 1 * 6 + 2j * 8], [3 * 5 + 4 * 7j, 3 * 6 + 4 * 8]])
    # trace-like: label only in A, summed out; batch label in A, B and C
    t = contract_pair_loops(A, [0, 1], np.ones(()), [], [])
    assert t == A.sum()
    d = contract_pair_loops(A, [0, 1], B, [0, 1], [0])
    assert np.array_equal(d, (A * B).sum(axis=1))


@pytest.mark.parametrize("seed", range(8))
def test_loops_match_einsum(seed):
    rng = np.random.default_rng(seed)
    labels = list(range(7))
    la = list(rng.choice(labels, size=rng.integers(0, 5), replace=False))
    lb = list(rng.choice(labels, size=rng.integers(0, 5), replace=False))
    pool = list(dict.fromkeys(la + lb))
    lc = [l for l in pool if rng.random() < 0.5]
    ext = {l: int(rng.integers(1, 4)) for l in labels}
    A = random_complex([ext[l] for l in la], seed + 10)
    B = random_complex([ext[l] for l in lb], seed + 20)
    got = contract_pair_loops(A, la, B, lb, lc)
    ref = contract_pair(A, la, B, lb, lc)
    assert np.abs(got - ref).max() <= 1e-12 * max(1, np.abs(ref).max())


@pytest.mark.parametrize("seed", range(24))
def test_matmul_pair_matches_loops(seed):
    """The batched-matmul contraction against the loop nest, over random
    label mixes: batch, summed, free and summed-out labels, scalar outputs."""
    rng = np.random.default_rng(100 + seed)
    labels = list(range(8))
    la = list(rng.choice(labels, size=rng.integers(0, 6), replace=False))
    lb = list(rng.choice(labels, size=rng.integers(0, 6), replace=False))
    pool = list(dict.fromkeys(la + lb))
    lc = [l for l in pool if rng.random() < 0.5]
    rng.shuffle(lc)
    ext = {l: int(rng.integers(1, 4)) for l in labels}
    A = random_complex([ext[l] for l in la], seed + 30)
    B = random_complex([ext[l] for l in lb], seed + 40)
    got = contract_pair_mm(A, la, B, lb, lc)
    ref = contract_pair_loops(A, la, B, lb, lc)
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() <= 1e-12 * max(1, np.abs(ref).max())


def test_matmul_path_equals_state_vector():
    """Whole-network contraction with the matmul pair equals O1."""
    n, ops = grid_random_circuit(3, 3, 6, 46)
    net = build_network(n, ops)
    bits = [-1] * n
    ts, ls, open_l = fix_outputs(net, bits)
    ext = {l: 2 for t in ls for l in t}
    got = contract_path(ts, ls, greedy_path(ls, ext, open_l), open_l, pair=contract_pair_mm).reshape(-1)
    ref = sv.simulate(n, ops).reshape(-1)
    assert np.abs(got - ref).max() <= 1e-12


def _net_amplitudes(n, ops, bits, path=None):
    net = build_network(n, ops)
    ts, ls, open_l = fix_outputs(net, bits)
    ext = {l: 2 for t in ls for l in t}
    if path is None:
        path = greedy_path(ls, ext, open_l)
    return contract_path(ts, ls, path, open_l).reshape(-1)


@pytest.mark.parametrize("rows,cols,cyc", [(2, 2, 1), (2, 2, 5), (2, 3, 4), (3, 3, 6), (3, 4, 8)])
def test_network_contraction_equals_state_vector(rows, cols, cyc):
    n, ops = grid_random_circuit(rows, cols, cyc, 40 + cyc)
    ref = sv.simulate(n, ops).reshape(-1)
    got = _net_amplitudes(n, ops, [-1] * n)
    assert np.abs(got - ref).max() <= 1e-13
    bits = [1, 0] * (n // 2) + [1] * (n % 2)
    a = _net_amplitudes(n, ops, bits)
    assert abs(a[0] - ref[int("".join(map(str, bits)), 2)]) <= 1e-14


def test_path_invariance():
    n, ops = grid_random_circuit(3, 3, 6, 5)
    net = build_network(n, ops)
    ts, ls, open_l = fix_outputs(net, [0] * n)
    ext = {l: 2 for t in ls for l in t}
    ref = contract_path(ts, ls, greedy_path(ls, ext, open_l), open_l)
    for seed in range(4):
        rng = SplitMix64(seed + 1)
        p = greedy_path(ls, ext, open_l, rng=rng, temperature=4.0)
        got = contract_path(ts, ls, p, open_l)
        assert abs(got - ref) <= 1e-14


def test_slicing_invariance_oracle():
    n, ops = grid_random_circuit(3, 3, 6, 6)
    net = build_network(n, ops)
    bits = [0, 1, 1, 0, 1, 0, 0, 1, 1]
    ts, ls, open_l = fix_outputs(net, bits)
    ext = {l: 2 for t in ls for l in t}
    path = greedy_path(ls, ext, open_l)
    full = contract_path(ts, ls, path, open_l)
    st = path_stats(ls, ext, path, open_l)
    budget = 8 * st["peak"] / 4
    sl = slice_path(ls, ext, path, set(open_l), budget)
    assert len(sl) >= 2
    assert 8 * path_stats(ls, ext, path, open_l, sl)["peak"] <= budget
    tot = 0
    for vals in itertools.product(range(2), repeat=len(sl)):
        ts2, ls2 = fix_labels(ts, ls, dict(zip(sl, vals)))
        tot = tot + contract_path(ts2, ls2, path, open_l)
    assert abs(tot - full) <= 1e-14


def test_cat_slice_paper_example():
    """Sec. 4.4: 60-qubit cat state, qubits 2 and 47 open (worked example)."""
    g = json.loads((GOLDEN / "cat_slice.json").read_text())
    n, ops = cat_circuit(60)
    for case in g["cases"]:
        bits = [case["others"]] * n
        for q in g["open_qubits"]:
            bits[q] = -1
        raw = _net_amplitudes(n, ops, bits)
        assert np.allclose(raw * math.sqrt(2), case["normalised_slice"], atol=1e-14)
        assert np.allclose(raw / np.linalg.norm(raw), case["normalised_slice"], atol=1e-14)
    bits = [0] * n
    bits[9] = 1
    bits[2] = bits[47] = -1
    assert np.abs(_net_amplitudes(n, ops, bits)).max() == 0


# -------------------------------------------------------------- paths (O6)

def test_cost_hand_example():
    # chain A[a,b] B[b,c] C[c,d], extents 2, all closed except a and d open
    leaves = [[0, 1], [1, 2], [2, 3]]
    ext = {0: 2, 1: 2, 2: 2, 3: 2}
    st = path_stats(leaves, ext, [(0, 1), (3, 2)], open_set={0, 3})
    assert st["flops"] == 8 * 8 + 8 * 8
    assert st["peak"] == 12 + 4 + 4 + 4        # live 12, |C|=4, |A|=|B|=4
    st2 = path_stats(leaves, ext, [(0, 1), (3, 2)], open_set={0, 3}, sliced=[1])
    assert st2["flops"] == 8 * 4 + 8 * 8 and st2["n_slices"] == 2 and st2["total_flops"] == 2 * 96


def _all_paths(ids, nxt):
    if len(ids) <= 1:
        yield []
        return
    for a, b in itertools.combinations(sorted(ids), 2):
        rest = [i for i in ids if i not in (a, b)] + [nxt]
        for tail in _all_paths(rest, nxt + 1):
            yield [(a, b)] + tail


def test_greedy_bounded_by_exhaustive_optimum():
    n, ops = grid_random_circuit(2, 3, 3, 8)
    net = build_network(n, ops)
    ts, ls, open_l = fix_outputs(net, [0] * n)
    assert len(ls) <= 7
    ext = {l: 2 for t in ls for l in t}
    best = min(path_stats(ls, ext, p, open_l)["flops"] for p in _all_paths(list(range(len(ls))), len(ls)))
    g = path_stats(ls, ext, greedy_path(ls, ext, open_l), open_l)["flops"]
    rg = path_stats(ls, ext, random_greedy_path(ls, ext, open_l, seed=1, trials=16), open_l)["flops"]
    assert best <= rg <= g


def test_splitmix64_reference_values():
    # published SplitMix64 outputs for seed 0 (first three draws)
    g = SplitMix64(0)
    assert [g.next_u64() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_contract_entries_match_full():
    from oracle.contract import contract_entries
    A = random_complex([2, 3, 2, 2], 1)
    B = random_complex([2, 2, 4], 2)
    la, lb, lc = [0, 1, 2, 3], [2, 0, 4], [4, 1, 3]
    full = contract_pair(A, la, B, lb, lc)
    idx = [(0, 0, 0), (3, 2, 1), (1, 1, 0)]
    got = contract_entries(A, la, B, lb, lc, idx)
    assert np.abs(got - np.array([full[i] for i in idx])).max() <= 1e-14
