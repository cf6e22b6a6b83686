"""Host-side checks of the native library (no GPU needed): the C ABI loads
and exports every declared entry point; the library's circuit-to-network
mapping, greedy and randomised-greedy paths, cost model and slicer agree
exactly with the oracle's independent implementation; host-side errors map
to the documented status codes."""

import ctypes
import math
import re
from pathlib import Path

import numpy as np
import pytest

import paper_2104_10523_amd as tn
from oracle.network import build_network
from oracle.paths import (SplitMix64, greedy_path, partition_path, partition_search, path_stats,
                          random_greedy_path, reconfigure_path, slice_path)
from workloads import Op, grid_random_circuit, chain_random_circuit, cat_circuit, qft_circuit

HEADER = Path(__file__).resolve().parent.parent / "include" / "tn.h"


def declared_functions():
    txt = HEADER.read_text()
    return sorted(set(re.findall(r"^\s*(?:tn_status|const char\*)\s+(tn_\w+)\s*\(", txt, re.M)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(str(tn._native.LIB_PATH))
    names = declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) <= set(tn._native.SIGNATURES)


def test_version_and_last_error():
    assert b"gfx950" in tn.lib().tn_version()


def _oracle_leaves(onet, open_q=()):
    outs = {onet.out_label[q] for q in range(onet.n_qubits) if q not in open_q}
    opened = {onet.out_label[q] for q in open_q}
    leaves = [[l for l in ls if l not in outs] for ls in onet.labels]
    return leaves, onet.extents(), opened


CIRCUITS = [
    ("c1_3x4x8", lambda: grid_random_circuit(3, 4, 8, 1)),
    ("grid_4x5x10", lambda: grid_random_circuit(4, 5, 10, 3)),
    ("chain_10x6", lambda: chain_random_circuit(10, 6, 5)),
    ("cat_16", lambda: cat_circuit(16)),
    ("qft_6", lambda: qft_circuit(6, 13)),
    ("lone_wires", lambda: (4, [Op("h", (0,)), Op("sqrt_x", (3,)), Op("cz", (0, 1))])),
]


@pytest.mark.parametrize("name,make", CIRCUITS, ids=[c[0] for c in CIRCUITS])
def test_network_matches_oracle(name, make):
    n, ops = make()
    onet = build_network(n, ops)
    lnet = tn.tn_build_network(n, ops)
    info = lnet.info()
    assert (info.n_qubits, info.n_tensors, info.n_labels) == (n, len(onet.tensors), onet.n_labels)
    assert lnet.output_labels() == onet.out_label
    for i in range(info.n_tensors):
        T, labels = lnet.tensor(i)
        assert labels == onet.labels[i]
        assert np.abs(T - onet.tensors[i]).max() <= 1e-15


@pytest.mark.parametrize("name,make", CIRCUITS, ids=[c[0] for c in CIRCUITS])
def test_greedy_path_and_cost_match_oracle(name, make):
    n, ops = make()
    onet = build_network(n, ops)
    lnet = tn.tn_build_network(n, ops)
    for open_q in ((), (0, n - 1)):
        mask = [1 if q in open_q else 0 for q in range(n)]
        leaves, ext, opened = _oracle_leaves(onet, open_q)
        p = tn.tn_find_path(lnet, "greedy", open_mask=mask)
        po = greedy_path(leaves, ext, opened)
        st = path_stats(leaves, ext, po, opened)
        assert p.pairs == po
        assert p.cost.flops_per_slice == st["flops"]
        assert p.cost.peak_elems == st["peak"]


def test_random_greedy_matches_oracle():
    n, ops = grid_random_circuit(4, 5, 10, 3)
    onet = build_network(n, ops)
    lnet = tn.tn_build_network(n, ops)
    leaves, ext, opened = _oracle_leaves(onet)
    # 40 trials spread over the library's host threads: the winner must still
    # be the sequential scan's
    for seed, T, trials in ((1, 1.0, 6), (77, 0.5, 6), (5, 0.5, 40)):
        p = tn.tn_find_path(lnet, "random_greedy", trials=trials, seed=seed, temperature=T)
        po = random_greedy_path(leaves, ext, opened, seed=seed, trials=trials, temperature=T)
        assert p.pairs == po


def test_random_greedy_with_budget_reranks_like_oracle():
    """With a memory budget the best candidates are re-ranked by their
    sliced total flops; library and oracle pick the same path and slices."""
    n, ops = grid_random_circuit(4, 5, 10, 3)
    onet = build_network(n, ops)
    lnet = tn.tn_build_network(n, ops)
    leaves, ext, opened = _oracle_leaves(onet)
    peak = path_stats(leaves, ext, greedy_path(leaves, ext, opened), opened)["peak"]
    for div, trials in ((16, 24), (256, 40)):
        budget = 8 * peak / div
        p = tn.tn_find_path(lnet, "random_greedy", trials=trials, seed=9, temperature=0.5, mem_budget_bytes=budget)
        po = random_greedy_path(leaves, ext, opened, seed=9, trials=trials, temperature=0.5, budget_bytes=budget)
        assert p.pairs == po
        assert p.sliced == slice_path(leaves, ext, po, opened, budget)


def test_slicing_matches_oracle_and_meets_budget():
    n, ops = grid_random_circuit(4, 5, 10, 3)
    onet = build_network(n, ops)
    lnet = tn.tn_build_network(n, ops)
    leaves, ext, opened = _oracle_leaves(onet)
    po = greedy_path(leaves, ext, opened)
    peak = path_stats(leaves, ext, po, opened)["peak"]
    for div in (4, 64):
        budget = 8 * peak / div
        p = tn.tn_find_path(lnet, "greedy", mem_budget_bytes=budget)
        so = slice_path(leaves, ext, po, opened, budget)
        assert p.sliced == so
        assert 8 * p.cost.peak_elems <= budget
        st = path_stats(leaves, ext, po, opened, so)
        assert p.cost.total_flops == st["total_flops"] and p.cost.n_slices == 2 ** len(so)


def test_c2_network_path_cost():
    """49-qubit 7x7 grid, 14 cycles of fSim: greedy path and slicing to a
    256 GiB budget, identical on both sides."""
    n, ops = grid_random_circuit(7, 7, 14, 2, two_qubit="fsim")
    onet = build_network(n, ops)
    lnet = tn.tn_build_network(n, ops)
    assert lnet.info().n_tensors == 294
    leaves, ext, opened = _oracle_leaves(onet)
    p = tn.tn_find_path(lnet, "greedy", mem_budget_bytes=256 * 2 ** 30)
    po = greedy_path(leaves, ext, opened)
    assert p.pairs == po
    assert 8 * p.cost.peak_elems <= 256 * 2 ** 30
    so = slice_path(leaves, ext, po, opened, 256 * 2 ** 30)
    assert p.sliced == so


def test_path_from_pairs_validates():
    n, ops = grid_random_circuit(3, 4, 8, 1)
    lnet = tn.tn_build_network(n, ops)
    p = tn.tn_find_path(lnet, "greedy")
    q = tn.tn_path_from_pairs(lnet, p.pairs)
    assert q.cost.flops_per_slice == p.cost.flops_per_slice
    with pytest.raises(tn.TnError, match="ARG"):
        tn.tn_path_from_pairs(lnet, p.pairs[:-1])
    bad = list(p.pairs)
    bad[-1] = (0, 1)
    with pytest.raises(tn.TnError, match="ARG"):
        tn.tn_path_from_pairs(lnet, bad)


def test_host_error_codes():
    with pytest.raises(tn.TnError, match="GATE"):
        tn.tn_build_network(2, [Op("cz", (0, 2))])
    with pytest.raises(tn.TnError, match="GATE"):
        tn.tn_build_network(2, [Op("cz", (1, 1))])
    with pytest.raises(tn.TnError, match="GATE"):
        tn.tn_build_network(2, [Op("depol1", (0,), (0.1,))])
    with pytest.raises(tn.TnError, match="GATE"):
        tn.tn_build_network(1, [Op(99, (0,))])
    with pytest.raises(tn.TnError, match="GATE"):
        tn.tn_build_network(2, [Op("custom2", (0, 1), (np.ones((4, 4)),))])
    with pytest.raises(tn.TnError, match="ARG"):
        tn.tn_build_network(0, [])
    n, ops = grid_random_circuit(3, 4, 8, 1)
    lnet = tn.tn_build_network(n, ops)
    with pytest.raises(tn.TnError, match="BUDGET"):
        tn.tn_find_path(lnet, "greedy", mem_budget_bytes=8.0)
    with pytest.raises(tn.TnError, match="STATE"):
        tn.tn_find_path(lnet, "learned")
    with pytest.raises(tn.TnError, match="ARG"):
        tn.tn_find_path(lnet, "random_greedy", temperature=0.0)


def test_custom_gates_match_named():
    from oracle.gates import gate_matrix
    n = 3
    ops_named = [Op("h", (0,)), Op("fsim", (0, 2), (0.4, 0.9)), Op("sqrt_w", (1,)), Op("cx", (1, 2))]
    ops_custom = [Op("custom1", (0,), (gate_matrix("h"),)),
                  Op("custom2", (0, 2), (gate_matrix("fsim", (0.4, 0.9)),)),
                  Op("custom1", (1,), (gate_matrix("sqrt_w"),)), Op("cx", (1, 2))]
    a = tn.tn_build_network(n, ops_named)
    b = tn.tn_build_network(n, ops_custom)
    for i in range(a.info().n_tensors):
        assert np.abs(a.tensor(i)[0] - b.tensor(i)[0]).max() <= 1e-15


def test_scorer_features_match_oracle():
    """The native featurizer of the learned path search equals the oracle's
    (O7) at several states along a path."""
    from oracle import gnn
    from oracle.paths import _State
    n, ops = grid_random_circuit(3, 4, 8, 1)
    onet = build_network(n, ops)
    lnet = tn.tn_build_network(n, ops)
    leaves, ext, opened = _oracle_leaves(onet)
    path = greedy_path(leaves, ext, opened)
    st = _State(leaves, opened, ())
    for t, step in enumerate(path[:-1]):
        if t % 5 == 0:
            cand, X, nbrs = tn.tn_model_state_features(lnet, path, t)
            ocand, oX, onbrs = gnn.candidates_and_features(st, ext, len(leaves))
            assert cand == ocand
            assert np.abs(X - oX).max() <= 1e-15
            assert [list(map(int, a)) for a in nbrs] == onbrs
        st.merge(*step)


def test_identity_coupled_7x7_has_benchmark_path():
    """The full-size GPU parity case (fSim(0, 0) couplers) has the network
    structure of the benchmark's 7x7 grid circuit (same tensors, labels and
    extents), so every path search plans it alike: here the recursive-
    bisection search at 64 trials with the benchmark's 160 GiB budget and
    time ranking (the full-size GPU test repeats this at the benchmark's 1024
    trials)."""
    n, ops = grid_random_circuit(7, 7, 14, 2, two_qubit="fsim")
    _, ops0 = grid_random_circuit(7, 7, 14, 2, two_qubit="fsim", fsim_params=(0.0, 0.0))
    a, b = tn.tn_build_network(n, ops), tn.tn_build_network(n, ops0)
    assert a.info().n_tensors == b.info().n_tensors
    for i in range(a.info().n_tensors):
        assert a.tensor(i)[1] == b.tensor(i)[1]
    opts = dict(trials=64, seed=1, mem_budget_bytes=160.0 * 2 ** 30, rank="time")
    p = tn.tn_find_path(a, "partition", **opts)
    p0 = tn.tn_find_path(b, "partition", **opts)
    assert p.pairs == p0.pairs and p.sliced == p0.sliced
    assert p.cost.n_sliced == p0.cost.n_sliced and p.cost.n_sliced >= 4


def _modelled_seconds(net, path, precision="auto"):
    """The library's kernel-time model of a whole job, from the plan's ops:
    max(flops / F, bytes / 4e12) + 5 us per op, F = 350e12 for split GEMMs
    and 120e12 otherwise; times the number of slices."""
    kind, fl, by, sh = tn.tn_amplitudes_plan_ops(net, path, precision)
    F = np.where((kind == 2) & (sh[:, 5] != 0), 350e12, 120e12)
    return path.cost.n_slices * float(np.sum(np.maximum(fl / F, by / 4e12) + 5e-6))


@pytest.mark.parametrize("rows,cols,cyc,budget", [(5, 5, 10, 2.0 ** 24), (6, 6, 12, 2.0 ** 28)])
def test_time_ranking_never_models_slower_than_the_flop_winner(rows, cols, cyc, budget):
    """Time ranking (the 16 best bisection trees by flops, each also
    reconfigured for modelled step time and re-sliced) picks a plan whose
    modelled time is at most that of the flop-ranked winner, which is one
    of its candidates; the path stays a complete contraction order."""
    n, ops = grid_random_circuit(rows, cols, cyc, 4, two_qubit="fsim")
    net = tn.tn_build_network(n, ops)
    opts = dict(trials=48, seed=2, mem_budget_bytes=budget)
    pf = tn.tn_find_path(net, "partition", **opts)
    pt = tn.tn_find_path(net, "partition", rank="time", rank_precision="auto", **opts)
    assert len(pt.pairs) == net.info().n_tensors - 1
    again = tn.tn_path_from_pairs(net, pt.pairs, mem_budget_bytes=budget)
    assert again.sliced == pt.sliced and again.cost.total_flops == pt.cost.total_flops
    assert 8.0 * pt.cost.peak_elems <= budget
    tf, tt = _modelled_seconds(net, pf), _modelled_seconds(net, pt)
    assert tt <= tf * (1 + 1e-12)


# ---- recursive-bisection path search -------------------------------------

@pytest.mark.parametrize("name,make", CIRCUITS, ids=[c[0] for c in CIRCUITS])
def test_partition_search_matches_oracle(name, make):
    """Library and oracle build the same bisection trees and pick the same
    winner (trials on host threads), with open legs and without."""
    n, ops = make()
    onet = build_network(n, ops)
    lnet = tn.tn_build_network(n, ops)
    for open_q in ((), (0, n - 1)):
        mask = [1 if q in open_q else 0 for q in range(n)]
        leaves, ext, opened = _oracle_leaves(onet, open_q)
        p = tn.tn_find_path(lnet, "partition", trials=12, seed=3, open_mask=mask)
        po = partition_search(leaves, ext, opened, seed=3, trials=12)
        assert p.pairs == po


def test_partition_trials_match_one_by_one():
    """Every single trial of the library equals the oracle's tree: with one
    trial the winner is that tree unless greedy is cheaper."""
    n, ops = grid_random_circuit(4, 5, 10, 3)
    onet = build_network(n, ops)
    leaves, ext, opened = _oracle_leaves(onet)
    for r in range(6):
        from oracle.paths import GOLDEN, MASK64
        g = SplitMix64((11 + r * GOLDEN) & MASK64)
        tree = partition_path(leaves, ext, opened, SplitMix64(g.next_u64()))
        st = path_stats(leaves, ext, tree, opened)       # a valid path over all leaves
        assert len(tree) == len(leaves) - 1
        lib = tn.tn_path_from_pairs(tn.tn_build_network(n, ops), tree)
        assert lib.cost.flops_per_slice == st["flops"]


def test_partition_with_budget_matches_oracle():
    n, ops = grid_random_circuit(4, 5, 12, 7)
    onet = build_network(n, ops)
    lnet = tn.tn_build_network(n, ops)
    leaves, ext, opened = _oracle_leaves(onet)
    unsliced = path_stats(leaves, ext, partition_search(leaves, ext, opened, seed=2, trials=8), opened)
    budget = 8.0 * unsliced["peak"] / 16
    p = tn.tn_find_path(lnet, "partition", trials=8, seed=2, mem_budget_bytes=budget)
    po = partition_search(leaves, ext, opened, seed=2, trials=8, budget_bytes=budget)
    assert p.pairs == po
    assert p.sliced == slice_path(leaves, ext, po, opened, budget)
    assert 8.0 * p.cost.peak_elems <= budget


def test_partition_tree_contracts_to_the_amplitude():
    """The oracle's own bisection tree, contracted by the oracle, gives the
    state-vector amplitude (the tree is a valid complete contraction)."""
    from oracle import statevector as sv
    from oracle.contract import contract_path
    from oracle.network import fix_outputs
    n, ops = grid_random_circuit(3, 3, 6, 5)
    onet = build_network(n, ops)
    bits = [1, 0, 1, 1, 0, 0, 1, 0, 1]
    tensors, labels, open_l = fix_outputs(onet, bits)
    improved = 0
    for r in range(3):
        ls = [list(l) for l in labels]
        tree = partition_path(ls, onet.extents(), set(), SplitMix64(100 + r))
        amp = complex(contract_path(tensors, labels, tree, []))
        assert abs(amp - sv.amplitudes(n, ops, bits)[0]) < 1e-12
        # the reconfigured tree is complete, never costs more, and contracts
        # to the same amplitude
        rt = reconfigure_path(ls, onet.extents(), set(), tree)
        f0 = path_stats(ls, onet.extents(), tree)["flops"]
        f1 = path_stats(ls, onet.extents(), rt)["flops"]
        assert f1 <= f0
        improved += f1 < f0
        amp_r = complex(contract_path(tensors, labels, rt, []))
        assert abs(amp_r - sv.amplitudes(n, ops, bits)[0]) < 1e-12
    assert improved >= 1


def test_noalloc_contract_pair_rejects_scratch_beyond_its_array():
    """Host-side check of the allocation-free tn_contract_pair variant: a GEMM
    whose 2^24-entry operand must be permuted needs 128 MiB of scratch, above
    the fixed 64 MiB array, and is refused before any device call (the data
    pointers are never dereferenced)."""
    from paper_2104_10523_amd._native import TnTensor
    TN_C64 = 0
    rng = np.random.default_rng(0)
    la = list(range(24))
    rng.shuffle(la)                        # labels 0..13 free, 14..23 contracted
    lb = list(range(14, 24)) + list(range(100, 106))
    lc = list(range(14)) + list(range(100, 106))

    def tensor(labels):
        ext = (ctypes.c_int64 * len(labels))(*([2] * len(labels)))
        return TnTensor(ctypes.c_void_p(0x1000), len(labels), TN_C64, ext), ext

    (TA, ea), (TB, eb), (TC, ec) = tensor(la), tensor(lb), tensor(lc)
    arr = lambda v: (ctypes.c_int32 * len(v))(*v)
    code = tn.lib().tn_contract_pair_noalloc(ctypes.byref(TA), arr(la), ctypes.byref(TB), arr(lb),
                                              ctypes.byref(TC), arr(lc), 0, None)
    assert code != 0
    msg = tn.lib().tn_last_error().decode()
    assert "67108864" in msg and "needs" in msg, msg
    with pytest.raises(tn.TnError, match="WORKSPACE"):
        tn._native.check(code)


@pytest.mark.parametrize("precision", ["f16x3", "auto"])
def test_fp16_packing_takes_the_producers_max(precision):
    """Packing an operand into scaled fp16 planes needs its largest |re|,
    |im| first.  Where a direct-to-LDS split GEMM or a 16-output matrix-core
    apply produced the operand, that op reports the max as it stores its
    result, so the plan has fewer max-abs passes than fp16 packings (the
    GPU tests contract this plan against the state vector)."""
    n, ops = grid_random_circuit(4, 5, 14, 2, two_qubit="fsim")
    net = tn.tn_build_network(n, ops)
    path = tn.tn_find_path(net, "greedy", open_mask=[1] * n)
    kind, _, _, sh = tn.tn_amplitudes_plan_ops(net, path, precision)
    perm = kind == 1
    maxabs = int(np.sum(perm & (sh[:, 3] == 3)))
    packs = int(np.sum(perm & (sh[:, 1] == 2) & (sh[:, 2] == 1) & (sh[:, 3] != 3)))
    assert packs > 0 and 0 < maxabs < packs
