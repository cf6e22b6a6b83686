"""Pins of the expectation-value oracle (Sec. 3.1, Eq. 2, Table 1) and the
host-side double-depth network builder of the library against it."""

import math

import numpy as np
import pytest

from oracle import observables as ob
from oracle.contract import contract_path
from oracle.network import fix_labels
from oracle.paths import greedy_path
from workloads import Op, ghz_circuit, grid_random_circuit, chain_random_circuit

rng = np.random.default_rng(77)


def random_pauli(n, weight, rng):
    codes = [0] * n
    for q in rng.choice(n, size=weight, replace=False):
        codes[int(q)] = int(rng.integers(1, 4))
    return codes


def test_ghz_closed_forms():
    n, ops = ghz_circuit(4)
    assert abs(ob.expectation(n, ops, "ZZII") - 1) < 1e-12
    assert abs(ob.expectation(n, ops, "IZIZ") - 1) < 1e-12
    assert abs(ob.expectation(n, ops, "ZIII")) < 1e-12
    assert abs(ob.expectation(n, ops, "XXXX") - 1) < 1e-12
    assert abs(ob.expectation(n, ops, "YYXX") + 1) < 1e-12
    assert abs(ob.expectation(n, ops, "YYYY") - 1) < 1e-12
    assert abs(ob.expectation(n, ops, "XIII")) < 1e-12


@pytest.mark.parametrize("gates,pauli,want", [
    ([Op("sqrt_x", (0,))], "Y", -1.0),
    ([Op("sqrt_x", (0,))], "Z", 0.0),
    ([Op("sqrt_y", (0,))], "X", 1.0),
    ([Op("h", (0,))], "X", 1.0),
    ([Op("h", (0,)), Op("s", (0,))], "Y", 1.0),
    ([], "Z", 1.0),
])
def test_one_qubit_rotations(gates, pauli, want):
    assert abs(ob.expectation(1, gates, pauli) - want) < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_three_evaluations_agree(seed):
    r = np.random.default_rng(seed)
    n, ops = grid_random_circuit(3, 3, 4 + seed, 300 + seed)
    codes = random_pauli(n, 1 + seed % 3, r)
    ref = ob.expectation(n, ops, codes)
    assert abs(ref.imag) < 1e-12 and abs(ref.real) <= 1 + 1e-12
    assert abs(ob.conjugate_network_value(n, ops, codes, collapse=False) - ref) < 1e-12
    assert abs(ob.conjugate_network_value(n, ops, codes, collapse=True) - ref) < 1e-12
    support = [q for q in range(n) if codes[q] in (1, 2)]
    extra = [q for q in range(n) if q not in support][: 6 - len(support)]
    assert abs(ob.sliced_expectation(n, ops, codes, support + extra) - ref) < 1e-12


def test_identity_string_is_one():
    n, ops = grid_random_circuit(2, 3, 5, 9)
    assert abs(ob.expectation(n, ops, [0] * n) - 1) < 1e-12
    assert ob.light_cone(n, ops, [0] * n) == []
    assert abs(ob.sliced_expectation(n, ops, [0] * n, [0, 2]) - 1) < 1e-12


def test_light_cone_of_a_chain():
    """Brickwork chain: a Z on one end qubit after d layers keeps the
    gates inside the cone that widens by one site per two-qubit layer."""
    n, ops = chain_random_circuit(8, 3, 4)
    kept = ob.light_cone(n, ops, [3] + [0] * 7)
    # every kept two-qubit gate touches the cone; every dropped one lies
    # strictly outside the support grown from the end
    live = {0}
    for k in range(len(ops) - 1, -1, -1):
        qs = set(ops[k].qubits)
        inside = bool(qs & live)
        assert (k in kept) == inside
        if inside:
            live |= qs
    assert len(kept) < len(ops)


def test_sliced_rejects_x_on_projected_qubit():
    n, ops = ghz_circuit(3)
    with pytest.raises(ValueError):
        ob.sliced_expectation(n, ops, "XII", [1, 2])


# ---- the library's host-side builder, contracted by the oracle ----------

def contract_closed(net, n):
    """All output legs projected on 0, contracted along the oracle's greedy path."""
    info = net.info()
    tensors, labels = [], []
    for i in range(info.n_tensors):
        T, ls = net.tensor(i)
        tensors.append(T)
        labels.append(ls)
    out = net.output_labels()
    tensors, labels = fix_labels(tensors, labels, {l: 0 for l in out})
    path = greedy_path([list(l) for l in labels], [2] * info.n_labels)
    return complex(contract_path(tensors, labels, path, []))


@pytest.mark.parametrize("seed", range(3))
def test_library_double_depth_network(seed):
    import paper_2104_10523_amd as tn
    r = np.random.default_rng(40 + seed)
    n, ops = grid_random_circuit(3, 3, 3 + seed, 500 + seed)
    codes = random_pauli(n, 1 + seed, r)
    net, kept = tn.tn_build_expectation_network(n, ops, codes)
    assert kept == len(ob.light_cone(n, ops, codes))
    assert abs(contract_closed(net, n) - ob.expectation(n, ops, codes)) < 1e-12


def test_library_double_depth_identity_and_errors():
    import paper_2104_10523_amd as tn
    n, ops = grid_random_circuit(2, 2, 3, 1)
    net, kept = tn.tn_build_expectation_network(n, ops, [0] * n)
    assert kept == 0
    assert abs(contract_closed(net, n) - 1) < 1e-12
    with pytest.raises(tn.TnError, match="TN_ERR_ARG"):
        tn.tn_build_expectation_network(n, ops, [0, 4, 0, 0])
    with pytest.raises(tn.TnError, match="TN_ERR_GATE"):
        tn.tn_build_expectation_network(n, ops + [Op("depol1", (0,), (0.1,))], "ZIII")


# ---- density matrix (Sec. 3.3, Eq. 3) -------------------------------------

from workloads import hh_circuit, noisy_ops


def test_dm_expectation_noiseless_equals_pure():
    r = np.random.default_rng(5)
    n, ops = grid_random_circuit(2, 3, 4, 61)
    for w in (1, 2, 3):
        codes = random_pauli(n, w, r)
        assert abs(ob.dm_expectation(n, ops, codes) - ob.expectation(n, ops, codes)) < 1e-12


def test_dm_expectation_depolarised_hh_closed_form():
    p, cyc = 0.03, 6
    _, ops = hh_circuit(cyc)
    ops = noisy_ops(ops, p, 0.0, 0.0)
    got = ob.dm_expectation(4, ops, "ZIII")
    assert abs(got - (1 - 4 * p / 3) ** (2 * cyc)) < 1e-12


@pytest.mark.parametrize("seed", range(3))
def test_library_density_network(seed):
    """The library's density-matrix network (host side), contracted by the
    oracle, equals Tr(rho P) of the density-matrix oracle."""
    import paper_2104_10523_amd as tn
    r = np.random.default_rng(90 + seed)
    n, ops = grid_random_circuit(2, 3, 3 + seed, 900 + seed)
    ops = noisy_ops(ops, 0.02, 0.05, 0.07)
    codes = random_pauli(n, 1 + seed, r)
    net, kept = tn.tn_build_density_network(n, ops, codes)
    assert net.info().n_qubits == 0 and kept <= len(ops)
    assert abs(contract_closed(net, 0) - ob.dm_expectation(n, ops, codes)) < 1e-12


def test_library_density_network_trace_and_light_cone():
    import paper_2104_10523_amd as tn
    n, ops = chain_random_circuit(6, 2, 8)
    ops = noisy_ops(ops, 0.01, 0.02, 0.03)
    net, kept = tn.tn_build_density_network(n, ops, [0] * n)
    assert kept == 0 and abs(contract_closed(net, 0) - 1) < 1e-12
    net, kept = tn.tn_build_density_network(n, ops, [3, 0, 0, 0, 0, 0])
    assert 0 < kept < len(ops)
    assert abs(contract_closed(net, 0) - ob.dm_expectation(n, ops, "ZIIIII")) < 1e-12
