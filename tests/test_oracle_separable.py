"""Pins of the closed-form slice value of identity-coupled circuits
(oracle/separable.py) against two independent routes: the generic network
contraction (O2) with the same bond labels fixed, and the state vector (O1)
as the sum over all values of the fixed labels."""

import itertools

import numpy as np
import pytest

from oracle import statevector as sv
from oracle.contract import contract_path
from oracle.network import build_network, fix_labels, fix_outputs
from oracle.paths import greedy_path
from oracle.separable import dominant_bits, separable_slice_amplitude
from workloads import Op, grid_random_circuit

IDENT = (0.0, 0.0)   # fSim(0, 0) is the identity


def _inner_labels(net):
    outs = set(net.out_label)
    return sorted({l for ls in net.labels for l in ls if l not in outs})


@pytest.mark.parametrize("rows,cols,cyc,seed", [(2, 3, 4, 1), (3, 3, 6, 2), (3, 4, 8, 3)])
def test_closed_form_equals_network_contraction(rows, cols, cyc, seed):
    n, ops = grid_random_circuit(rows, cols, cyc, seed, two_qubit="fsim", fsim_params=IDENT)
    net = build_network(n, ops)
    rng = np.random.default_rng(seed)
    inner = _inner_labels(net)
    for trial in range(3):
        bits = [int(b) for b in rng.integers(0, 2, n)]
        pick = sorted(int(l) for l in rng.choice(inner, size=min(5, len(inner)), replace=False))
        fixed = {l: int(rng.integers(0, 2)) for l in pick}
        ts, ls, open_l = fix_outputs(net, bits)
        ts, ls = fix_labels(ts, ls, fixed)
        ext = {l: 2 for t in ls for l in t}
        ref = complex(contract_path(ts, ls, greedy_path(ls, ext, open_l), open_l))
        got = separable_slice_amplitude(n, ops, bits, fixed)
        assert abs(got - ref) <= 1e-14 * max(1.0, abs(ref)), (trial, got, ref)


def test_sum_over_slices_is_state_vector_amplitude():
    n, ops = grid_random_circuit(3, 3, 5, 7, two_qubit="fsim", fsim_params=IDENT)
    psi = sv.simulate(n, ops)
    net = build_network(n, ops)
    inner = _inner_labels(net)
    pick = inner[::max(1, len(inner) // 4)][:4]
    for bits in ([0] * n, [1, 0, 1, 1, 0, 0, 1, 0, 1]):
        tot = sum(separable_slice_amplitude(n, ops, bits, dict(zip(pick, vals)))
                  for vals in itertools.product(range(2), repeat=len(pick)))
        ref = psi[tuple(bits)]
        assert abs(tot - ref) <= 1e-14


def test_lone_wire_and_rejects_entangling_gates():
    ops = [Op("h", (0,)), Op("sqrt_x", (2,)), Op("fsim", (0, 1), IDENT), Op("sqrt_y", (1,))]
    psi = sv.simulate(3, ops)
    for bits in itertools.product(range(2), repeat=3):
        assert abs(separable_slice_amplitude(3, ops, bits, {}) - psi[bits]) <= 1e-15
    with pytest.raises(ValueError):
        separable_slice_amplitude(2, [Op("cz", (0, 1))], [0, 0], {})


def test_dominant_bits_maximise_the_slice_value():
    """Brute force over all bit-strings of a 3x3 identity-coupled circuit."""
    n, ops = grid_random_circuit(3, 3, 6, 4, two_qubit="fsim", fsim_params=IDENT)
    net = build_network(n, ops)
    inner = _inner_labels(net)
    rng = np.random.default_rng(9)
    for trial in range(3):
        pick = sorted(int(l) for l in rng.choice(inner, size=4, replace=False))
        fixed = {l: int(rng.integers(0, 2)) for l in pick}
        best = max(abs(separable_slice_amplitude(n, ops, bits, fixed))
                   for bits in itertools.product(range(2), repeat=n))
        got = abs(separable_slice_amplitude(n, ops, dominant_bits(n, ops, fixed), fixed))
        assert got == pytest.approx(best, rel=1e-14)
