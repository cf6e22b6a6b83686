"""Expectation values of Pauli strings (Sec. 3.1, operator expectation values:
Eq. 2 and the two methods of Table 1).  Test infrastructure, like the rest of
this package.

<P> = <Psi|P|Psi> with Psi = C|0...0> has a plain definition on the O1 state
vector: apply P's one-qubit factors to Psi and take the inner product with
Psi.  The paper's two ways of reaching it are written out beside it, each
from its own statement:

* conjugate (double-depth) network: <0...0| C^dagger P C |0...0>, i.e. apply
  C, then P, then the adjoints of C's gates in reverse order, and read entry
  0.  A tensor contracted directly with its own conjugate drops out; walking
  C backwards from P's support, a gate whose qubits are all outside the
  support grown so far commutes past everything later and meets its
  conjugate, so only the gates in P's backward light cone are applied.
* density matrix (Sec. 3.3, Eq. 3): for a circuit with noise channels,
  Tr(rho P) with rho from the O3 density-matrix simulator; for a noiseless
  circuit it equals <Psi|P|Psi>.
* wave-function slicing: fix the projected qubits to every assignment s,
  take the open slice psi_s of the state, and sum <psi_s|P_open|psi_s>; a Z
  factor on a projected qubit gives slice s the sign (-1)^{s_q}; X and Y
  factors must act on open qubits.

A Pauli string is a sequence of codes 0 (I), 1 (X), 2 (Y), 3 (Z), one per
qubit, or a string such as "IZZI".

Pins (tests): GHZ closed forms (<Z_i Z_j> = 1, <Z_i> = 0, <X...X> = 1,
<YYXX> = -1); one-qubit rotations of |0> (R_X(pi/2) gives <Y> = -1, R_Y(pi/2)
gives <X> = 1, S H gives <Y> = 1); the conjugate-network value with and
without the light-cone collapse and the sliced value all equal the direct
definition on random circuits; <I...I> = 1; values of Hermitian strings are
real and lie in [-1, 1]; Tr(rho P) of a noiseless circuit equals the
pure-state value, and a depolarising H-H chain follows its closed form.
"""

from __future__ import annotations

import itertools
from typing import List, Sequence

import numpy as np

from .gates import PAULIS, gate_matrix
from .noise import dm_simulate
from .statevector import apply_gate, simulate

CODES = {"I": 0, "X": 1, "Y": 2, "Z": 3}


def pauli_codes(n: int, pauli) -> List[int]:
    if isinstance(pauli, str):
        codes = [CODES[c] for c in pauli.upper()]
    else:
        codes = [int(c) for c in pauli]
    if len(codes) != n or any(c < 0 or c > 3 for c in codes):
        raise ValueError("a Pauli string needs one code 0..3 per qubit")
    return codes


def apply_pauli(psi: np.ndarray, codes: Sequence[int]) -> np.ndarray:
    """P |psi> for a state of shape (2,)*n."""
    out = psi
    for q, c in enumerate(codes):
        if c:
            out = apply_gate(out, PAULIS[c], [q])
    return out


def expectation(n: int, ops, pauli) -> complex:
    """<Psi|P|Psi> from the full state vector (the definition, Eq. 2)."""
    codes = pauli_codes(n, pauli)
    psi = simulate(n, ops)
    return complex(np.vdot(psi.reshape(-1), apply_pauli(psi, codes).reshape(-1)))


def light_cone(n: int, ops, pauli) -> List[int]:
    """Indices of C's ops in the backward light cone of P's support."""
    live = [c != 0 for c in pauli_codes(n, pauli)]
    kept = []
    for k in range(len(ops) - 1, -1, -1):
        qs = ops[k].qubits
        if any(live[q] for q in qs):
            kept.append(k)
            for q in qs:
                live[q] = True
    return sorted(kept)


def conjugate_network_value(n: int, ops, pauli, collapse: bool = True) -> complex:
    """<0|C^dagger P C|0> evaluated gate by gate on the state vector."""
    codes = pauli_codes(n, pauli)
    idx = light_cone(n, ops, codes) if collapse else list(range(len(ops)))
    psi = np.zeros((2,) * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    for k in idx:
        psi = apply_gate(psi, gate_matrix(ops[k].name, ops[k].params), ops[k].qubits)
    psi = apply_pauli(psi, codes)
    for k in reversed(idx):
        U = gate_matrix(ops[k].name, ops[k].params)
        psi = apply_gate(psi, U.conj().T, ops[k].qubits)
    return complex(psi[(0,) * n])


def sliced_expectation(n: int, ops, pauli, open_qubits: Sequence[int]) -> complex:
    """Sum over the projected qubits' assignments of <psi_s|P_open|psi_s>."""
    codes = pauli_codes(n, pauli)
    open_q = sorted(int(q) for q in open_qubits)
    proj = [q for q in range(n) if q not in open_q]
    if any(codes[q] in (1, 2) for q in proj):
        raise ValueError("X and Y factors must act on open qubits")
    psi = simulate(n, ops)
    open_codes = [codes[q] for q in open_q]
    total = 0j
    for vals in itertools.product((0, 1), repeat=len(proj)):
        idx = [slice(None)] * n
        sign = 1.0
        for q, v in zip(proj, vals):
            idx[q] = v
            if codes[q] == 3 and v == 1:
                sign = -sign
        s = np.asarray(psi[tuple(idx)])
        if s.ndim == 0:
            total += sign * abs(complex(s)) ** 2
            continue
        total += sign * np.vdot(s.reshape(-1), apply_pauli(s, open_codes).reshape(-1))
    return complex(total)


def dm_expectation(n: int, ops, pauli) -> complex:
    """Tr(rho P) of the O3 density matrix (ket axes 0..n-1, bra n..2n-1)."""
    codes = pauli_codes(n, pauli)
    rho = dm_simulate(n, ops)
    d = 1 << n
    prho = apply_pauli(rho, codes + [0] * n)      # P acting on the ket index: (P rho)
    return complex(np.trace(prho.reshape(d, d)))
