"""O1: brute-force state-vector simulator in complex128.

The amplitude <x|U|0...0> of Eq. 1 (Sec. 3.1.1) has a plain definition: apply
every gate of the circuit to the full state vector and read entry x.  The
state is an array of shape (2,)*n whose axis q is qubit q, so qubit 0 is the
most significant bit of a flat index.

A bit-string entry of -1 leaves that qubit open (Sec. 4.4): the result is
the 2^(#open) slice of the state with the other qubits fixed, open qubits in
ascending order, the first open qubit the most significant bit.

Parity pins (tests): norm 1; Bell, GHZ and cat closed forms; the paper's
60-qubit cat marginal slice (through the network oracle, since 2^60 entries
do not fit); QFT of a basis state; identity circuits; Porter-Thomas shape of
random-circuit outputs.
"""

from __future__ import annotations

from typing import Sequence

import numpy as np

from .gates import gate_matrix, is_channel


def apply_gate(psi: np.ndarray, U: np.ndarray, qubits: Sequence[int]) -> np.ndarray:
    """Apply a k-qubit matrix to axes ``qubits`` of psi (shape (2,)*n)."""
    k = len(qubits)
    Ut = U.reshape((2,) * (2 * k))
    out = np.tensordot(Ut, psi, axes=(list(range(k, 2 * k)), list(qubits)))
    return np.moveaxis(out, list(range(k)), list(qubits))


def simulate(n: int, ops) -> np.ndarray:
    """Final state of a noiseless circuit, shape (2,)*n."""
    psi = np.zeros((2,) * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    for op in ops:
        if is_channel(op.name):
            raise ValueError("noiseless simulator got a channel; use oracle.noise")
        psi = apply_gate(psi, gate_matrix(op.name, op.params), op.qubits)
    return psi


def amplitudes(n: int, ops, bits: Sequence[int]) -> np.ndarray:
    """Amplitude slice for one bit-string with entries 0, 1 or -1 (open)."""
    psi = simulate(n, ops)
    return slice_of(psi, bits)


def slice_of(psi: np.ndarray, bits: Sequence[int]) -> np.ndarray:
    idx = tuple(slice(None) if int(b) < 0 else int(b) for b in bits)
    return np.asarray(psi[idx]).reshape(-1)


def expect_z(psi: np.ndarray) -> np.ndarray:
    """<Z_q> for every qubit of a normalised state."""
    n = psi.ndim
    p = np.abs(psi) ** 2
    out = np.empty(n)
    for q in range(n):
        axes = tuple(a for a in range(n) if a != q)
        m = p.sum(axis=axes)
        out[q] = m[0] - m[1]
    return out
