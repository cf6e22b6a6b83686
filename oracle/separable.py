"""Closed form for one slice of a circuit whose two-qubit gates are all the
identity (test infrastructure, like the rest of this package).

Such a circuit keeps every wire independent, so the network of Sec. 3.1
(same structure, labels and slicing as the general circuit of that shape)
contracts to a product of one factor per qubit.  Slicing (Sec. 3.3, Fig. 3)
fixes the value of some bond labels; a bond created by a two-qubit gate on
wire q carries the wire's basis value right after that gate (single-qubit
gates that follow fold into the next gate's input side), so fixing it to b
projects the wire's state onto |b> at that point.  The final bond of each
wire is its output leg, projected on the requested bit after the trailing
single-qubit gates.

Labels follow the network definition: each two-qubit gate on (a, b)
creates a's new label, then b's, in circuit order; wires with no two-qubit
gate get their single label after all gates, in qubit order.

Pins (tests): equals the generic oracle contraction of the network with the
same labels fixed, and the sum over all values of the fixed labels equals
the state-vector amplitude (a product state).
"""

from __future__ import annotations

from typing import Dict, Sequence

import numpy as np

from .gates import gate_matrix


def separable_slice_amplitude(n: int, ops, bits: Sequence[int], fixed: Dict[int, int]) -> complex:
    """<bits| C |0...0> restricted to the bond values in `fixed`
    (label -> 0/1), for a circuit whose two-qubit gates are identities."""
    state = [np.array([1.0, 0.0], dtype=np.complex128) for _ in range(n)]
    touched = [False] * n
    nxt = 0
    for op in ops:
        if len(op.qubits) == 1:
            q = op.qubits[0]
            state[q] = gate_matrix(op.name, op.params) @ state[q]
            continue
        U = gate_matrix(op.name, op.params)
        if np.abs(U - np.eye(4)).max() > 1e-15:
            raise ValueError("separable_slice_amplitude needs identity two-qubit gates")
        for q in op.qubits:
            touched[q] = True
            if nxt in fixed:
                b = fixed[nxt]
                keep = np.zeros(2, dtype=np.complex128)
                keep[b] = state[q][b]
                state[q] = keep
            nxt += 1
    amp = 1.0 + 0.0j
    for q in range(n):
        if not touched[q]:
            if nxt in fixed:
                raise ValueError("a lone wire's label is its output leg; it cannot be sliced")
            nxt += 1
        amp *= state[q][int(bits[q])]
    return complex(amp)


def dominant_bits(n: int, ops, fixed: Dict[int, int]):
    """The bit-string with the largest |slice value| for the given bond
    values: the product form lets each wire take its larger final component."""
    state = [np.array([1.0, 0.0], dtype=np.complex128) for _ in range(n)]
    nxt = 0
    for op in ops:
        if len(op.qubits) == 1:
            q = op.qubits[0]
            state[q] = gate_matrix(op.name, op.params) @ state[q]
            continue
        for q in op.qubits:
            if nxt in fixed:
                b = fixed[nxt]
                keep = np.zeros(2, dtype=np.complex128)
                keep[b] = state[q][b]
                state[q] = keep
            nxt += 1
    return [int(np.abs(state[q][1]) > np.abs(state[q][0])) for q in range(n)]
