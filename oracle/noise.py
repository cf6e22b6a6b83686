"""O3: density-matrix simulator and O4: stochastic Kraus trajectories
(Sec. 3.3, Eq. 3: rho -> sum_k A_k rho A_k^dagger, with sum_k A_k^+ A_k = 1).

O3 applies gates as rho -> U rho U^dagger and channels by the Kraus sum.
O4 follows one pure state: after a channel it draws branch k with
probability p_k = |A_k psi|^2 / |psi|^2, using the caller's uniform u for that
event (k = first index with u < p_0 + ... + p_k; the last index if rounding
leaves none), then renormalises.  Uniforms are consumed one per channel event
in circuit order, so the native library can be driven by the same numbers.

Parity pins (tests): depolarising H-H chains give <Z> = (1 - 4p/3)^(2n); one
p reproduces the paper's printed noisy H-H curves (Sec. 4.2) to their printed
precision; amplitude damping of |1> gives <Z> = 1 - 2(1 - g)^m; the
trajectory mean agrees with O3 within its statistical error.
"""

from __future__ import annotations

import numpy as np

from .gates import gate_matrix, kraus_ops, is_channel
from .statevector import apply_gate, expect_z


def dm_simulate(n: int, ops) -> np.ndarray:
    """Final density matrix, shape (2,)*(2n): ket axes 0..n-1, bra n..2n-1."""
    rho = np.zeros((2,) * (2 * n), dtype=np.complex128)
    rho[(0,) * (2 * n)] = 1.0
    for op in ops:
        if is_channel(op.name):
            acc = np.zeros_like(rho)
            for K in kraus_ops(op.name, op.params):
                acc += _sandwich(rho, K, op.qubits, n)
            rho = acc
        else:
            rho = _sandwich(rho, gate_matrix(op.name, op.params), op.qubits, n)
    return rho


def _sandwich(rho, K, qubits, n):
    out = apply_gate(rho, K, list(qubits))                               # K on the ket
    return apply_gate(out, K.conj(), [n + q for q in qubits])            # conj(K) on the bra


def dm_expect_z(rho: np.ndarray, n: int) -> np.ndarray:
    d = 1 << n
    diag = np.real(np.diagonal(rho.reshape(d, d))).reshape((2,) * n)
    z = np.empty(n)
    for q in range(n):
        axes = tuple(a for a in range(n) if a != q)
        m = diag.sum(axis=axes)
        z[q] = (m[0] - m[1]) / diag.sum()
    return z


def trajectory(n: int, ops, uniforms, margins: list | None = None) -> tuple:
    """One trajectory: returns (final normalised state, branch list).  If
    `margins` is a list, the distance of each event's uniform from the
    nearest cumulative-probability boundary is appended to it (a small
    margin means a lower-precision run may pick the neighbouring branch)."""
    psi = np.zeros((2,) * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    e = 0
    branches = []
    for op in ops:
        if not is_channel(op.name):
            psi = apply_gate(psi, gate_matrix(op.name, op.params), op.qubits)
            continue
        u = float(uniforms[e])
        e += 1
        norm2 = float(np.sum(np.abs(psi) ** 2))
        cands = [apply_gate(psi, K, op.qubits) for K in kraus_ops(op.name, op.params)]
        probs = [float(np.sum(np.abs(c) ** 2)) / norm2 for c in cands]
        acc = 0.0
        k = len(probs) - 1
        for i, p in enumerate(probs):
            acc += p
            if u < acc:
                k = i
                break
        if margins is not None:
            cdf = np.cumsum(probs)[:-1]
            margins.append(float(np.min(np.abs(u - cdf))) if cdf.size else 1.0)
        branches.append(k)
        psi = cands[k] / np.sqrt(probs[k] * norm2)
    return psi, branches


def trajectories_expect_z(circuits, traj_per_circ: int, uniforms) -> np.ndarray:
    """<Z_q> of every trajectory; trajectory t = c * traj_per_circ + j runs
    circuit c with uniforms row t."""
    out = []
    for c, (n, ops) in enumerate(circuits):
        for j in range(traj_per_circ):
            psi, _ = trajectory(n, ops, uniforms[c * traj_per_circ + j])
            out.append(expect_z(psi))
    return np.array(out)
