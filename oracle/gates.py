"""Gate and channel matrices (complex128), built from their names.

Conventions
    * matrices are row = output, column = input;
    * a two-qubit matrix acts on |a b> with the op's first qubit a as the
      more significant bit;
    * sqrt_x, sqrt_y, sqrt_w are half-turn-halved rotations
      R_P(pi/2) = cos(pi/4) I - i sin(pi/4) P with P = X, Y and
      W = (X + Y)/sqrt(2);
    * fsim(theta, phi) mixes |01> and |10> with cos(theta) on the diagonal and
      -i sin(theta) off it, and puts exp(-i phi) on |11>;
    * cphase(phi) puts exp(i phi) on |11>.

Kraus sets (the order fixes which uniform interval selects which branch)
    depol1(p): sqrt(1-p) I, sqrt(p/3) X, sqrt(p/3) Y, sqrt(p/3) Z
    depol2(p): sqrt(1-p) II, then sqrt(p/15) P(x)Q for the 15 non-identity
               pairs, P the more significant, both running over I, X, Y, Z
    amp_damp(g): [[1,0],[0,sqrt(1-g)]], [[0,sqrt(g)],[0,0]]
These satisfy sum_k A_k^dagger A_k = 1 (Sec. 3.3, Eq. 3); the pin is a test.

Parity pins: unitarity, Kraus completeness, and the Bell, GHZ, QFT and cat
closed forms reached through the state-vector simulator.
"""

from __future__ import annotations

import math

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
PAULIS = (I2, X, Y, Z)


def _rot(P: np.ndarray, theta: float) -> np.ndarray:
    return math.cos(theta / 2) * I2 - 1j * math.sin(theta / 2) * P


def gate_matrix(name: str, params=()) -> np.ndarray:
    """Unitary of a named gate (2x2 or 4x4, complex128)."""
    if name == "sqrt_x":
        return _rot(X, math.pi / 2)
    if name == "sqrt_y":
        return _rot(Y, math.pi / 2)
    if name == "sqrt_w":
        W = (X + Y) / math.sqrt(2.0)
        return _rot(W, math.pi / 2)
    if name == "h":
        return np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)
    if name == "x":
        return X.copy()
    if name == "y":
        return Y.copy()
    if name == "z":
        return Z.copy()
    if name == "s":
        return np.diag([1, 1j]).astype(np.complex128)
    if name == "t":
        return np.diag([1, np.exp(1j * math.pi / 4)]).astype(np.complex128)
    if name == "rz":
        (phi,) = params
        return np.diag([np.exp(-0.5j * phi), np.exp(0.5j * phi)]).astype(np.complex128)
    if name == "cz":
        return np.diag([1, 1, 1, -1]).astype(np.complex128)
    if name == "cx":
        U = np.zeros((4, 4), dtype=np.complex128)
        U[0, 0] = U[1, 1] = 1
        U[2, 3] = U[3, 2] = 1
        return U
    if name == "swap":
        U = np.zeros((4, 4), dtype=np.complex128)
        U[0, 0] = U[3, 3] = 1
        U[1, 2] = U[2, 1] = 1
        return U
    if name == "cphase":
        (phi,) = params
        return np.diag([1, 1, 1, np.exp(1j * phi)]).astype(np.complex128)
    if name == "fsim":
        theta, phi = params
        c, s = math.cos(theta), math.sin(theta)
        U = np.zeros((4, 4), dtype=np.complex128)
        U[0, 0] = 1
        U[1, 1] = U[2, 2] = c
        U[1, 2] = U[2, 1] = -1j * s
        U[3, 3] = np.exp(-1j * phi)
        return U
    raise KeyError(f"unknown gate {name!r}")


def kraus_ops(name: str, params=()) -> list:
    """Kraus operators of a named channel, in branch order."""
    if name == "depol1":
        (p,) = params
        ops = [math.sqrt(1 - p) * I2]
        ops += [math.sqrt(p / 3) * P for P in (X, Y, Z)]
        return ops
    if name == "depol2":
        (p,) = params
        ops = [math.sqrt(1 - p) * np.eye(4, dtype=np.complex128)]
        for a in range(4):
            for b in range(4):
                if a == 0 and b == 0:
                    continue
                ops.append(math.sqrt(p / 15) * np.kron(PAULIS[a], PAULIS[b]))
        return ops
    if name == "amp_damp":
        (g,) = params
        return [np.array([[1, 0], [0, math.sqrt(1 - g)]], dtype=np.complex128),
                np.array([[0, math.sqrt(g)], [0, 0]], dtype=np.complex128)]
    raise KeyError(f"unknown channel {name!r}")


def is_channel(name: str) -> bool:
    return name in ("depol1", "depol2", "amp_damp")
