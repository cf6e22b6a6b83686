"""Bit-string sampling from a marginal wave-function slice (Sec. 4.4 computes
such slices; Table 1 lists sampling from partial state vectors as a mode).
Test infrastructure, like the rest of this package.

A slice psi (2^k amplitudes, the other qubits projected) defines the
conditional distribution p_x = |psi_x|^2 / sum |psi|^2.  A draw at a uniform
u in [0, 1) is the inverse of its cumulative distribution: the first index k
with C(k) > u * C(last), C the running sum of |psi|^2 in index order (FP64).

Pins (tests): a point mass always returns its index; two outcomes with
weights a and 1 - a return the first exactly when u < a; a uniform slice of
2^k entries returns floor(u * 2^k) for dyadic u away from the boundaries;
sample frequencies of many draws match p within a chi-square bound.
"""

from __future__ import annotations

import numpy as np


def cumulative(psi) -> np.ndarray:
    p = np.abs(np.asarray(psi, dtype=np.complex128).reshape(-1)) ** 2
    return np.cumsum(p)


def sample_indices(psi, uniforms) -> np.ndarray:
    """First k with C(k) > u * C(last), for every uniform u."""
    C = cumulative(psi)
    u = np.asarray(uniforms, dtype=np.float64).reshape(-1)
    return np.searchsorted(C, u * C[-1], side="right").astype(np.int64)
