"""Seeded bit-strings, complex tensors and uniforms (no simulation arithmetic)."""

from __future__ import annotations

from typing import Sequence

import numpy as np


def random_bitstrings(n_strings: int, n_qubits: int, seed: int) -> np.ndarray:
    """Uniform 0/1 bit-strings, shape (n_strings, n_qubits), int8, indexed by qubit."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2, size=(n_strings, n_qubits), dtype=np.int8)


def random_complex(shape: Sequence[int], seed: int, scale: float = 1.0,
                   dtype=np.complex128) -> np.ndarray:
    """I.i.d. complex normal entries with unit variance (times ``scale``)."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(size=tuple(shape))
    im = rng.standard_normal(size=tuple(shape))
    z = (re + 1j * im) * (scale / np.sqrt(2.0))
    return z.astype(dtype)


def trajectory_uniforms(n_traj: int, n_events: int, seed: int) -> np.ndarray:
    """Uniforms in [0, 1) for channel branch choices, shape (n_traj, n_events).

    Row t feeds trajectory t; column e is consumed by its e-th channel event in
    circuit order.
    """
    rng = np.random.default_rng(seed)
    return rng.random(size=(n_traj, max(n_events, 1)))


def scorer_init(n_params_by_shape, seed: int) -> np.ndarray:
    """Initial parameters of the contraction-order scorer: each weight matrix
    (fan_in, fan_out) drawn N(0, 2 / fan_in), biases zero; flattened in the
    given order.  ``n_params_by_shape`` is a list of (name, shape)."""
    rng = np.random.default_rng(seed)
    out = []
    for name, shp in n_params_by_shape:
        if len(shp) == 2:
            out.append(rng.standard_normal(shp).reshape(-1) * np.sqrt(2.0 / shp[0]))
        elif name == "wo":
            out.append(rng.standard_normal(shp) * np.sqrt(1.0 / shp[0]))
        else:
            out.append(np.zeros(shp))
    return np.concatenate(out).astype(np.float64)
