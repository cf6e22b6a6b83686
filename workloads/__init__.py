"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This package only draws random choices (gate names, qubit pairs, bit values,
uniform numbers, tensor entries).  It holds none of the simulation
arithmetic: gate matrices, contraction, noise and truncation are each
implemented separately by the oracle and by the native library.
"""

from .circuits import (  # noqa: F401
    Op,
    grid_random_circuit,
    path_search_circuit,
    chain_random_circuit,
    cat_circuit,
    ghz_circuit,
    bell_circuit,
    qft_circuit,
    hh_circuit,
    noisy_ops,
    count_channel_events,
)
from .data import (  # noqa: F401
    random_bitstrings,
    random_complex,
    trajectory_uniforms,
    scorer_init,
)
