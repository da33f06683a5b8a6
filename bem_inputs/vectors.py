"""Seeded input vectors (densities, right-hand sides, plane-wave directions)."""

from __future__ import annotations

import numpy as np


def random_vector(n: int, seed: int, nrhs: int = 1, complex_: bool = False) -> np.ndarray:
    """Standard-normal entries, shape [nrhs, n]; complex draws real then imaginary parts."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((nrhs, n))
    if complex_:
        x = x + 1j * rng.standard_normal((nrhs, n))
    return x


def random_directions(count: int, seed: int) -> np.ndarray:
    """Unit vectors g/|g| with g ~ N(0, I3), shape [count, 3]."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((count, 3))
    return g / np.linalg.norm(g, axis=1)[:, None]
