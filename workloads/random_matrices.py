"""Seeded test matrices drawn for randomized algorithms (no method arithmetic)."""

from __future__ import annotations

import numpy as np


def gaussian_test_matrix(n: int, cols: int, seed: int) -> np.ndarray:
    """[n][cols] complex Gaussian with independent N(0, 1/2) real and
    imaginary parts, from PCG64(seed): real parts of all entries first, then
    imaginary parts (row-major order)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    re = rng.standard_normal((n, cols))
    im = rng.standard_normal((n, cols))
    return (re + 1j * im) / np.sqrt(2.0)
