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


def hermitian_lowrank_factors(n: int, rank: int, scale: float, diag: float, seed: int):
    """Seeded factors of a Hermitian rank-r operator K = K_diag + S V^H:
    G [n][r] complex Gaussian / sqrt(n) from gaussian_test_matrix, lambda_j drawn
    uniformly from [-scale, scale] (after G, same generator family, seed + 1),
    S = G diag(lambda), V^H = G^H, K_diag = diag (a constant).  Returns
    (kdiag [n], S [n][r], V^H [r][n]) as complex128 arrays."""
    g = gaussian_test_matrix(n, rank, seed) / np.sqrt(n)
    lam = np.random.Generator(np.random.PCG64(seed + 1)).uniform(-scale, scale, size=rank)
    return (np.full(n, diag, dtype=np.complex128), np.ascontiguousarray(g * lam[None, :]),
            np.ascontiguousarray(g.conj().T))
