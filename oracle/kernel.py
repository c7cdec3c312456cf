"""Electron-hole kernel of the lattice model (oracle).

Paper: Sec. "Two-particle electron-hole kernel", Eq. (sigma-from-k) defines
dSigma_{mnk} = sum K_{mnk,m'n'k'} rho_{m'n'k'}; Eq. (bse-direct-def) defines the
direct term  -sum_GG' M_{n1 n3} W_GG'(q) M*_{n2 n4}, q = k - k'.  Keeping only
G = G' = 0 and replacing the plane-wave matrix element by the overlap of the
periodic parts gives, per unit-cell area A = a^2 and N_k points,

    K_{(n m k),(n' m' k')} = -W(|q|) / (N_k A) * <n k|n' k'> <m' k'|m k>,

with the 2D Rytova-Keldysh screened interaction W(q) = 2 pi / (q (1 + r0 q)).
The q = 0 term is replaced by the average of W over the grid's square cell
around q = 0 (Appendix B: W(q=0) is replaced by an average over a small region
of the Brillouin zone).

Pair index p within a k point:
  block "all": p = n * nb + m  for every (n, m);
  block "eh" : p = (c - nv) * nv + v for conduction c, valence v (the
               conduction-valence block only).
Matrix index i = k * P + p (k-major).
"""

from __future__ import annotations

import numpy as np


def pair_table(nb: int, nv: int, block: str):
    """List of (row band, column band) of rho for each pair index p."""
    if block == "all":
        return [(n, m) for n in range(nb) for m in range(nb)]
    if block == "eh":
        return [(c, v) for c in range(nv, nb) for v in range(nv)]
    raise ValueError(block)


def rytova_keldysh(q, r0: float):
    """W(q) = 2 pi / (q (1 + r0 q)) for q > 0 (hartree * bohr^2)."""
    q = np.asarray(q, dtype=np.float64)
    return 2.0 * np.pi / (q * (1.0 + r0 * q))


def cell_average_w0(h: float, r0: float, nquad: int = 64) -> float:
    """Average of W over the square [-h, h]^2 around q = 0.

    In polar coordinates over the eight symmetric triangles of the square,
    avg = (1 / 4h^2) * 8 * int_0^{pi/4} int_0^{h sec t} W(q) q dq dt
        = (4 pi / (r0 h^2)) int_0^{pi/4} ln(1 + r0 h sec t) dt,
    evaluated with nquad-point Gauss-Legendre quadrature in t.
    """
    x, w = np.polynomial.legendre.leggauss(nquad)
    th = (np.pi / 8.0) * (x + 1.0)               # map [-1, 1] -> [0, pi/4]
    integrand = np.log1p(r0 * h / np.cos(th))
    integral = (np.pi / 8.0) * np.dot(w, integrand)
    return 4.0 * np.pi / (r0 * h * h) * integral


def fold_q(dk: np.ndarray, a: float) -> np.ndarray:
    """Fold a k difference per component into [-pi/a, pi/a) (minimum image)."""
    g = 2.0 * np.pi / a
    return dk - g * np.floor(dk / g + 0.5)


def coulomb_matrix(kpts: np.ndarray, nk1: int, nk2: int, a: float, r0: float) -> np.ndarray:
    """W(|fold(k_i - k_j)|) for every pair of grid points, W-bar at q = 0."""
    dq = fold_q(kpts[:, None, :] - kpts[None, :, :], a)
    q = np.sqrt((dq ** 2).sum(-1))
    w = np.empty_like(q)
    zero = q < 1e-12 * (2.0 * np.pi / a)
    w[~zero] = rytova_keldysh(q[~zero], r0)
    h = np.pi / (nk1 * a)
    if nk1 != nk2:
        raise ValueError("square grids only")
    w[zero] = cell_average_w0(h, r0)
    return w


def build_kernel(model, r0: float, block: str) -> np.ndarray:
    """Dense complex128 kernel K [N][N], N = N_k * P (see module docstring)."""
    nk, nb, nv = model.nk, model.nb, model.nv
    pairs = pair_table(nb, nv, block)
    pa = np.array([p[0] for p in pairs])
    pb = np.array([p[1] for p in pairs])
    w = coulomb_matrix(model.kpts, model.nk1, model.nk2, model.a, r0)
    # overlap O[k, k', n, n'] = <n k | n' k'> = sum_alpha conj(C_k[alpha, n]) C_k'[alpha, n']
    ov = np.einsum("kan,lam->klnm", model.evec.conj(), model.evec)
    # <n k|n' k'> for the row band a_p and column band a_p'
    first = ov[:, :, pa[:, None], pa[None, :]]            # [k][k'][p][p']
    # <m' k'|m k> = conj(<m k|m' k'>) for m = b_p, m' = b_p'
    second = ov[:, :, pb[:, None], pb[None, :]].conj()
    area = model.a * model.a
    kk = -(w / (nk * area))[:, :, None, None] * first * second
    npair = len(pairs)
    return np.ascontiguousarray(kk.transpose(0, 2, 1, 3).reshape(nk * npair, nk * npair))


def kernel_element(model, r0: float, block: str, i: int, j: int) -> complex:
    """One element K_ij computed on its own, for sampled checks at large sizes."""
    pairs = pair_table(model.nb, model.nv, block)
    npair = len(pairs)
    k, p = divmod(int(i), npair)
    kp, pp = divmod(int(j), npair)
    n, m = pairs[p]
    n2, m2 = pairs[pp]
    if k == kp:
        w = cell_average_w0(np.pi / (model.nk1 * model.a), r0)
    else:
        dq = fold_q(model.kpts[k] - model.kpts[kp], model.a)
        w = float(rytova_keldysh(np.sqrt((dq ** 2).sum()), r0))
    ck, ckp = model.evec[k], model.evec[kp]
    o1 = np.vdot(ck[:, n], ckp[:, n2])          # <n k | n' k'>
    o2 = np.vdot(ckp[:, m2], ck[:, m])          # <m' k' | m k>
    return complex(-w / (model.nk * model.a * model.a) * o1 * o2)
