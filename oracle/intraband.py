"""Intraband part of the field coupling (oracle).

Paper, Eq. (tdagw): the field enters as -e E(t).[r, rho] in the length gauge,
with r the position operator in the smooth (parallel-transport) gauge of
Appendix A.1.  The k-local part of r is the interband dipole matrix d (see
propagate.py); its intraband part acts on rho as a covariant derivative in k:
  [r_intra, rho]_k = i (rho)_{;k},
so with e = +1 the equation of motion gains
  d rho_k / dt  +=  -E(t) e_hat . (rho)_{;k}.

Reading of the covariant derivative on the uniform grid (the paper gives no
discretisation): a central difference over the periodic grid, after carrying
the neighbours' matrices into the gauge of k with link matrices,
  (rho)_{;a}(k) = [ L_a(k) rho(k + b_a) L_a(k)^H
                    - L_a(k - b_a)^H rho(k - b_a) L_a(k - b_a) ] / (2 |b_a|),
  |b_a| = 2 pi / (N_a a),
where L_a(k) is the parallel transport from k + b_a to k of the occupied and
of the empty subspace separately: the unitary polar factor of each diagonal
block (valence-valence, conduction-conduction) of the overlap
  M_a(k) = evec_k^H evec_{k + b_a},   M_nm = <n k | m k + b_a>,
and zero between the subspaces (the interband part of r is d).  The polar
factor of a block B = U s V^H is U V^H.  The links are unitary, so the total
charge sum_k Tr rho_k is conserved and rho_eq is left unchanged.
"""

from __future__ import annotations

import numpy as np


def _neighbour(model, axis: int, step: int) -> np.ndarray:
    """k index of k + step * b_axis for every k (k = i1 * nk2 + i2, periodic)."""
    i1, i2 = np.divmod(np.arange(model.nk), model.nk2)
    if axis == 0:
        i1 = (i1 + step) % model.nk1
    else:
        i2 = (i2 + step) % model.nk2
    return i1 * model.nk2 + i2


def polar_unitary(b: np.ndarray) -> np.ndarray:
    """Unitary polar factor U V^H of B = U s V^H."""
    u, _, vh = np.linalg.svd(b)
    return u @ vh


def transport_links(model) -> np.ndarray:
    """Links L[a][k] (a = x, y): block-diagonal polar factors of
    evec_k^H evec_{k + b_a}, complex128 [2][nk][nb][nb]."""
    nv = model.nv
    links = np.zeros((2, model.nk, model.nb, model.nb), dtype=np.complex128)
    for a in range(2):
        fwd = _neighbour(model, a, +1)
        for k in range(model.nk):
            m = model.evec[k].conj().T @ model.evec[fwd[k]]
            links[a, k, :nv, :nv] = polar_unitary(m[:nv, :nv])
            links[a, k, nv:, nv:] = polar_unitary(m[nv:, nv:])
    return links


def grid_spacing(model, axis: int) -> float:
    """|b_a| = 2 pi / (N_a a)."""
    n = model.nk1 if axis == 0 else model.nk2
    return 2.0 * np.pi / (n * model.a)


def covariant_derivative(model, links: np.ndarray, y: np.ndarray, ex: float, ey: float) -> np.ndarray:
    """e_hat . (y)_{;k} for a per-k matrix field y [nk][nb][nb]."""
    out = np.zeros_like(y)
    for a, e in ((0, ex), (1, ey)):
        if e == 0.0:
            continue
        fwd = _neighbour(model, a, +1)
        bwd = _neighbour(model, a, -1)
        lf = links[a]
        lb = links[a][bwd]
        lfh = lf.conj().transpose(0, 2, 1)
        lbh = lb.conj().transpose(0, 2, 1)
        diff = lf @ y[fwd] @ lfh - lbh @ y[bwd] @ lb
        out += (e / (2.0 * grid_spacing(model, a))) * diff
    return out
