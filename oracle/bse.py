"""Linear response of the TD-aGW equation = Bethe-Salpeter problem (oracle).

Paper, Sec. "Two-particle electron-hole kernel": in the linear-response limit
TD-aGW is equivalent to GW-BSE, whose exciton energies are the eigenvalues of
the non-interacting pair energies plus the kernel.  Linearising Eq. (tdagw)
around the diagonal equilibrium rho_eq (occupations f_n) gives, for each
pair (n, m) of a k point,

  i d(drho_nm)/dt = (e_n - e_m) drho_nm + (f_m - f_n) dSigma_nm
                    - E(t) (f_m - f_n) (e_hat . d)_nm .

Only pairs with f_n != f_m move at first order.  On that sector the operator
is L = diag(e_n - e_m) + diag(f_m - f_n) K restricted to the sector: the full
(resonant + anti-resonant) BSE Hamiltonian when all pairs are kept, and the
Tamm-Dancoff A = dE + K_eh for the conduction-valence block.  The solution
from drho(0) = 0 is drho(t) = -i int_0^t exp(-i L (t - s)) S E(s) ds with
S_nm = -(f_m - f_n) (e_hat . d)_nm, evaluated through the eigendecomposition
L = R diag(l) R^-1.
"""

from __future__ import annotations

import numpy as np

from .kernel import pair_table
from .propagate import field_at


def _occupations(model):
    f = np.zeros(model.nb)
    f[: model.nv] = 1.0
    return f


def linear_operator(model, k: np.ndarray, block: str):
    """L on the moving sector and the (k, n, m) label of each of its rows."""
    pairs = pair_table(model.nb, model.nv, block)
    npair = len(pairs)
    f = _occupations(model)
    sect = [p for p, (n, m) in enumerate(pairs) if f[n] != f[m]]
    rows = np.array([kk * npair + p for kk in range(model.nk) for p in sect])
    lab = np.array([(kk, pairs[p][0], pairs[p][1]) for kk in range(model.nk) for p in sect])
    kn, n, m = lab[:, 0], lab[:, 1], lab[:, 2]
    de = model.eps[kn, n] - model.eps[kn, m]
    w = f[m] - f[n]
    lmat = w[:, None] * k[np.ix_(rows, rows)]
    lmat[np.arange(len(rows)), np.arange(len(rows))] += de
    return lmat, lab


def _response_integrals(lam, fields, b, dt, nsteps, nodes: int = 16):
    """g_l(t_n) = int_0^{t_n} exp(-i l (t_n - s)) E(s) ds for n = 0..nsteps."""
    x, w = np.polynomial.legendre.leggauss(nodes)
    g = np.zeros((nsteps + 1, lam.shape[0]), dtype=np.complex128)
    prop = np.exp(-1j * lam * dt)
    for n in range(nsteps):
        t0 = n * dt
        s = t0 + 0.5 * dt * (x + 1.0)
        e = np.array([field_at(si, fields, b) for si in s])
        # int_{t_n}^{t_n+1} exp(-i l (t_{n+1} - s)) E(s) ds
        inc = 0.5 * dt * (np.exp(-1j * np.outer(t0 + dt - s, lam)) * (w * e)[:, None]).sum(0)
        g[n + 1] = prop * g[n] + inc
    return g


def sector_trace(drho: np.ndarray, a: np.ndarray, lab: np.ndarray, block: str) -> np.ndarray:
    """Re Tr(a drho) per time from the sector rows: sum of a_mn drho_nm over the
    rows (k, n, m); the conduction-valence block also carries the rows
    drho_vc = conj(drho_cv), whose terms a_cv conj(drho_cv) are the complex
    conjugates of the a_vc drho_cv terms (a Hermitian)."""
    kn, n, m = lab[:, 0], lab[:, 1], lab[:, 2]
    t = drho * a[kn, m, n][None, :]
    if block == "eh":
        t = t + t.conj()
    return t.sum(1).real


def linear_response(model, k: np.ndarray, block: str, fields, dt: float, nsteps: int,
                    instance: int = 0) -> dict:
    """First-order P(t), J(t) from the eigendecomposition of L; also its eigenvalues."""
    b = instance
    lmat, lab = linear_operator(model, k, block)
    f = _occupations(model)
    kn, n, m = lab[:, 0], lab[:, 1], lab[:, 2]
    ex, ey = float(fields.ex[b]), float(fields.ey[b])
    d = ex * model.dip[0] + ey * model.dip[1]
    v = ex * model.vel[0] + ey * model.vel[1]
    src = -(f[m] - f[n]) * d[kn, n, m]
    lam, rvec = np.linalg.eig(lmat)
    coef = np.linalg.solve(rvec, src)
    g = _response_integrals(lam, fields, b, dt, nsteps)
    drho = -1j * (g * coef[None, :]) @ rvec.T          # [t][row]
    j_eq = sum(v[:, i, i].sum() for i in range(model.nv)).real
    return {
        "P": sector_trace(drho, d, lab, block) / model.nk,
        "J": (sector_trace(drho, v, lab, block) + j_eq) / model.nk,
        "eig": lam,
        "drho": drho,
        "labels": lab,
    }
