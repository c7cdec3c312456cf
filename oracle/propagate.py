"""RK4 integration of the TD-aGW equation of motion (oracle).

Paper, Eq. (tdagw): i d rho_k / dt = [H^QP + dSigma(t) - e E(t).r, rho]_k,
with dSigma from Eq. (sigma-from-k) applied to the non-equilibrium change of
rho (dSigma = K . (rho - rho_eq)); Eq. (svd_acc) replaces K by
K_diag + S~ V~^H, applied as K_diag o x + S~ (V~^H x).
Readings where the paper is silent:
  * e = +1, so the field term of the Hamiltonian is -E(t) e_hat . d_k;
  * rho_eq is diagonal with 1 on valence and 0 on conduction bands;
  * kernel restricted to the conduction-valence block: dSigma_cv = (K_eh x)_cv,
    dSigma_vc = conj(dSigma_cv), dSigma_cc = dSigma_vv = 0;
  * the integrator, which the paper does not name, is classical RK4 with the
    field evaluated at t_n, t_n + dt/2 (twice) and t_n + dt; t_n = n dt.
With transport links (intraband.py) the field also acts through the
intraband part of r: d rho_k/dt gains -E(t) e_hat . (rho)_{;k}.
"""

from __future__ import annotations

import numpy as np

from .intraband import covariant_derivative
from .kernel import pair_table
from .observables import observables


def field_at(t: float, fields, b: int) -> float:
    """E_b(t) = E0 exp(-(t - t0)^2 / (2 tau^2)) cos(omega t)."""
    return float(fields.e0[b] * np.exp(-(t - fields.t0[b]) ** 2 / (2.0 * fields.tau[b] ** 2))
                 * np.cos(fields.omega[b] * t))


class DenseOp:
    """dSigma = K x (Eq. sigma-from-k)."""

    def __init__(self, k: np.ndarray):
        self.k = k

    def apply(self, x: np.ndarray) -> np.ndarray:
        return self.k @ x


class LowRankOp:
    """dSigma = K_diag o x + S~ (V~^H x) (Eq. svd_acc)."""

    def __init__(self, kdiag: np.ndarray, us: np.ndarray, vh: np.ndarray):
        self.kdiag, self.us, self.vh = kdiag, us, vh

    @staticmethod
    def from_factors(f: dict) -> "LowRankOp":
        return LowRankOp(f["kdiag"], f["US"], f["Vh"])

    def apply(self, x: np.ndarray) -> np.ndarray:
        return self.kdiag * x + self.us @ (self.vh @ x)


class ChannelOp:
    """dSigma with channel-wise factors (Eq. svd-channel-wise): pair p of k
    receives sum_k' K^{pp}[k, k'] x[k' P + p] + sum_{q != p} S^{pq} (V^{pq H} x_q)[k],
    x_q = x[q::P] (channel blocks of the k-major pair index)."""

    def __init__(self, factors: dict, nk: int, npair: int):
        self.f, self.nk, self.npair = factors, nk, npair

    def apply(self, x: np.ndarray) -> np.ndarray:
        P = self.npair
        xs = x.reshape(self.nk, P)
        y = np.zeros_like(xs)
        for p in range(P):
            y[:, p] = self.f["diag"][p] @ xs[:, p]
            for q in range(P):
                if q != p:
                    s, vh, _ = self.f["off"][(p, q)]
                    y[:, p] += s @ (vh @ xs[:, q])
        return y.reshape(-1)


def minus_i_commutator(h: np.ndarray, rho: np.ndarray) -> np.ndarray:
    """-i [H, rho] per k point."""
    return -1j * (h @ rho - rho @ h)


def rho_equilibrium(model) -> np.ndarray:
    occ = np.zeros(model.nb)
    occ[: model.nv] = 1.0
    return np.broadcast_to(np.diag(occ).astype(np.complex128), (model.nk, model.nb, model.nb)).copy()


def propagate(model, op, block: str, fields, dt: float, instance: int = 0,
              nsteps: int | None = None, rho0: np.ndarray | None = None, links: np.ndarray | None = None) -> dict:
    """Integrate one field instance; observables at t_0 .. t_nsteps.
    links: transport links of intraband.transport_links, or None for the
    k-local field coupling only.

    Returns dict(P, J, occ, tr, herm: [nsteps + 1] arrays, rho: final state).
    """
    b = instance
    nsteps = int(fields.nsteps[b]) if nsteps is None else int(nsteps)
    pairs = pair_table(model.nb, model.nv, block)
    pa = np.array([p[0] for p in pairs])
    pb = np.array([p[1] for p in pairs])
    rho_eq = rho_equilibrium(model)
    h0 = np.zeros((model.nk, model.nb, model.nb), dtype=np.complex128)
    idx = np.arange(model.nb)
    h0[:, idx, idx] = model.eps
    ex, ey = float(fields.ex[b]), float(fields.ey[b])
    dfield = ex * model.dip[0] + ey * model.dip[1]

    def delta_sigma(drho):
        x = drho[:, pa, pb].reshape(-1)
        y = op.apply(x).reshape(model.nk, len(pairs))
        ds = np.zeros_like(drho)
        ds[:, pa, pb] = y
        if block == "eh":
            ds[:, pb, pa] = y.conj()
        return ds

    def rhs(t, rho):
        e = field_at(t, fields, b)
        h = h0 + delta_sigma(rho - rho_eq) - e * dfield
        f = minus_i_commutator(h, rho)
        if links is not None:
            f = f - e * covariant_derivative(model, links, rho, ex, ey)
        return f

    rho = rho_eq.copy() if rho0 is None else np.array(rho0, dtype=np.complex128)
    out = {key: np.zeros(nsteps + 1) for key in ("P", "J", "occ", "tr", "herm")}

    def record(n, r):
        o = observables(model, r, ex, ey, grid_trace=links is not None)
        for key in out:
            out[key][n] = o[key]

    record(0, rho)
    for n in range(nsteps):
        t = n * dt
        k1 = rhs(t, rho)
        k2 = rhs(t + 0.5 * dt, rho + (0.5 * dt) * k1)
        k3 = rhs(t + 0.5 * dt, rho + (0.5 * dt) * k2)
        k4 = rhs(t + dt, rho + dt * k3)
        rho = rho + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        record(n + 1, rho)
    out["rho"] = rho
    return out
