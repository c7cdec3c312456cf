"""Reverse-mode derivative of the discrete RK4 propagation (oracle).

Not in the paper, which integrates forward only; this is the exact gradient
of the scheme of propagate.py (classical RK4 with the field at t_n,
t_n + dt/2 twice and t_n + dt), written out stage by stage, for a real loss
L that depends on the observable series:
  dL = sum_n gP_n dP_n + gJ_n dJ_n + gocc_n docc_n.
Complex gradients follow dL = Re sum conj(G) dZ, i.e. G = dL/dRe Z + i dL/dIm Z.

For f(t, y) = -i [H(t, y), y] with H = diag(eps) + dSigma(y - rho_eq) - E(t) D
and a cotangent g of f, the pullback is
  ybar  = i [H^H, g] + scatter(K^H sbar),  sbar = gather of Sbar = -i [y^H, g]
          (e-h block: sbar_cv = Sbar_cv + conj(Sbar_vc), the vc entries of
          dSigma being the conjugates of the cv entries),
  dL/dE(t) = Re sum conj(g) (i [D, y]),
and, for dSigma = K_diag o x + S (V^H x) with x = gather(y - rho_eq),
  dL/dS += sbar (V^H x)^H,  dL/dV^H += (S^H sbar) x^H.
With the intraband term of intraband.py, f gains -E(t) D(y), D = e_hat.(.)_{;k};
D is anti-self-adjoint for Re sum conj(a) b (the transport to k + b and back
to k - b are each other's adjoints, the central difference swaps them), so
  ybar += E(t) D(g),  dL/dE(t) += -Re sum conj(g) D(y).
The RK4 step rho' = rho + dt/6 (k1 + 2 k2 + 2 k3 + k4), k_s = f(t_s, y_s),
y_1 = rho, y_2 = rho + dt/2 k1, y_3 = rho + dt/2 k2, y_4 = rho + dt k3, is
pulled back from stage 4 to stage 1.  The pulse parameters enter through
E(t) = e0 exp(-(t - t0)^2 / (2 tau^2)) cos(omega t).
"""

from __future__ import annotations

import numpy as np

from .intraband import covariant_derivative
from .kernel import pair_table
from .propagate import LowRankOp, field_at, minus_i_commutator, rho_equilibrium


def field_param_derivs(t: float, fields, b: int) -> np.ndarray:
    """dE/d(e0, omega, tau, t0) at time t."""
    e0, w, tau, t0 = (float(fields.e0[b]), float(fields.omega[b]), float(fields.tau[b]), float(fields.t0[b]))
    g = np.exp(-(t - t0) ** 2 / (2.0 * tau * tau))
    c, s = np.cos(w * t), np.sin(w * t)
    return np.array([g * c, -e0 * g * t * s, e0 * g * c * (t - t0) ** 2 / tau ** 3, e0 * g * c * (t - t0) / tau ** 2])


def pull_commutator(h: np.ndarray, y: np.ndarray, g: np.ndarray):
    """Pullback of f = -i [H, y] (per k) for a cotangent g:
    (cotangent of y at fixed H, cotangent of H at fixed y) = (i [H^H, g], -i [y^H, g])."""
    hh = h.conj().transpose(0, 2, 1)
    yh = y.conj().transpose(0, 2, 1)
    return 1j * (hh @ g - g @ hh), -1j * (yh @ g - g @ yh)


def pull_field(dmat: np.ndarray, y: np.ndarray, g: np.ndarray) -> float:
    """dL/dE for f = -i [-E D, y] = i E [D, y]: Re sum conj(g) i [D, y]."""
    return float(np.sum((g.conj() * (1j * (dmat @ y - y @ dmat))).real))


def observable_cotangent(model, ex: float, ey: float, gp: float, gj: float, gocc: float) -> np.ndarray:
    """dL/drho_n for L = gp P_n + gj J_n + gocc occ_n (P, J, occ as in observables.py)."""
    d = ex * model.dip[0] + ey * model.dip[1]
    v = ex * model.vel[0] + ey * model.vel[1]
    # Re Tr(A rho) = Re sum conj(A^H) rho  ->  cotangent A^H
    g = gp * d.conj().transpose(0, 2, 1) + gj * v.conj().transpose(0, 2, 1)
    g = g.astype(np.complex128)
    g[:, model.nv, model.nv] += gocc
    return g / model.nk


def propagate_adjoint(model, op, block: str, fields, dt: float, gP=None, gJ=None, gocc=None,
                      instance: int = 0, nsteps: int | None = None, rho0: np.ndarray | None = None,
                      links: np.ndarray | None = None) -> dict:
    """Gradient of L = sum_n gP_n P_n + gJ_n J_n + gocc_n occ_n for one instance
    (links: the intraband term of propagate.propagate, or None).

    Returns dict(dE [nsteps][4] (dL/dE at the four stage times of each step),
    dfield [4] (dL/d e0, omega, tau, t0), drho0, and for a LowRankOp dus, dvh).
    """
    b = instance
    nsteps = int(fields.nsteps[b]) if nsteps is None else int(nsteps)
    zeros = np.zeros(nsteps + 1)
    gP = zeros if gP is None else np.asarray(gP, dtype=np.float64)
    gJ = zeros if gJ is None else np.asarray(gJ, dtype=np.float64)
    gocc = zeros if gocc is None else np.asarray(gocc, dtype=np.float64)
    pairs = pair_table(model.nb, model.nv, block)
    pa = np.array([p[0] for p in pairs])
    pb = np.array([p[1] for p in pairs])
    rho_eq = rho_equilibrium(model)
    h0 = np.zeros((model.nk, model.nb, model.nb), dtype=np.complex128)
    idx = np.arange(model.nb)
    h0[:, idx, idx] = model.eps
    ex, ey = float(fields.ex[b]), float(fields.ey[b])
    dmat = ex * model.dip[0] + ey * model.dip[1]
    lowrank = isinstance(op, LowRankOp)

    def gather(m):
        return m[:, pa, pb].reshape(-1)

    def delta_sigma(x):
        y = op.apply(x).reshape(model.nk, len(pairs))
        ds = np.zeros((model.nk, model.nb, model.nb), dtype=np.complex128)
        ds[:, pa, pb] = y
        if block == "eh":
            ds[:, pb, pa] = y.conj()
        return ds

    def hamiltonian(t, y):
        return h0 + delta_sigma(gather(y - rho_eq)) - field_at(t, fields, b) * dmat

    def rhs(t, y):
        f = minus_i_commutator(hamiltonian(t, y), y)
        if links is not None:
            f = f - field_at(t, fields, b) * covariant_derivative(model, links, y, ex, ey)
        return f

    def apply_adjoint(sbar):
        if lowrank:
            return op.kdiag.conj() * sbar + op.vh.conj().T @ (op.us.conj().T @ sbar)
        return op.k.conj().T @ sbar

    grads = {"dE": np.zeros((nsteps, 4)), "dfield": np.zeros(4)}
    if lowrank:
        grads["dus"] = np.zeros_like(op.us)
        grads["dvh"] = np.zeros_like(op.vh)

    def pullback(t, y, g, n, s):
        """Cotangent of y_s from the cotangent g of k_s = f(t, y_s)."""
        ybar, sig_bar = pull_commutator(hamiltonian(t, y), y, g)
        sbar = sig_bar[:, pa, pb]
        if block == "eh":
            sbar = sbar + sig_bar[:, pb, pa].conj()
        sbar = sbar.reshape(-1)
        xbar = apply_adjoint(sbar).reshape(model.nk, len(pairs))
        ybar[:, pa, pb] += xbar
        de = pull_field(dmat, y, g)
        if links is not None:
            e = field_at(t, fields, b)
            ybar += e * covariant_derivative(model, links, g, ex, ey)
            de -= float(np.sum((g.conj() * covariant_derivative(model, links, y, ex, ey)).real))
        grads["dE"][n, s] = de
        grads["dfield"] += de * field_param_derivs(t, fields, b)
        if lowrank:
            x = gather(y - rho_eq)
            z = op.vh @ x
            grads["dus"] += np.outer(sbar, z.conj())
            grads["dvh"] += np.outer(op.us.conj().T @ sbar, x.conj())
        return ybar

    # forward, keeping every state
    rho = rho_eq.copy() if rho0 is None else np.array(rho0, dtype=np.complex128)
    states = [rho]
    for n in range(nsteps):
        t = n * dt
        k1 = rhs(t, rho)
        k2 = rhs(t + 0.5 * dt, rho + (0.5 * dt) * k1)
        k3 = rhs(t + 0.5 * dt, rho + (0.5 * dt) * k2)
        k4 = rhs(t + dt, rho + dt * k3)
        rho = rho + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        states.append(rho)

    # backward
    abar = observable_cotangent(model, ex, ey, gP[nsteps], gJ[nsteps], gocc[nsteps])
    for n in range(nsteps - 1, -1, -1):
        t = n * dt
        rho = states[n]
        y1 = rho
        k1 = rhs(t, y1)
        y2 = rho + (0.5 * dt) * k1
        k2 = rhs(t + 0.5 * dt, y2)
        y3 = rho + (0.5 * dt) * k2
        k3 = rhs(t + 0.5 * dt, y3)
        y4 = rho + dt * k3
        g1, g2, g3, g4 = (dt / 6.0) * abar, (dt / 3.0) * abar, (dt / 3.0) * abar, (dt / 6.0) * abar
        acc = abar.copy()
        ybar = pullback(t + dt, y4, g4, n, 3)
        acc += ybar
        g3 = g3 + dt * ybar
        ybar = pullback(t + 0.5 * dt, y3, g3, n, 2)
        acc += ybar
        g2 = g2 + (0.5 * dt) * ybar
        ybar = pullback(t + 0.5 * dt, y2, g2, n, 1)
        acc += ybar
        g1 = g1 + (0.5 * dt) * ybar
        acc += pullback(t, y1, g1, n, 0)
        abar = acc + observable_cotangent(model, ex, ey, gP[n], gJ[n], gocc[n])
    grads["drho0"] = abar
    return grads


def harmonic_loss(j: np.ndarray, omega: float, dt: float, order: int = 3):
    """L = |m w dt sum_n J_n exp(-i m w t_n)|^2 (m = order): the intensity of the
    m-th harmonic of J, with the high-harmonic spectrum's definition.
    Returns (L, dL/dJ_n, explicit dL/domega at fixed J)."""
    m = float(order)
    t = np.arange(j.shape[0]) * dt
    ph = np.exp(-1j * m * omega * t)
    s = np.sum(j * ph)
    a = m * omega * dt * s
    loss = float(abs(a) ** 2)
    gj = 2.0 * (a.conj() * m * omega * dt * ph).real
    da_dw = m * dt * s + m * omega * dt * np.sum(j * ph * (-1j * m * t))
    gw = float(2.0 * (a.conj() * da_dw).real)
    return loss, gj, gw
