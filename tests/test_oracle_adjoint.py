"""Pins of the oracle's reverse-mode derivative: central finite differences of
the oracle's own forward propagation (a different computation: no pullback
formula is involved), for the pulse parameters, the low-rank factors and the
initial state, on dense and low-rank operators and both kernel blocks."""

import numpy as np
import pytest

import oracle as O
from workloads import FS_AU, HARTREE_EV, FieldTable, dirac_model, tb4_model
from workloads.configs import R0_STABLE

A = 6.0
DT = 0.2 * FS_AU
NSTEPS = 40


def _fields(e0=8e-3, omega_ev=1.2, tau_fs=2.0, t0_fs=4.0):
    return FieldTable.single(e0, omega_ev / HARTREE_EV, tau_fs * FS_AU, t0_fs * FS_AU, NSTEPS)


def _weights(seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(NSTEPS + 1), rng.standard_normal(NSTEPS + 1), rng.standard_normal(NSTEPS + 1)


def _loss(model, op, block, fields, w, rho0=None, links=None):
    r = O.propagate(model, op, block, fields, DT, rho0=rho0, links=links)
    return float(np.dot(w[0], r["P"]) + np.dot(w[1], r["J"]) + np.dot(w[2], r["occ"]))


def _with(fields, name, value):
    f = FieldTable(fields.e0.copy(), fields.omega.copy(), fields.tau.copy(), fields.t0.copy(),
                   fields.ex, fields.ey, fields.nsteps)
    getattr(f, name)[0] = value
    return f


@pytest.fixture(scope="module")
def tb4_4():
    return tb4_model(4, A, 0.5)


@pytest.fixture(scope="module")
def lowrank_tb4(tb4_4):
    return O.LowRankOp.from_factors(O.compress(O.build_kernel(tb4_4, R0_STABLE, "eh"), "rank", 12))


def _check_field_params(model, op, block, fields, w, grads, links=None):
    for i, name in enumerate(("e0", "omega", "tau", "t0")):
        v = float(getattr(fields, name)[0])
        h = 1e-5 * abs(v)
        fd = (_loss(model, op, block, _with(fields, name, v + h), w, links=links)
              - _loss(model, op, block, _with(fields, name, v - h), w, links=links)) / (2 * h)
        assert abs(grads["dfield"][i] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(grads["dfield"]).max()), name


def test_adjoint_field_params_lowrank_eh(tb4_4, lowrank_tb4):
    f = _fields()
    w = _weights(1)
    g = O.propagate_adjoint(tb4_4, lowrank_tb4, "eh", f, DT, *w)
    _check_field_params(tb4_4, lowrank_tb4, "eh", f, w, g)


def test_adjoint_field_params_dense_all_pairs():
    m = dirac_model(4, 1.0, 1.5, A, 0.5)
    op = O.DenseOp(O.build_kernel(m, R0_STABLE, "all"))
    f = _fields(e0=2e-2, omega_ev=2.0)
    w = _weights(2)
    g = O.propagate_adjoint(m, op, "all", f, DT, *w)
    _check_field_params(m, op, "all", f, w, g)


def _directional(fun, base, direction, eps):
    return (fun(base + eps * direction) - fun(base - eps * direction)) / (2 * eps)


def test_adjoint_lowrank_factors_and_initial_state(tb4_4, lowrank_tb4):
    f = _fields()
    w = _weights(3)
    op = lowrank_tb4
    g = O.propagate_adjoint(tb4_4, op, "eh", f, DT, *w)
    rng = np.random.default_rng(4)

    def cplx(shape):
        return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)

    d_us = cplx(op.us.shape)
    fd = _directional(lambda us: _loss(tb4_4, O.LowRankOp(op.kdiag, us, op.vh), "eh", f, w), op.us, d_us,
                      1e-6 * np.abs(op.us).max())
    assert abs(np.sum((g["dus"].conj() * d_us).real) - fd) <= 1e-6 * abs(fd)
    d_vh = cplx(op.vh.shape)
    fd = _directional(lambda vh: _loss(tb4_4, O.LowRankOp(op.kdiag, op.us, vh), "eh", f, w), op.vh, d_vh,
                      1e-6 * np.abs(op.vh).max())
    assert abs(np.sum((g["dvh"].conj() * d_vh).real) - fd) <= 1e-6 * abs(fd)
    rho_eq = O.rho_equilibrium(tb4_4)
    d_rho = cplx(rho_eq.shape)
    d_rho = 0.5 * (d_rho + d_rho.conj().transpose(0, 2, 1))
    fd = _directional(lambda r0: _loss(tb4_4, op, "eh", f, w, rho0=r0), rho_eq, d_rho, 1e-6)
    assert abs(np.sum((g["drho0"].conj() * d_rho).real) - fd) <= 1e-6 * abs(fd)


def test_harmonic_loss_gradient(tb4_4, lowrank_tb4):
    """Third-harmonic intensity of J: d/d omega through the dynamics (adjoint)
    plus the explicit dependence of the harmonic frequency."""
    f = _fields(e0=2e-2, omega_ev=0.8)

    def total(fields):
        r = O.propagate(tb4_4, lowrank_tb4, "eh", fields, DT)
        return O.harmonic_loss(r["J"], float(fields.omega[0]), DT)

    loss, gj, gw = total(f)
    g = O.propagate_adjoint(tb4_4, lowrank_tb4, "eh", f, DT, gJ=gj)
    grad = g["dfield"].copy()
    grad[1] += gw
    for i, name in enumerate(("e0", "omega", "tau", "t0")):
        v = float(getattr(f, name)[0])
        h = 1e-5 * abs(v)
        fd = (total(_with(f, name, v + h))[0] - total(_with(f, name, v - h))[0]) / (2 * h)
        assert abs(grad[i] - fd) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(grad).max()), name


def test_adjoint_with_intraband_term(tb4_4, lowrank_tb4):
    """The intraband (covariant k-derivative) term: field parameters and the
    initial state against central differences, field along (0.6, 0.8)."""
    f = FieldTable.single(8e-3, 1.2 / HARTREE_EV, 2.0 * FS_AU, 4.0 * FS_AU, NSTEPS, ex=0.6, ey=0.8)
    w = _weights(7)
    links = O.transport_links(tb4_4)
    g = O.propagate_adjoint(tb4_4, lowrank_tb4, "eh", f, DT, *w, links=links)
    g_local = O.propagate_adjoint(tb4_4, lowrank_tb4, "eh", f, DT, *w)
    assert np.abs(g["dfield"] - g_local["dfield"]).max() > 1e-3 * np.abs(g["dfield"]).max()  # the term matters
    _check_field_params(tb4_4, lowrank_tb4, "eh", f, w, g, links=links)
    rng = np.random.default_rng(8)
    rho_eq = O.rho_equilibrium(tb4_4)
    d_rho = rng.standard_normal(rho_eq.shape) + 1j * rng.standard_normal(rho_eq.shape)
    d_rho = 0.5 * (d_rho + d_rho.conj().transpose(0, 2, 1))
    fd = _directional(lambda r0: _loss(tb4_4, lowrank_tb4, "eh", f, w, rho0=r0, links=links), rho_eq, d_rho, 1e-6)
    assert abs(np.sum((g["drho0"].conj() * d_rho).real) - fd) <= 1e-6 * abs(fd)
