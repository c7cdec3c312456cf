"""Pins of the oracle's intraband field coupling (covariant k-derivative with
parallel-transport links) against facts other than the oracle itself:

* the polar factor's defining properties (unitary, L^H B Hermitian positive
  definite) and the links' block structure;
* the semi-discrete drift equation d y/dt = -E(t) e.D y - i (e_n - e_m) y on a
  periodic grid, solved exactly mode by mode with the FFT (the central
  difference multiplies exp(i q i) by i sin(q) / |b|);
* a population packet moves by A(t) = int E dt in k (force +E for e = +1);
* gauge covariance: the same physics in rotated Bloch bases (per-k unitaries
  within the degenerate valence and conduction subspaces, or per-band phases)
  gives the same gauge-invariant observables and the rotated density matrix;
* conservation of the total charge sum_k Tr rho_k and of rho_eq.
"""

import numpy as np
import pytest
import scipy.special

import oracle as O
from workloads import FS_AU, HARTREE_EV, FieldTable, diagonal_band_model, flat_band_model, tb4_model
from workloads.configs import R0_STABLE

A = 6.0
DT = 0.05 * FS_AU


def _zero_op(n):
    return O.LowRankOp(np.zeros(n, complex), np.zeros((n, 1), complex), np.zeros((1, n), complex))


def _gauss_pulse(e0, tau, t0, nsteps, ex, ey):
    """Carrier-free Gaussian pulse (omega = 0): its area A(t) has a closed form."""
    return FieldTable.single(e0, 0.0, tau, t0, nsteps, ex, ey)


def _pulse_area(e0, tau, t0, t):
    """int_0^t e0 exp(-(s - t0)^2 / (2 tau^2)) ds."""
    s = np.sqrt(2.0) * tau
    return e0 * tau * np.sqrt(np.pi / 2.0) * (scipy.special.erf((t - t0) / s) + scipy.special.erf(t0 / s))


def _random_hermitian_drho(model, seed, scale=1e-2, diagonal_only=False):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((model.nk, model.nb, model.nb)) + 1j * rng.standard_normal((model.nk, model.nb, model.nb))
    d = 0.5 * scale * (z + z.conj().transpose(0, 2, 1))
    if diagonal_only:
        d = d * np.eye(model.nb)[None]
    return d


def _drift_closed_form(model, drho0, area, ex, ey, t):
    """Exact solution of the semi-discrete drift + flat phase equation."""
    n1, n2, nb = model.nk1, model.nk2, model.nb
    q1 = 2.0 * np.pi * np.fft.fftfreq(n1) * n1 / n1
    q2 = 2.0 * np.pi * np.fft.fftfreq(n2) * n2 / n2
    b1 = 2.0 * np.pi / (n1 * model.a)
    b2 = 2.0 * np.pi / (n2 * model.a)
    lam = ex * np.sin(q1)[:, None] / b1 + ey * np.sin(q2)[None, :] / b2
    out = np.zeros_like(drho0)
    for n in range(nb):
        for m in range(nb):
            de = model.eps[0, n] - model.eps[0, m]
            y = np.fft.fft2(drho0[:, n, m].reshape(n1, n2))
            y *= np.exp(-1j * de * t - 1j * area * lam)
            out[:, n, m] = np.fft.ifft2(y).reshape(-1)
    return out


def _rotate_phases(model, seed):
    """The same model in another Bloch gauge: |n k> -> exp(i phi_nk) |n k>."""
    rng = np.random.default_rng(seed)
    ph = np.exp(1j * rng.uniform(0.0, 2.0 * np.pi, size=(model.nk, model.nb)))
    m = type(model)(**{f: getattr(model, f) for f in model.__dataclass_fields__})
    m.evec = model.evec * ph[:, None, :]
    m.dip = ph.conj()[None, :, :, None] * model.dip * ph[None, :, None, :]
    m.vel = ph.conj()[None, :, :, None] * model.vel * ph[None, :, None, :]
    return m, ph


@pytest.fixture(scope="module")
def tb4_6():
    return tb4_model(6, A, 0.5)


def test_links_are_block_diagonal_polar_factors(tb4_6):
    m = tb4_6
    links = O.transport_links(m)
    nv = m.nv
    eye = np.eye(m.nb)
    for a in range(2):
        i1, i2 = np.divmod(np.arange(m.nk), m.nk2)
        fwd = ((i1 + (a == 0)) % m.nk1) * m.nk2 + (i2 + (a == 1)) % m.nk2
        for k in range(m.nk):
            lk = links[a, k]
            assert np.abs(lk.conj().T @ lk - eye).max() < 1e-13
            assert np.all(lk[:nv, nv:] == 0) and np.all(lk[nv:, :nv] == 0)
            ov = m.evec[k].conj().T @ m.evec[fwd[k]]
            for sl in (slice(0, nv), slice(nv, m.nb)):
                p = lk[sl, sl].conj().T @ ov[sl, sl]       # the positive factor of the block
                assert np.abs(p - p.conj().T).max() < 1e-13
                assert np.linalg.eigvalsh(0.5 * (p + p.conj().T)).min() > 1e-3
                assert np.abs(lk[sl, sl] @ p - ov[sl, sl]).max() < 1e-13


def test_links_identity_for_constant_states():
    m = diagonal_band_model(5, 3, a=A)
    links = O.transport_links(m)
    assert np.abs(links - np.eye(m.nb)[None, None]).max() < 1e-15


def test_links_gauge_covariant(tb4_6):
    m2, ph = _rotate_phases(tb4_6, 11)
    l1 = O.transport_links(tb4_6)
    l2 = O.transport_links(m2)
    m = tb4_6
    i1, i2 = np.divmod(np.arange(m.nk), m.nk2)
    for a in range(2):
        fwd = ((i1 + (a == 0)) % m.nk1) * m.nk2 + (i2 + (a == 1)) % m.nk2
        expect = ph.conj()[:, :, None] * l1[a] * ph[fwd][:, None, :]
        assert np.abs(l2[a] - expect).max() < 1e-13


@pytest.mark.parametrize("ex,ey", [(0.8, 0.6), (1.0, 0.0), (0.0, -1.0)])
def test_drift_matches_fft_closed_form(ex, ey):
    m = flat_band_model(8, 6, nb=4, nv=2, gap_ev=0.5, a=A)
    tau, t0, dt, nsteps = 80.0, 240.0, 0.5, 960
    f = _gauss_pulse(2e-3, tau, t0, nsteps, ex, ey)
    rho_eq = O.rho_equilibrium(m)
    drho0 = _random_hermitian_drho(m, 5)
    out = O.propagate(m, _zero_op(m.nk * 4), "eh", f, dt, rho0=rho_eq + drho0, links=O.transport_links(m))
    t = nsteps * dt
    expect = rho_eq + _drift_closed_form(m, drho0, _pulse_area(2e-3, tau, t0, t), ex, ey, t)
    assert np.abs(out["rho"] - expect).max() < 1e-8 * np.abs(drho0).max()
    # a real move: the state differs from the field-free one by far more than the tolerance
    still = rho_eq + _drift_closed_form(m, drho0, 0.0, ex, ey, t)
    assert np.abs(out["rho"] - still).max() > 1e-2 * np.abs(drho0).max()


def test_population_packet_moves_by_pulse_area():
    m = diagonal_band_model(24, 20, a=A)
    kx, ky = m.kpts[:, 0], m.kpts[:, 1]
    g1, g2 = 2.0 * np.pi / A, 2.0 * np.pi / A
    # a smooth periodic packet in the first conduction band
    bump = np.exp(3.0 * (np.cos(kx * A) - 1.0) + 3.0 * (np.cos(ky * A) - 1.0))
    rho_eq = O.rho_equilibrium(m)
    rho0 = rho_eq.copy()
    rho0[:, m.nv, m.nv] += 0.05 * bump
    tau, t0, dt, nsteps = 100.0, 300.0, 2.0, 300
    ex, ey = 0.8, 0.6
    f = _gauss_pulse(1.5e-3, tau, t0, nsteps, ex, ey)
    out = O.propagate(m, _zero_op(m.nk * 4), "eh", f, dt, rho0=rho0, links=O.transport_links(m))
    area = _pulse_area(1.5e-3, tau, t0, nsteps * dt)
    pop = out["rho"][:, m.nv, m.nv].real

    def centroid(w, k, g):
        return np.angle(np.sum(w * np.exp(1j * k * (2.0 * np.pi / g)))) * g / (2.0 * np.pi)

    shift_x = centroid(pop, kx, g1) - centroid(0.05 * bump, kx, g1)
    shift_y = centroid(pop, ky, g2) - centroid(0.05 * bump, ky, g2)
    assert area * ex > 0.2                                  # several grid spacings
    assert abs(shift_x - area * ex) < 0.03 * area * ex
    assert abs(shift_y - area * ey) < 0.03 * area * ey
    # only the drift acts on populations of k-independent states: the closed form holds
    expect = _drift_closed_form(m, (rho0 - rho_eq) * np.eye(m.nb)[None], area, ex, ey, nsteps * dt)
    got = (out["rho"] - rho_eq) * np.eye(m.nb)[None]
    assert np.abs(got - expect).max() < 1e-7 * 0.05      # RK4 error at dt = 2 a.u.: 1.6e-9


def test_rotated_degenerate_bases_give_the_same_dynamics():
    m_id = flat_band_model(6, 6, dip_seed=5, a=A)
    m_rot = flat_band_model(6, 6, dip_seed=5, gauge_seed=7, a=A)
    f = FieldTable.single(5e-3, 1.0 / HARTREE_EV, 40.0, 120.0, 120, 0.6, 0.8)
    res = []
    for m in (m_id, m_rot):
        op = O.DenseOp(O.build_kernel(m, R0_STABLE, "eh"))
        res.append(O.propagate(m, op, "eh", f, DT, links=O.transport_links(m)))
    r = m_rot.evec
    back = r @ res[1]["rho"] @ r.conj().transpose(0, 2, 1)
    drho = res[0]["rho"] - O.rho_equilibrium(m_id)
    assert np.abs(drho).max() > 1e-3
    assert np.abs(back - res[0]["rho"]).max() < 1e-11 * np.abs(drho).max() + 1e-15
    assert np.abs(res[1]["P"] - res[0]["P"]).max() < 1e-10 * np.abs(res[0]["P"]).max()


def test_band_phases_leave_observables_unchanged(tb4_6):
    m2, _ = _rotate_phases(tb4_6, 3)
    f = FieldTable.single(5e-3, 1.5 / HARTREE_EV, 40.0, 120.0, 100, 0.6, 0.8)
    res = []
    for m in (tb4_6, m2):
        op = O.DenseOp(O.build_kernel(m, R0_STABLE, "eh"))
        res.append(O.propagate(m, op, "eh", f, DT, links=O.transport_links(m)))
    for key in ("P", "J", "occ"):
        scale = np.abs(res[0][key] - res[0][key][0]).max()
        assert scale > 0
        assert np.abs(res[1][key] - res[0][key]).max() < 1e-10 * scale + 1e-14


def test_total_charge_and_equilibrium_conserved(tb4_6):
    m = tb4_6
    links = O.transport_links(m)
    rho_eq = O.rho_equilibrium(m)
    assert np.abs(O.covariant_derivative(m, links, rho_eq, 0.6, 0.8)).max() < 1e-13
    f = FieldTable.single(1e-2, 1.5 / HARTREE_EV, 30.0, 90.0, 90, 0.6, 0.8)
    op = O.DenseOp(O.build_kernel(m, R0_STABLE, "eh"))
    # from rho_eq every band drifts alike and each Tr rho_k stays N_v; start
    # instead from per-k traces that differ (their grid mean still N_v)
    drho = _random_hermitian_drho(m, 9)
    drho[:, 0, 0] -= np.mean(np.einsum("knn->k", drho))
    rho0 = rho_eq + drho
    out = O.propagate(m, op, "eh", f, DT, rho0=rho0, links=links)
    moved = np.einsum("knn->k", out["rho"] - rho0).real
    assert np.abs(moved).max() > 1e-4                      # charge moved between k points
    assert np.abs(out["tr"]).max() < 1e-14                 # but the total is conserved
    assert np.abs(out["herm"]).max() < 1e-13
    # and without the initial trace differences each Tr rho_k stays N_v
    out = O.propagate(m, op, "eh", f, DT, links=links)
    assert np.abs(np.einsum("knn->k", out["rho"]).real - m.nv).max() < 1e-13
