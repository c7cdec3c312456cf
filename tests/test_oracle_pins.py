"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed
forms, theorems, invariants of the equation of motion, textbook special cases
and brute force on tiny inputs.  None of these use the HIP library.
"""

import numpy as np
import pytest
import scipy.integrate
import scipy.special

import oracle as O
from workloads import HARTREE_EV, FS_AU, FieldTable, dirac_model, tb4_model
from workloads.configs import R0_LITERAL, R0_STABLE

A = 6.0
DT = 0.05 * FS_AU


@pytest.fixture(scope="module")
def dirac6():
    return dirac_model(6, 1.0, 1.5, A, 0.5)


@pytest.fixture(scope="module")
def tb4_4():
    return tb4_model(4, A, 0.5)


@pytest.fixture(scope="module")
def k_dirac6(dirac6):
    return O.build_kernel(dirac6, R0_STABLE, "all")


@pytest.fixture(scope="module")
def k_tb4_eh(tb4_4):
    return O.build_kernel(tb4_4, R0_STABLE, "eh")


def strong_pulse(nsteps, e0=5e-3, omega_ev=1.5):
    t = nsteps * DT
    return FieldTable.single(e0, omega_ev / HARTREE_EV, t / 10.0, t / 2.0, nsteps)


# --- inputs (band structure, dipoles) ---------------------------------------

def test_dirac_bands_closed_form(dirac6):
    m = dirac6
    d, t = 1.0 / HARTREE_EV, 1.5 / HARTREE_EV
    s2 = np.sin(m.kpts[:, 0] * A) ** 2 + np.sin(m.kpts[:, 1] * A) ** 2
    e = np.sqrt(d * d + t * t * s2)
    np.testing.assert_allclose(m.eps[:, 0], -e, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(m.eps[:, 1], e, rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("kind", ["dirac", "tb4"])
def test_velocity_diagonal_is_band_slope(kind):
    """Hellmann-Feynman: v_nn = d e_n / dk, checked by central differences."""
    h = 1e-5
    base = dirac_model(4, 1.0, 1.5, A, 0.5) if kind == "dirac" else tb4_model(4, A, 0.5)
    for axis in range(2):
        sh = np.zeros(2)
        sh[axis] = h
        if kind == "dirac":
            def bands(kp):
                d, t = 1.0 / HARTREE_EV, 1.5 / HARTREE_EV
                e = np.sqrt(d * d + t * t * (np.sin(kp[:, 0] * A) ** 2 + np.sin(kp[:, 1] * A) ** 2))
                return np.stack([-e, e], 1)
        else:
            from workloads.models import load_tb4_table, tb4_hamiltonian
            tab = load_tb4_table()

            def bands(kp):
                hk, _ = tb4_hamiltonian(kp, A, tab["tx"] / HARTREE_EV, tab["ty"] / HARTREE_EV,
                                        tab["delta_ev"] / HARTREE_EV)
                return np.linalg.eigvalsh(hk)
        fd = (bands(base.kpts + sh) - bands(base.kpts - sh)) / (2 * h)
        vdiag = np.einsum("knn->kn", base.vel[axis]).real
        np.testing.assert_allclose(vdiag, fd, atol=1e-8 * np.abs(fd).max())


def test_dipole_is_finite_difference_berry_connection(tb4_4):
    """d_nm = i <n k | d/dk m k> for n != m across the gap, from gauge-aligned
    eigenvectors at k +- h (an independent route to the Berry connection)."""
    from workloads.models import load_tb4_table, tb4_hamiltonian
    tab = load_tb4_table()
    m = tb4_4
    h = 1e-5

    def states(kp):
        hk, _ = tb4_hamiltonian(kp, A, tab["tx"] / HARTREE_EV, tab["ty"] / HARTREE_EV,
                                tab["delta_ev"] / HARTREE_EV)
        _, u = np.linalg.eigh(hk)
        # align each state's phase with the stored state at k
        ov = np.einsum("kan,kan->kn", m.evec.conj(), u)
        return u * (np.abs(ov) / ov)[:, None, :]

    for axis in range(2):
        sh = np.zeros(2)
        sh[axis] = h
        du = (states(m.kpts + sh) - states(m.kpts - sh)) / (2 * h)
        berry = 1j * np.einsum("kan,kam->knm", m.evec.conj(), du)
        for n in range(2):
            for c in range(2, 4):
                np.testing.assert_allclose(m.dip[axis][:, n, c], berry[:, n, c],
                                           atol=1e-6 * np.abs(berry[:, n, c]).max())
                np.testing.assert_allclose(m.dip[axis][:, c, n], berry[:, c, n],
                                           atol=1e-6 * np.abs(berry[:, c, n]).max())


# --- kernel -----------------------------------------------------------------

def test_kernel_hermitian_and_pair_swap(dirac6, k_dirac6):
    k = k_dirac6
    assert np.abs(k - k.conj().T).max() <= 1e-16 * np.abs(k).max()
    # K_(mn),(m'n') = K_(n'm'),(nm): swapping both pairs' bands transposes K
    nb = dirac6.nb
    perm = np.array([kk * nb * nb + m * nb + n for kk in range(dirac6.nk)
                     for n in range(nb) for m in range(nb)])
    np.testing.assert_allclose(k[np.ix_(perm, perm)], k.T, rtol=0, atol=1e-16 * np.abs(k).max())


def test_kernel_diagonal_closed_form(dirac6, k_dirac6):
    m = dirac6
    w0 = O.cell_average_w0(np.pi / (m.nk1 * A), R0_STABLE)
    np.testing.assert_allclose(np.diag(k_dirac6), -w0 / (m.nk * A * A), rtol=1e-14)
    # same k, different band channel: overlaps of orthonormal states vanish
    p = 4
    for kk in range(m.nk):
        blk = k_dirac6[kk * p:(kk + 1) * p, kk * p:(kk + 1) * p]
        off = blk - np.diag(np.diag(blk))
        assert np.abs(off).max() < 1e-15 * np.abs(blk).max()


def test_kernel_matches_elementwise_definition(tb4_4, k_tb4_eh):
    rng = np.random.default_rng(0)
    for i, j in rng.integers(0, k_tb4_eh.shape[0], size=(40, 2)):
        assert abs(k_tb4_eh[i, j] - O.kernel_element(tb4_4, R0_STABLE, "eh", i, j)) \
            <= 1e-15 * np.abs(k_tb4_eh).max()


def test_w0_cell_average():
    h = np.pi / (36 * A)
    w64 = O.cell_average_w0(h, R0_STABLE, 64)
    w128 = O.cell_average_w0(h, R0_STABLE, 128)
    assert abs(w64 - w128) <= 1e-14 * w64
    # r0 -> 0: average of 2 pi / q over the square is (4 pi / h) ln(1 + sqrt 2)
    r0 = 1e-9
    np.testing.assert_allclose(O.cell_average_w0(h, r0), 4 * np.pi / h * np.log1p(np.sqrt(2)), rtol=1e-7)
    # independent route: adaptive Cartesian quadrature over one quadrant
    f = lambda y, x: 2 * np.pi / (np.hypot(x, y) * (1 + R0_STABLE * np.hypot(x, y)))  # noqa: E731
    val, _ = scipy.integrate.dblquad(f, 0, h, 0, h, epsabs=0, epsrel=1e-11)
    np.testing.assert_allclose(w64, val / (h * h), rtol=1e-8)


def test_flat_band_kernel_is_circulant():
    """t = 0: Bloch states do not depend on k, the e-h kernel is a 2D circulant
    and the Tamm-Dancoff exciton energies are 2 Delta plus the 2D DFT of one row."""
    nk = 6
    m = dirac_model(nk, 1.0, 0.0, A, 0.5)
    k = O.build_kernel(m, R0_STABLE, "eh")
    amat = np.diag(m.eps[:, 1] - m.eps[:, 0]) + k
    ev = np.linalg.eigvalsh(amat)
    row = k[0].real.reshape(nk, nk)
    # k index 0 sits at grid (0, 0); row[j] = w(k_0 - k_j): a circulant in both directions
    spec = np.fft.fft2(row).real
    ref = np.sort(2.0 / HARTREE_EV + spec.ravel())
    np.testing.assert_allclose(ev, ref, rtol=0, atol=1e-14)


def _bz_integral_of_w(r0):
    """(1 / (2 pi)^2) int over the square Brillouin zone of W(q) d^2q, in polar
    coordinates over its eight triangles (adaptive quadrature)."""
    g = np.pi / A
    inner = scipy.integrate.quad(lambda th: np.log1p(r0 * g / np.cos(th)) / r0, 0, np.pi / 4,
                                 epsabs=0, epsrel=1e-13)[0]
    return 8.0 * inner * 2.0 * np.pi / (2.0 * np.pi) ** 2


def test_kernel_row_sum_is_brillouin_zone_integral():
    """Flat bands: -sum_k' K_(k),(k') is the Riemann sum (1/(N_k A)) sum_q W(q) of
    the continuum integral (1/(2 pi)^2) int_BZ W(q) d^2q; this fixes the kernel's
    normalisation independently of how the oracle writes it."""
    ref = _bz_integral_of_w(R0_STABLE)
    rel = []
    for nk in (24, 36):
        m = dirac_model(nk, 1.0, 0.0, A, 0.5)
        k = O.build_kernel(m, R0_STABLE, "eh")
        rel.append(abs(-k[0].sum().real / ref - 1.0))
    assert rel[1] < 0.03 and rel[1] < rel[0]


def test_literal_r0_is_unstable():
    m = dirac_model(12, 1.0, 1.5, A, 0.5)
    keh = O.build_kernel(m, R0_LITERAL, "eh")
    lowest = np.linalg.eigvalsh(np.diag(m.eps[:, 1] - m.eps[:, 0]) + keh)[0] * HARTREE_EV
    assert lowest < -2.0          # the ground state is not stable
    keh = O.build_kernel(m, R0_STABLE, "eh")
    lowest = np.linalg.eigvalsh(np.diag(m.eps[:, 1] - m.eps[:, 0]) + keh)[0] * HARTREE_EV
    assert 1.6 < lowest < 1.7     # bound exciton below the 2.28 eV gap


# --- compression ------------------------------------------------------------

def test_svd_eckart_young(k_tb4_eh):
    kdiag, koff = O.split_diag(k_tb4_eh)
    u, s, vh = O.svd_offdiag(koff, "svd")
    for r in (1, 7, 20, 40):
        kr = (u[:, :r] * s[:r]) @ vh[:r]
        np.testing.assert_allclose(np.linalg.norm(koff - kr, 2), s[r], rtol=1e-10)
        np.testing.assert_allclose(np.linalg.norm(koff - kr) ** 2, np.sum(s[r:] ** 2), rtol=1e-10)
    # Hermitian K_off: singular values are |eigenvalues|
    np.testing.assert_allclose(np.sort(s), np.sort(np.abs(np.linalg.eigvalsh(koff))), rtol=1e-10,
                               atol=1e-14 * s[0])
    u2, s2, vh2 = O.svd_offdiag(koff, "eigh")
    np.testing.assert_allclose(s2, s, rtol=1e-10, atol=1e-14 * s[0])
    r = 30
    np.testing.assert_allclose((u2[:, :r] * s2[:r]) @ vh2[:r], (u[:, :r] * s[:r]) @ vh[:r],
                               atol=1e-12 * s[0])
    full = O.compress(k_tb4_eh, "rank", koff.shape[0])
    rec = np.diag(full["kdiag"]) + full["US"] @ full["Vh"]
    np.testing.assert_allclose(rec, k_tb4_eh, atol=1e-13 * np.abs(k_tb4_eh).max())


def test_rank_rules(k_tb4_eh):
    kdiag, koff = O.split_diag(k_tb4_eh)
    _, s, _ = O.svd_offdiag(koff)
    f = O.compress(k_tb4_eh, "rel_cut", 1e-2)
    assert f["r"] == np.count_nonzero(s > 1e-2 * s[0])
    f = O.compress(k_tb4_eh, "fraction", 0.05)
    assert f["r"] == max(1, round(0.05 * s.shape[0]))
    # R^2 rule against brute force over every rank
    f = O.compress(k_tb4_eh, "r2", 0.9)
    u, s, vh = np.linalg.svd(koff)
    mean_dev = np.sum(np.abs(koff - koff.mean()) ** 2)
    r2 = [1 - np.sum(np.abs(koff - (u[:, :r] * s[:r]) @ vh[:r]) ** 2) / mean_dev
          for r in range(s.shape[0] + 1)]
    assert f["r"] == next(r for r, v in enumerate(r2) if v >= 0.9)


def test_rank_never_splits_equal_singular_values():
    s = np.array([5.0, 4.0, 3.0, 3.0, 3.0 * (1 - 1e-12), 1.0, 0.5])
    assert O.choose_rank(s, "rank", 3) == 5
    assert O.choose_rank(s, "rank", 2) == 2
    assert O.choose_rank(s, "rel_cut", 0.5) == 5


# --- propagation invariants -------------------------------------------------

def test_stationary_at_zero_field_bitwise(tb4_4, k_tb4_eh):
    f = FieldTable.single(0.0, 0.05, 100.0, 200.0, 40)
    out = O.propagate(tb4_4, O.DenseOp(k_tb4_eh), "eh", f, DT)
    assert np.array_equal(out["rho"], O.rho_equilibrium(tb4_4))
    assert np.all(out["P"] == 0.0) and np.all(out["occ"] == 0.0)


def test_trace_and_hermiticity_conserved(dirac6, k_dirac6):
    out = O.propagate(dirac6, O.DenseOp(k_dirac6), "all", strong_pulse(600, 2e-2), DT)
    assert out["occ"].max() > 1e-3          # the pulse really excites the system
    assert out["tr"].max() < 1e-13
    assert out["herm"].max() < 1e-14


def _idempotency(rho):
    return np.abs(np.einsum("kab,kbc->kac", rho, rho) - rho).max()


def test_density_matrix_spectrum_conserved_to_rk4_order(tb4_4, k_tb4_eh):
    """Commutator dynamics keeps the eigenvalues of rho_k (0 or 1); RK4 breaks
    that at O(dt^4): halving dt divides ||rho^2 - rho|| by about 16."""
    f = strong_pulse(400, 2e-2)
    e1 = _idempotency(O.propagate(tb4_4, O.DenseOp(k_tb4_eh), "eh", f, DT)["rho"])
    e2 = _idempotency(O.propagate(tb4_4, O.DenseOp(k_tb4_eh), "eh", f, DT / 2, nsteps=800)["rho"])
    assert e1 > 1e-12
    assert 10.0 < e1 / e2 < 24.0


def _energy(model, k, block, rho):
    from oracle.kernel import pair_table
    pairs = pair_table(model.nb, model.nv, block)
    pa = np.array([p[0] for p in pairs])
    pb = np.array([p[1] for p in pairs])
    drho = rho - O.rho_equilibrium(model)
    x = drho[:, pa, pb].reshape(-1)
    y = (k @ x).reshape(model.nk, len(pairs))
    ds = np.zeros_like(drho)
    ds[:, pa, pb] = y
    if block == "eh":
        ds[:, pb, pa] = y.conj()
    e_band = np.einsum("kn,knn->", model.eps, rho).real
    return e_band + 0.5 * np.einsum("knm,kmn->", drho, ds).real


@pytest.mark.parametrize("block", ["all", "eh"])
def test_energy_conserved_after_pulse(dirac6, k_dirac6, tb4_4, k_tb4_eh, block):
    """With the field off, E = sum Tr(eps rho) + 1/2 Tr(drho dSigma) is a constant
    of the motion (K is Hermitian with the pair-swap symmetry); RK4 keeps it to
    O(dt^4): the drift falls by more than 12x per halving of dt."""
    model, k = (dirac6, k_dirac6) if block == "all" else (tb4_4, k_tb4_eh)
    f = FieldTable.single(2e-2, 1.5 / HARTREE_EV, 1.0 * FS_AU, 4.0 * FS_AU, 400)
    # after t = 12 fs the envelope is below exp(-32) of its peak
    drift = []
    for div in (1, 2):
        out = O.propagate(model, O.DenseOp(k), block, f, DT / div, nsteps=240 * div)
        e_mid = _energy(model, k, block, out["rho"])
        out2 = O.propagate(model, O.DenseOp(k), block, f, DT / div, nsteps=400 * div)
        e_end = _energy(model, k, block, out2["rho"])
        drift.append(abs(e_end - e_mid))
    e_exc = e_mid - _energy(model, k, block, O.rho_equilibrium(model))
    assert e_exc > 1e-3
    assert drift[1] < 1e-5 * e_exc
    assert drift[0] / drift[1] > 12.0


def test_rk4_fourth_order(tb4_4, k_tb4_eh):
    f = strong_pulse(200, 1e-2)
    ref = O.propagate(tb4_4, O.DenseOp(k_tb4_eh), "eh", f, DT / 8, nsteps=1600)["P"][::8]
    errs = []
    for div in (1, 2):
        p = O.propagate(tb4_4, O.DenseOp(k_tb4_eh), "eh", f, DT / div, nsteps=200 * div)["P"][::div]
        errs.append(np.abs(p - ref).max())
    assert 12.0 < errs[0] / errs[1] < 20.0


def test_lowrank_full_rank_equals_dense(tb4_4, k_tb4_eh):
    f = strong_pulse(300)
    dense = O.propagate(tb4_4, O.DenseOp(k_tb4_eh), "eh", f, DT)
    fac = O.compress(k_tb4_eh, "rank", k_tb4_eh.shape[0])
    low = O.propagate(tb4_4, O.LowRankOp.from_factors(fac), "eh", f, DT)
    for key in ("P", "J", "occ"):
        np.testing.assert_allclose(low[key], dense[key], rtol=0, atol=1e-12 * np.abs(dense[key]).max())


# --- linear response: closed form and Bethe-Salpeter brute force --------------

def _two_level_closed_form(model, fields, dt, nsteps):
    """K = 0: drho_cv(t) = i (e.d_cv) int_0^t exp(-i dE (t - s)) E(s) ds, with the
    Gaussian-cosine integral written through the Faddeeva function."""
    e0, om, tau, t0 = (float(fields.e0[0]), float(fields.omega[0]), float(fields.tau[0]),
                       float(fields.t0[0]))
    de = model.eps[:, 1] - model.eps[:, 0]
    t = np.arange(nsteps + 1) * dt
    s2t = np.sqrt(2.0) * tau

    def gauss_int(beta, s):
        # exp(-(s - t0)^2 / (2 tau^2) + i beta (s - t0)) * w(i z), z = (s - t0)/(s2t) - i beta tau / sqrt2
        u = (s - t0) / s2t
        z = u - 1j * beta * tau / np.sqrt(2.0)
        return np.exp(-u * u + 1j * beta * (s - t0)) * scipy.special.wofz(1j * z)

    out = np.zeros((nsteps + 1, model.nk), dtype=np.complex128)
    for sign in (+1.0, -1.0):
        beta = de[None, :] + sign * om            # exp(i dE s) exp(+-i w s)
        # int_0^t exp(i beta s) exp(-(s - t0)^2/(2 tau^2)) ds
        val = tau * np.sqrt(np.pi / 2.0) * np.exp(1j * beta * t0) * (
            gauss_int(beta, 0.0 * t[:, None]) - gauss_int(beta, t[:, None]))
        out += 0.5 * e0 * val
    g = np.exp(-1j * de[None, :] * t[:, None]) * out          # int_0^t e^{-i dE (t-s)} E(s) ds
    d = model.dip[0]
    v = model.vel[0]
    drho_cv = 1j * d[None, :, 1, 0] * g
    p = 2.0 * (d[None, :, 0, 1] * drho_cv).real.sum(1) / model.nk
    j = (2.0 * (v[None, :, 0, 1] * drho_cv).real.sum(1) + v[:, 0, 0].real.sum()) / model.nk
    return p, j, g


def test_two_level_closed_form(dirac6):
    m = dirac6
    f = FieldTable.single(1e-6, 2.0 / HARTREE_EV, 3.0 * FS_AU, 8.0 * FS_AU, 480)
    p_ref, j_ref, g = _two_level_closed_form(m, f, DT / 2, 480)
    # the closed form itself against adaptive quadrature at one k and time
    t_chk = 300 * DT / 2
    de = m.eps[0, 1] - m.eps[0, 0]
    ef = lambda s: 1e-6 * np.exp(-(s - f.t0[0]) ** 2 / (2 * f.tau[0] ** 2)) * np.cos(f.omega[0] * s)  # noqa: E731
    re = scipy.integrate.quad(lambda s: np.cos(de * (t_chk - s)) * ef(s), 0, t_chk, limit=400)[0]
    im = scipy.integrate.quad(lambda s: -np.sin(de * (t_chk - s)) * ef(s), 0, t_chk, limit=400)[0]
    np.testing.assert_allclose(g[300, 0], re + 1j * im, rtol=1e-8)
    kzero = np.zeros((m.nk * 4, m.nk * 4), dtype=np.complex128)
    out = O.propagate(m, O.DenseOp(kzero), "all", f, DT / 2, nsteps=480)
    assert np.abs(out["P"] - p_ref).max() < 1e-5 * np.abs(p_ref).max()
    jd = j_ref - j_ref[0]
    assert np.abs(out["J"] - j_ref).max() < 1e-5 * np.abs(jd).max()


def test_weak_pulse_matches_bse_linear_response(dirac6, k_dirac6):
    f = FieldTable.single(1e-6, 2.0 / HARTREE_EV, 3.0 * FS_AU, 8.0 * FS_AU, 800)
    lr = O.linear_response(dirac6, k_dirac6, "all", f, DT / 2, 800)
    out = O.propagate(dirac6, O.DenseOp(k_dirac6), "all", f, DT / 2, nsteps=800)
    assert np.abs(out["P"] - lr["P"]).max() < 2e-5 * np.abs(lr["P"]).max()
    jd = lr["J"] - lr["J"][0]
    assert np.abs((out["J"] - out["J"][0]) - jd).max() < 2e-5 * np.abs(jd).max()


def test_weak_pulse_matches_tamm_dancoff_linear_response(tb4_4, k_tb4_eh):
    """Conduction-valence block: a weak pulse's P(t), J(t) equal the linear
    response of the Tamm-Dancoff problem A = dE + K_eh (the e-h branch of the
    linear response), to O(E0^2) and the RK4 error."""
    f = FieldTable.single(1e-7, 2.0 / HARTREE_EV, 3.0 * FS_AU, 8.0 * FS_AU, 800)
    lr = O.linear_response(tb4_4, k_tb4_eh, "eh", f, DT / 2, 800)
    out = O.propagate(tb4_4, O.DenseOp(k_tb4_eh), "eh", f, DT / 2, nsteps=800)
    assert np.abs(lr["P"]).max() > 1e-9
    assert np.abs(out["P"] - lr["P"]).max() < 2e-5 * np.abs(lr["P"]).max()
    jd = lr["J"] - lr["J"][0]
    assert np.abs((out["J"] - out["J"][0]) - jd).max() < 1e-4 * np.abs(jd).max()


def test_absorption_matches_sum_over_states(tb4_4, k_tb4_eh):
    """A narrow kick excites every exciton.  The absorption spectrum of the
    time-domain run equals the textbook linear-response spectrum built from the
    eigenpairs (W_S, A^S) of the Tamm-Dancoff A = dE + K_eh, with the same
    damping eta:
      A(w) = w Im chi(w),
      chi(w) = (1/nk) sum_S |<A^S|d_cv>|^2 [1/(W_S - w - i eta) + 1/(W_S + w + i eta)],
    over 0.2-1.2 eV to 2 % of its maximum (the rest: the finite window and the
    kick's width).  Within 0.1 eV of the lowest bright exciton the spectrum's
    maximum lies within the transform's resolution 2 pi/T of it."""
    m = tb4_4
    nsteps = 3000
    kick = FieldTable.single(1e-6, 0.0, 0.125 * FS_AU, 0.5 * FS_AU, nsteps)
    out = O.propagate(m, O.DenseOp(k_tb4_eh), "eh", kick, DT)
    amat, lab = O.linear_operator(m, k_tb4_eh, "eh")
    ev, vec = np.linalg.eigh(amat)
    kn, n, mm = lab[:, 0], lab[:, 1], lab[:, 2]
    osc = np.abs(vec.conj().T @ m.dip[0][kn, n, mm]) ** 2
    t = np.arange(out["P"].shape[0]) * DT
    efield = np.array([O.field_at(ti, kick, 0) for ti in t])
    eta = 0.02 / HARTREE_EV
    om = np.linspace(0.2 / HARTREE_EV, 1.2 / HARTREE_EV, 1001)
    spec = O.absorption(out["P"], efield, DT, om, eta)
    chi = (osc[None, :] * (1.0 / (ev[None, :] - om[:, None] - 1j * eta)
                           + 1.0 / (ev[None, :] + om[:, None] + 1j * eta))).sum(1) / m.nk
    ref = om * chi.imag
    assert np.abs(spec - ref).max() < 2e-2 * ref.max()
    target = ev[osc > 1e-2 * osc.max()][0]
    win = np.linspace(target - 0.1 / HARTREE_EV, target + 0.1 / HARTREE_EV, 401)
    assert np.sum(np.abs(ev - target) < 0.1 / HARTREE_EV) == 1      # an isolated exciton
    peak = win[np.argmax(O.absorption(out["P"], efield, DT, win, eta))]
    assert abs(peak - target) < 2 * np.pi / (nsteps * DT)


def _geometric(x, count):
    """sum_{n < count} exp(i x n)"""
    z = np.exp(1j * x)
    return complex(count) if abs(1.0 - z) < 1e-14 else (1.0 - z ** count) / (1.0 - z)


def test_hhg_of_a_pure_harmonic_closed_form():
    """HHG(W) = |W dt sum_n J_n exp(-i W t_n)|^2 for J_n = cos(a t_n): the two
    exponentials of the cosine sum as geometric series, at the harmonic
    (where the sum grows as count/2) and away from it."""
    dt, count, a = 0.37, 1500, 0.21
    j = np.cos(a * np.arange(count) * dt)
    om = np.array([a, 2 * a, 3 * a, 0.5 * a, 1.013 * a])
    got = O.hhg(j, dt, om)
    ref = np.array([abs(w * dt * 0.5 * (_geometric((a - w) * dt, count) + _geometric(-(a + w) * dt, count))) ** 2
                    for w in om])
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-12 * ref.max())
    assert abs(got[0] / (a * dt * count / 2) ** 2 - 1.0) < 1e-2
    # the spectrum's maximum sits at the harmonic, within the resolution 2 pi / (count dt)
    fine = np.linspace(0.5 * a, 1.5 * a, 2001)
    assert abs(fine[np.argmax(O.hhg(j, dt, fine))] - a) < 2 * np.pi / (count * dt)


def test_harmonic_loss_closed_form():
    """The third-harmonic intensity of J_n = cos(3 w t_n) + cos(w t_n) is the
    geometric-series value at 3w, and equals hhg at 3w."""
    dt, count, w = 0.29, 1200, 0.11
    t = np.arange(count) * dt
    j = np.cos(3 * w * t) + np.cos(w * t)
    loss, _, _ = O.harmonic_loss(j, w, dt, order=3)
    s = sum(0.5 * (_geometric((c - 3 * w) * dt, count) + _geometric(-(c + 3 * w) * dt, count)) for c in (3 * w, w))
    assert abs(loss - abs(3 * w * dt * s) ** 2) <= 1e-10 * loss
    assert abs(loss - O.hhg(j, dt, np.array([3 * w]))[0]) <= 1e-12 * loss


def test_linear_response_of_literal_r0_grows():
    """With r0 = 5 bohr the full BSE has complex eigenvalues: the oracle reports
    the instability (growing response) rather than a spectrum."""
    m = dirac_model(6, 1.0, 1.5, A, 0.5)
    k = O.build_kernel(m, R0_LITERAL, "all")
    lmat, _ = O.linear_operator(m, k, "all")
    assert np.abs(np.linalg.eigvals(lmat).imag).max() > 1e-3


# --- randomized range finder (an addition for large kernels, not the paper's) --

def test_randomized_full_width_is_exact(k_tb4_eh):
    """With as many test vectors as rows the range finder spans everything and
    the factorisation equals the exact truncated SVD."""
    from workloads.random_matrices import gaussian_test_matrix
    n = k_tb4_eh.shape[0]
    exact = O.compress(k_tb4_eh, "rank", 20)
    rnd = O.randomized_compress(k_tb4_eh, 20, gaussian_test_matrix(n, n, 1), power_iters=0)
    np.testing.assert_allclose(rnd["s"][:20], exact["s"][:20], rtol=1e-10)
    np.testing.assert_allclose(rnd["US"] @ rnd["Vh"], exact["US"] @ exact["Vh"], atol=1e-12 * exact["s"][0])


def test_randomized_recovers_a_low_rank_plus_noise_matrix():
    """Planted spectrum with a gap: the randomized factors find the top
    eigenpairs; the residual obeys the Eckart-Young floor."""
    from workloads.random_matrices import gaussian_test_matrix
    rng = np.random.default_rng(3)
    n, r = 200, 12
    q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    lam = np.concatenate([np.linspace(5, 2, r) * rng.choice([-1, 1], r), 1e-3 * rng.standard_normal(n - r)])
    koff = (q * lam) @ q.conj().T
    k = koff + np.diag(rng.standard_normal(n))          # diagonal is split off first
    k = 0.5 * (k + k.conj().T)
    rnd = O.randomized_compress(k, r, gaussian_test_matrix(n, r + 10, 2), power_iters=2)
    exact = O.compress(k, "rank", r)
    np.testing.assert_allclose(rnd["s"][:r], exact["s"][:r], rtol=1e-4)
    _, koff_k = O.split_diag(k)
    resid = np.linalg.norm(koff_k - rnd["US"] @ rnd["Vh"], 2)
    assert resid <= 1.01 * exact["s"][r]


# --- channel-wise SVD (Eq. svd-channel-wise) ---------------------------------

def test_channel_blocks_follow_the_element_definition(tb4_4, k_tb4_eh):
    """Element (k, k') of channel (p, q) is the kernel element of pair p at k
    and pair q at k', from the element-by-element definition."""
    P = 4
    blocks = O.channel_blocks(k_tb4_eh, tb4_4.nk, P)
    rng = np.random.default_rng(5)
    for _ in range(40):
        p, q = rng.integers(0, P, 2)
        kk, kq = rng.integers(0, tb4_4.nk, 2)
        ref = O.kernel_element(tb4_4, R0_STABLE, "eh", kk * P + p, kq * P + q)
        assert abs(blocks[(p, q)][kk, kq] - ref) <= 1e-14 * abs(ref) + 1e-18


def test_channel_pairing_and_eckart_young(tb4_4, k_tb4_eh):
    """K Hermitian => K^{qp} = (K^{pq})^H, so the two channels share singular
    values; each truncated channel's residual is its discarded tail."""
    P, nk = 4, tb4_4.nk
    f = O.compress_channelwise(k_tb4_eh, nk, P, "rank", 5)
    blocks = O.channel_blocks(k_tb4_eh, nk, P)
    for (p, q), (s_, vh, sv) in f["off"].items():
        np.testing.assert_allclose(sv, f["off"][(q, p)][2], rtol=1e-12, atol=1e-14 * sv[0])
        r = f["ranks"][(p, q)]
        resid = blocks[(p, q)] - s_ @ vh
        np.testing.assert_allclose(np.linalg.norm(resid) ** 2, np.sum(sv[r:] ** 2), rtol=1e-9)
        np.testing.assert_allclose(np.linalg.norm(resid, 2), sv[r], rtol=1e-9)
    for p in range(P):
        np.testing.assert_array_equal(f["diag"][p], blocks[(p, p)])


def test_channelwise_full_rank_equals_dense(tb4_4, k_tb4_eh):
    P, nk = 4, tb4_4.nk
    f = O.compress_channelwise(k_tb4_eh, nk, P, "fraction", 1.0)
    op = O.ChannelOp(f, nk, P)
    rng = np.random.default_rng(6)
    x = rng.standard_normal(nk * P) + 1j * rng.standard_normal(nk * P)
    ref = k_tb4_eh @ x
    assert np.abs(op.apply(x) - ref).max() <= 1e-13 * np.abs(ref).max()


def test_channelwise_truncation_keeps_hermiticity(tb4_4, k_tb4_eh):
    """Equal ranks on (p, q) and (q, p) give a Hermitian operator: <y, A x> = <A y, x>."""
    P, nk = 4, tb4_4.nk
    op = O.ChannelOp(O.compress_channelwise(k_tb4_eh, nk, P, "rank", 4), nk, P)
    rng = np.random.default_rng(7)
    x = rng.standard_normal(nk * P) + 1j * rng.standard_normal(nk * P)
    y = rng.standard_normal(nk * P) + 1j * rng.standard_normal(nk * P)
    a = np.vdot(y, op.apply(x))
    b = np.vdot(op.apply(y), x)
    assert abs(a - b) <= 1e-13 * abs(a)
