"""The pins bite: plausible mistakes planted in the oracle (on the CPU) make
at least one pin fail.  Each case patches one oracle function for the duration
of the test and runs the pin that should catch it."""

import numpy as np
import pytest

import importlib

import oracle as O
import test_oracle_pins as pins
from workloads import dirac_model, tb4_model
from workloads.configs import R0_STABLE

A = pins.A
# the package re-exports functions under the submodules' names, so fetch the modules
KERNEL = importlib.import_module("oracle.kernel")
OBSERVABLES = importlib.import_module("oracle.observables")
PROPAGATE = importlib.import_module("oracle.propagate")
BSE = importlib.import_module("oracle.bse")
ADJOINT = importlib.import_module("oracle.adjoint")
INTRABAND = importlib.import_module("oracle.intraband")
COMPRESS = importlib.import_module("oracle.compress")
SPECTRA = importlib.import_module("oracle.spectra")


@pytest.fixture(scope="module")
def small():
    d6 = dirac_model(6, 1.0, 1.5, A, 0.5)
    t4 = tb4_model(4, A, 0.5)
    return d6, t4


def _transposed_dense(self, x):
    return self.k.T @ x


def _flipped_commutator(h, rho):
    return -1j * (rho @ h - h @ rho)


def _no_conj_kernel(model, r0, block):
    nk, nb, nv = model.nk, model.nb, model.nv
    pairs = KERNEL.pair_table(nb, nv, block)
    pa = np.array([p[0] for p in pairs])
    pb = np.array([p[1] for p in pairs])
    w = KERNEL.coulomb_matrix(model.kpts, model.nk1, model.nk2, model.a, r0)
    ov = np.einsum("kan,lam->klnm", model.evec.conj(), model.evec)
    kk = -(w / (nk * model.a ** 2))[:, :, None, None] * ov[:, :, pa[:, None], pa[None, :]] \
        * ov[:, :, pb[:, None], pb[None, :]]
    return np.ascontiguousarray(kk.transpose(0, 2, 1, 3).reshape(nk * len(pairs), -1))


def _transposed_trace(a, rho):
    return complex(np.einsum("knm,knm->", a, rho))


def _pull_commutator_unconjugated(h, y, g):
    return 1j * (h @ g - g @ h), -1j * (g @ y - y @ g)


def _pull_commutator_ybar_sign(h, y, g):
    a, b = ADJOINT.__dict__["_real_pull_commutator"](h, y, g)
    return -a, b


def _pull_field_no_conj(dmat, y, g):
    return float(np.sum((g * (1j * (dmat @ y - y @ dmat))).real))


def _omega_derivative_sign(t, fields, b):
    d = ADJOINT.__dict__["_real_field_param_derivs"](t, fields, b)
    d[1] = -d[1]
    return d


def _cotangent_wrong_band(model, ex, ey, gp, gj, gocc):
    d = ex * model.dip[0] + ey * model.dip[1]
    v = ex * model.vel[0] + ey * model.vel[1]
    g = (gp * d.conj().transpose(0, 2, 1) + gj * v.conj().transpose(0, 2, 1)).astype(np.complex128)
    g[:, model.nv - 1, model.nv - 1] += gocc
    return g / model.nk


def _channel_wrong_source(self, x):
    P = self.npair
    xs = x.reshape(self.nk, P)
    y = np.zeros_like(xs)
    for p in range(P):
        y[:, p] = self.f["diag"][p] @ xs[:, p]
        for q in range(P):
            if q != p:
                s, vh, _ = self.f["off"][(p, q)]
                y[:, p] += s @ (vh @ xs[:, p])
    return y.reshape(-1)


def _backward_link_not_daggered(model, links, y, ex, ey):
    out = np.zeros_like(y)
    for a, e in ((0, ex), (1, ey)):
        fwd = INTRABAND._neighbour(model, a, +1)
        bwd = INTRABAND._neighbour(model, a, -1)
        lf, lb = links[a], links[a][bwd]
        diff = lf @ y[fwd] @ lf.conj().transpose(0, 2, 1) - lb @ y[bwd] @ lb.conj().transpose(0, 2, 1)
        out += (e / (2.0 * INTRABAND.grid_spacing(model, a))) * diff
    return out


def _vh_unconjugated(self, x):
    return self.kdiag * x + self.us @ (self.vh.conj() @ x)


def _diagonal_left_in(k):
    return np.diag(k).copy(), k.copy()


def _eigh_route_without_signs(koff, method="svd"):
    if method == "svd":
        return COMPRESS._real_svd_offdiag(koff, method)
    lam, q = np.linalg.eigh(koff)
    order = np.argsort(-np.abs(lam), kind="stable")
    q = q[:, order]
    return q, np.abs(lam[order]), q.conj().T


def _fraction_off_by_one(s, rule, value, koff_fro2=None, koff_mean_dev2=None):
    r = COMPRESS._real_choose_rank(s, rule, value, koff_fro2, koff_mean_dev2)
    return r + 1 if rule == "fraction" else r


def _randomized_vh_unconjugated(k, rank, omega, power_iters=2):
    f = COMPRESS._real_randomized_compress(k, rank, omega, power_iters)
    f["Vh"] = f["Vh"].conj()
    return f


def _randomized_ritz_signs_dropped(k, rank, omega, power_iters=2):
    f = COMPRESS._real_randomized_compress(k, rank, omega, power_iters)
    u = f["Vh"].conj().T
    f["US"] = u * f["s"][None, :f["r"]]
    return f


def _one_band_too_many_filled(model):
    occ = np.zeros(model.nb)
    occ[: model.nv + 1] = 1.0
    return np.broadcast_to(np.diag(occ).astype(np.complex128), (model.nk, model.nb, model.nb)).copy()


def _current_not_averaged(model, rho, ex, ey, grid_trace=False):
    o = OBSERVABLES.observables(model, rho, ex, ey, grid_trace)
    o["J"] *= model.nk
    return o


def _sector_trace_partner_dropped(drho, a, lab, block):
    kn, n, m = lab[:, 0], lab[:, 1], lab[:, 2]
    return (drho * a[kn, m, n][None, :]).sum(1).real


def _sector_trace_transposed(drho, a, lab, block):
    kn, n, m = lab[:, 0], lab[:, 1], lab[:, 2]
    t = drho * a[kn, n, m][None, :]
    if block == "eh":
        t = t + t.conj()
    return t.sum(1).real


def _absorption_no_frequency(p, e, dt, omegas, eta):
    return SPECTRA._real_absorption(p, e, dt, omegas, eta) / omegas


def _hhg_no_frequency(j, dt, omegas):
    return SPECTRA._real_hhg(j, dt, omegas) / omegas ** 2


def _hhg_no_dt(j, dt, omegas):
    return SPECTRA._real_hhg(j, dt, omegas) / dt ** 2


def _harmonic_loss_fundamental(j, omega, dt, order=3):
    return ADJOINT._real_harmonic_loss(j, omega, dt, order=1)


SPECTRA._real_absorption = SPECTRA.absorption
SPECTRA._real_hhg = SPECTRA.hhg
ADJOINT._real_harmonic_loss = ADJOINT.harmonic_loss
INTRABAND._real_neighbour = INTRABAND._neighbour
COMPRESS._real_svd_offdiag = COMPRESS.svd_offdiag
COMPRESS._real_choose_rank = COMPRESS.choose_rank
COMPRESS._real_randomized_compress = COMPRESS.randomized_compress
INTRABAND._real_covariant_derivative = INTRABAND.covariant_derivative
ADJOINT._real_pull_commutator = ADJOINT.pull_commutator
ADJOINT._real_field_param_derivs = ADJOINT.field_param_derivs

CASES = {
    "dense operand transposed": (O.DenseOp, "apply", _transposed_dense, "weak_bse"),
    "commutator sign flipped": (PROPAGATE, "minus_i_commutator", _flipped_commutator, "two_level"),
    "field sign flipped": (PROPAGATE, "field_at",
                           lambda t, f, b: -BSE.field_at(t, f, b), "two_level"),
    "second overlap not conjugated": (KERNEL, "build_kernel", _no_conj_kernel, "hermitian"),
    "interaction doubled": (KERNEL, "rytova_keldysh",
                            lambda q, r0: 4 * np.pi / (np.asarray(q) * (1 + r0 * np.asarray(q))), "row_sum"),
    "k difference not folded": (KERNEL, "fold_q", lambda dk, a: dk, "circulant"),
    "trace operand transposed": (OBSERVABLES, "_trace_prod", _transposed_trace, "two_level"),
    "channel-wise: off-diagonal channel reads its own pair": (PROPAGATE.ChannelOp, "apply", _channel_wrong_source,
                                                            "channel_full_rank"),
    "adjoint: commutator pullback order swapped": (ADJOINT, "pull_commutator", _pull_commutator_unconjugated,
                                                   "adjoint_factors"),
    "adjoint: state cotangent sign flipped": (ADJOINT, "pull_commutator", _pull_commutator_ybar_sign,
                                              "adjoint_fields"),
    "adjoint: field pullback not conjugated": (ADJOINT, "pull_field", _pull_field_no_conj, "adjoint_fields"),
    "adjoint: omega derivative sign": (ADJOINT, "field_param_derivs", _omega_derivative_sign, "adjoint_fields"),
    "adjoint: occupation cotangent on the wrong band": (ADJOINT, "observable_cotangent", _cotangent_wrong_band,
                                                        "adjoint_fields"),
    "intraband: backward link not conjugate-transposed": (PROPAGATE, "covariant_derivative",
                                                          _backward_link_not_daggered, "intra_rotated"),
    "adjoint: intraband term with the backward link not conjugate-transposed": (
        ADJOINT, "covariant_derivative", _backward_link_not_daggered, "adjoint_intraband"),
    "intraband: drift sign flipped": (PROPAGATE, "covariant_derivative",
                                      lambda *a: -INTRABAND._real_covariant_derivative(*a), "intra_fft"),
    "intraband: grid spacing halved": (INTRABAND, "grid_spacing",
                                       lambda model, axis: np.pi / ((model.nk1, model.nk2)[axis] * model.a),
                                       "intra_fft"),
    "intraband: axes swapped": (INTRABAND, "_neighbour",
                                lambda model, axis, step: INTRABAND._real_neighbour(model, 1 - axis, step),
                                "intra_fft"),
    "intraband: raw overlap instead of its polar factor": (INTRABAND, "polar_unitary", lambda b: b.copy(),
                                                           "intra_charge"),
    "equilibrium: one band too many filled": (PROPAGATE, "rho_equilibrium", _one_band_too_many_filled,
                                               "two_level"),
    "current not averaged over the k grid": (PROPAGATE, "observables", _current_not_averaged, "two_level"),
    "low rank: V^H applied unconjugated": (PROPAGATE.LowRankOp, "apply", _vh_unconjugated, "lowrank_full_rank"),
    "compression: diagonal left in K_off": (COMPRESS, "split_diag", _diagonal_left_in, "eckart_young"),
    "compression: eigenvector route drops the eigenvalue signs": (COMPRESS, "svd_offdiag",
                                                                  _eigh_route_without_signs, "eckart_young"),
    "compression: fraction rule keeps one value too many": (COMPRESS, "choose_rank", _fraction_off_by_one,
                                                             "rank_rules"),
    "randomized: V^H unconjugated": (COMPRESS, "randomized_compress", _randomized_vh_unconjugated,
                                     "randomized_full_width"),
    "randomized: Ritz value signs dropped": (COMPRESS, "randomized_compress", _randomized_ritz_signs_dropped,
                                             "randomized_full_width"),
    "intraband: polar factor conjugate-transposed": (INTRABAND, "polar_unitary",
                                                     lambda b: np.linalg.svd(b)[2].conj().T
                                                     @ np.linalg.svd(b)[0].conj().T, "intra_rotated"),
    "linear response (e-h): the conjugate partner rows dropped": (BSE, "sector_trace",
                                                                  _sector_trace_partner_dropped, "weak_tda"),
    "linear response: trace operand transposed": (BSE, "sector_trace", _sector_trace_transposed, "weak_tda"),
    "absorption: frequency prefactor dropped": (SPECTRA, "absorption", _absorption_no_frequency, "absorption"),
    "hhg: frequency prefactor dropped": (SPECTRA, "hhg", _hhg_no_frequency, "hhg"),
    "hhg: time step dropped": (SPECTRA, "hhg", _hhg_no_dt, "hhg"),
    "harmonic loss taken at the fundamental": (ADJOINT, "harmonic_loss", _harmonic_loss_fundamental,
                                               "harmonic_loss"),
}


def _run_pin(name, small):
    d6, t4 = small
    if name == "weak_bse":
        pins.test_weak_pulse_matches_bse_linear_response(d6, O.build_kernel(d6, R0_STABLE, "all"))
    elif name == "weak_tda":
        pins.test_weak_pulse_matches_tamm_dancoff_linear_response(t4, O.build_kernel(t4, R0_STABLE, "eh"))
    elif name == "absorption":
        pins.test_absorption_matches_sum_over_states(t4, O.build_kernel(t4, R0_STABLE, "eh"))
    elif name == "hhg":
        pins.test_hhg_of_a_pure_harmonic_closed_form()
    elif name == "harmonic_loss":
        pins.test_harmonic_loss_closed_form()
    elif name == "two_level":
        pins.test_two_level_closed_form(d6)
    elif name == "hermitian":
        pins.test_kernel_hermitian_and_pair_swap(d6, KERNEL.build_kernel(d6, R0_STABLE, "all"))
    elif name == "row_sum":
        pins.test_kernel_row_sum_is_brillouin_zone_integral()
    elif name == "circulant":
        pins.test_flat_band_kernel_is_circulant()
    elif name in ("lowrank_full_rank", "eckart_young", "rank_rules", "randomized_full_width"):
        k = O.build_kernel(t4, R0_STABLE, "eh")
        if name == "lowrank_full_rank":
            pins.test_lowrank_full_rank_equals_dense(t4, k)
        elif name == "eckart_young":
            pins.test_svd_eckart_young(k)
        elif name == "rank_rules":
            pins.test_rank_rules(k)
        else:
            pins.test_randomized_full_width_is_exact(k)
    elif name == "channel_full_rank":
        pins.test_channelwise_full_rank_equals_dense(t4, O.build_kernel(t4, R0_STABLE, "eh"))
    elif name.startswith("intra_"):
        import test_oracle_intraband as intra
        if name == "intra_fft":
            intra.test_drift_matches_fft_closed_form(0.8, 0.6)
        elif name == "intra_rotated":
            intra.test_rotated_degenerate_bases_give_the_same_dynamics()
        else:
            intra.test_total_charge_and_equilibrium_conserved(tb4_model(6, A, 0.5))
    elif name == "adjoint_intraband":
        import test_oracle_adjoint as adj
        adj.test_adjoint_with_intraband_term(t4, O.LowRankOp.from_factors(
            O.compress(O.build_kernel(t4, R0_STABLE, "eh"), "rank", 12)))
    elif name in ("adjoint_fields", "adjoint_factors"):
        import test_oracle_adjoint as adj
        lr = O.LowRankOp.from_factors(O.compress(O.build_kernel(t4, R0_STABLE, "eh"), "rank", 12))
        if name == "adjoint_fields":
            adj.test_adjoint_field_params_lowrank_eh(t4, lr)
        else:
            adj.test_adjoint_lowrank_factors_and_initial_state(t4, lr)


@pytest.mark.parametrize("case", sorted(CASES))
def test_planted_mistake_is_caught(case, small, monkeypatch):
    target, attr, repl, pin = CASES[case]
    _run_pin(pin, small)                       # passes on the real oracle
    orig = getattr(target, attr)
    monkeypatch.setattr(target, attr, repl)
    if getattr(O, attr, None) is orig:
        monkeypatch.setattr(O, attr, repl)     # the package's re-export of the same function
    with pytest.raises(AssertionError):
        _run_pin(pin, small)
