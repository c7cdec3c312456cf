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
}


def _run_pin(name, small):
    d6, t4 = small
    if name == "weak_bse":
        pins.test_weak_pulse_matches_bse_linear_response(d6, O.build_kernel(d6, R0_STABLE, "all"))
    elif name == "two_level":
        pins.test_two_level_closed_form(d6)
    elif name == "hermitian":
        pins.test_kernel_hermitian_and_pair_swap(d6, KERNEL.build_kernel(d6, R0_STABLE, "all"))
    elif name == "row_sum":
        pins.test_kernel_row_sum_is_brillouin_zone_integral()
    elif name == "circulant":
        pins.test_flat_band_kernel_is_circulant()


@pytest.mark.parametrize("case", sorted(CASES))
def test_planted_mistake_is_caught(case, small, monkeypatch):
    target, attr, repl, pin = CASES[case]
    _run_pin(pin, small)                       # passes on the real oracle
    monkeypatch.setattr(target, attr, repl)
    if target is KERNEL and attr == "build_kernel":
        monkeypatch.setattr(O, "build_kernel", repl)
    with pytest.raises(AssertionError):
        _run_pin(pin, small)
