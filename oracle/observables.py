"""Observables of the density matrix (oracle).

Paper, Sec. "SVD acceleration of TD-aGW": the absorption spectrum follows
from the polarisation P(t); the high-harmonic spectrum from the current
J(t) = Tr(rho(t) v) with v the velocity operator; the band occupation of the
first conduction band is (1/N_k) sum_k rho_{c1 c1 k}(t).  P and J are taken
along the field direction e and normalised per k point as the occupation is:
  P = (1/N_k) sum_k Tr(e.d_k rho_k),  J = (1/N_k) sum_k Tr(e.v_k rho_k),
real parts reported.  Two diagnostics ride along: the largest deviation of a
per-k trace from the number of valence bands, and the largest element of
rho_k - rho_k^H.  With the intraband (k-derivative) field coupling charge
moves between k points, so the trace diagnostic is then the deviation of the
grid average, |(1/N_k) sum_k Tr rho_k - N_v|.
"""

from __future__ import annotations

import numpy as np


def _trace_prod(a: np.ndarray, rho: np.ndarray) -> complex:
    # sum_k Tr(a_k rho_k) = sum_k sum_nm a_k[n, m] rho_k[m, n]
    return complex(np.einsum("knm,kmn->", a, rho))


def observables(model, rho: np.ndarray, ex: float, ey: float, grid_trace: bool = False) -> dict:
    nk = model.nk
    d = ex * model.dip[0] + ey * model.dip[1]
    v = ex * model.vel[0] + ey * model.vel[1]
    tr = np.einsum("knn->k", rho)
    return {
        "P": _trace_prod(d, rho).real / nk,
        "J": _trace_prod(v, rho).real / nk,
        "occ": float(np.sum(rho[:, model.nv, model.nv].real)) / nk,
        "tr": float(abs(np.mean(tr) - model.nv)) if grid_trace else float(np.max(np.abs(tr - model.nv))),
        "herm": float(np.max(np.abs(rho - rho.conj().transpose(0, 2, 1)))),
    }
