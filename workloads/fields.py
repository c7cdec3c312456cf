"""Driving-field parameter tables (no field evaluation here).

The pulse shape used by the configs is a Gaussian-enveloped carrier,
E_b(t) = E0_b exp(-(t - t0_b)^2 / (2 tau_b^2)) cos(omega_b t) along the unit
vector (ex_b, ey_b); each instance b runs nsteps_b RK4 steps.  This module only
stores the parameters (atomic units); each side evaluates E(t) itself.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class FieldTable:
    e0: np.ndarray      # [B] a.u.
    omega: np.ndarray   # [B] Ha
    tau: np.ndarray     # [B] a.u. of time
    t0: np.ndarray      # [B] a.u. of time
    ex: np.ndarray      # [B]
    ey: np.ndarray      # [B]
    nsteps: np.ndarray  # [B] int64

    @property
    def batch(self) -> int:
        return int(self.e0.shape[0])

    def as_records(self) -> np.ndarray:
        """[B][8] float64 rows: e0, omega, tau, t0, ex, ey, nsteps, 0."""
        rec = np.zeros((self.batch, 8), dtype=np.float64)
        rec[:, 0] = self.e0
        rec[:, 1] = self.omega
        rec[:, 2] = self.tau
        rec[:, 3] = self.t0
        rec[:, 4] = self.ex
        rec[:, 5] = self.ey
        rec[:, 6] = self.nsteps
        return rec

    def subset(self, idx) -> "FieldTable":
        idx = np.atleast_1d(idx)
        return FieldTable(self.e0[idx], self.omega[idx], self.tau[idx], self.t0[idx],
                          self.ex[idx], self.ey[idx], self.nsteps[idx])

    @staticmethod
    def single(e0, omega, tau, t0, nsteps, ex=1.0, ey=0.0) -> "FieldTable":
        f = lambda v: np.array([v], dtype=np.float64)  # noqa: E731
        return FieldTable(f(e0), f(omega), f(tau), f(t0), f(ex), f(ey),
                          np.array([nsteps], dtype=np.int64))

    @staticmethod
    def stack(tables) -> "FieldTable":
        cat = lambda name: np.concatenate([getattr(t, name) for t in tables])  # noqa: E731
        return FieldTable(cat("e0"), cat("omega"), cat("tau"), cat("t0"), cat("ex"), cat("ey"),
                          cat("nsteps").astype(np.int64))
