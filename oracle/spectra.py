"""Spectra from time series (oracle).

Paper, Sec. "SVD acceleration of TD-aGW": the absorption spectrum is the
Fourier transform of the polarisation after a pulse; the high-harmonic
spectrum is HHG(w) = |w int J(t) exp(-i w t) dt|^2.  Readings: the transform
is a plain sum over the samples t_n = n dt with an exp(-eta t) damping, and
A(w) = w Im[P(w) / E(w)] with both transforms taken the same way.
"""

from __future__ import annotations

import numpy as np


def _ft(x: np.ndarray, dt: float, omegas: np.ndarray, eta: float, sign: float) -> np.ndarray:
    t = np.arange(x.shape[0]) * dt
    ph = np.exp(sign * 1j * np.outer(omegas, t) - eta * t[None, :])
    return ph @ x * dt


def absorption(p: np.ndarray, e: np.ndarray, dt: float, omegas: np.ndarray, eta: float) -> np.ndarray:
    pw = _ft(p - p[0], dt, omegas, eta, +1.0)
    ew = _ft(e, dt, omegas, eta, +1.0)
    return omegas * (pw / ew).imag


def hhg(j: np.ndarray, dt: float, omegas: np.ndarray) -> np.ndarray:
    jw = _ft(j, dt, omegas, 0.0, -1.0)
    return np.abs(omegas * jw) ** 2
