"""Lattice models standing in for the paper's mean-field inputs.

The method consumes band energies, Bloch states, a position (dipole) matrix
and a velocity operator (Eq. tdagw and Appendix A.1 of the paper); the paper
takes them from DFT + GW.  Here they come from two small tight-binding models:

* a two-band massive Dirac lattice model  H(k) = D sz + t (sin kx a sx + sin ky a sy);
* a seeded random Hermitian four-band nearest-neighbour model
  H(k) = H0 + sum_a (T_a exp(i k_a a) + h.c.),  H0 = diag(D, D, -D, -D).

Hartree atomic units throughout (energies in Ha, lengths in bohr).
Layouts (all C-contiguous):
  kpts  [nk][2]        float64, k index = i1 * nk2 + i2
  eps   [nk][nb]       float64, ascending
  evec  [nk][nb][nb]   complex128, evec[k][alpha, n] = <alpha | n k>
  vel   [2][nk][nb][nb] complex128, v^a_nm = <n k| dH/dk_a |m k>
  dip   [2][nk][nb][nb] complex128, interband Berry connection
"""

from __future__ import annotations

import json
import os
from dataclasses import dataclass

import numpy as np

HARTREE_EV = 27.211386245988          # eV per hartree
FS_AU = 41.341373335                  # atomic time units per femtosecond
BOHR_NM = 0.0529177210903             # nm per bohr
EFIELD_AU_V_PER_CM = 5.14220674763e9  # V/cm per atomic unit of field

_DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


@dataclass
class Model:
    name: str
    nk1: int
    nk2: int
    shift: float
    a: float
    nb: int
    nv: int
    kpts: np.ndarray
    eps: np.ndarray
    evec: np.ndarray
    vel: np.ndarray
    dip: np.ndarray
    hk: np.ndarray

    @property
    def nk(self) -> int:
        return self.nk1 * self.nk2

    @property
    def nc(self) -> int:
        return self.nb - self.nv


def mp_grid(nk1: int, nk2: int, a: float, shift: float = 0.5) -> np.ndarray:
    """Uniform grid k_i = (2 pi / a) ((i + shift) / N - 1/2), i = 0..N-1.

    shift = 0.5 is the Monkhorst-Pack grid for even N (Gamma excluded);
    shift = 0 is Gamma-centred for even N.
    """
    g1 = (2.0 * np.pi / a) * ((np.arange(nk1) + shift) / nk1 - 0.5)
    g2 = (2.0 * np.pi / a) * ((np.arange(nk2) + shift) / nk2 - 0.5)
    kx, ky = np.meshgrid(g1, g2, indexing="ij")
    return np.stack([kx.ravel(), ky.ravel()], axis=1)


_SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def _canonical_phase(evec: np.ndarray) -> np.ndarray:
    """Fix each eigenvector's phase: its largest-magnitude component is made
    real and positive (the lowest orbital index among components within 1e-9
    of the maximum)."""
    mag = np.abs(evec)                                 # [nk][alpha][n]
    mx = mag.max(axis=1, keepdims=True)
    first = np.argmax(mag >= mx * (1.0 - 1e-9), axis=1)  # [nk][n]
    comp = np.take_along_axis(evec, first[:, None, :], axis=1)[:, 0, :]
    phase = comp / np.abs(comp)
    return evec / phase[:, None, :]


def _bands(hk: np.ndarray, dh: np.ndarray, nv: int):
    """Diagonalise H(k) and express dH/dk and the Berry connection in the band basis."""
    eps, evec = np.linalg.eigh(hk)
    evec = _canonical_phase(evec)
    vel = np.einsum("kan,xkab,kbm->xknm", evec.conj(), dh, evec)
    nb = hk.shape[-1]
    de = eps[:, None, :] - eps[:, :, None]             # de[k, n, m] = e_m - e_n
    inter = np.zeros((nb, nb), dtype=bool)
    inter[:nv, nv:] = True
    inter[nv:, :nv] = True
    dip = np.zeros_like(vel)
    safe = np.where(inter[None], de, 1.0)
    dip[:, :, inter] = (1j * vel / safe[None])[:, :, inter]
    return eps, evec, vel, dip


def dirac_model(nk: int = 12, delta_ev: float = 1.0, t_ev: float = 1.5,
                a: float = 6.0, shift: float = 0.5) -> Model:
    """Two-band massive Dirac lattice model, one valence and one conduction band."""
    kpts = mp_grid(nk, nk, a, shift)
    d = delta_ev / HARTREE_EV
    t = t_ev / HARTREE_EV
    sx = np.sin(kpts[:, 0] * a)[:, None, None]
    sy = np.sin(kpts[:, 1] * a)[:, None, None]
    cx = np.cos(kpts[:, 0] * a)[:, None, None]
    cy = np.cos(kpts[:, 1] * a)[:, None, None]
    hk = d * _SZ[None] + t * (sx * _SX[None] + sy * _SY[None])
    dh = np.stack([t * a * cx * _SX[None], t * a * cy * _SY[None]])
    eps, evec, vel, dip = _bands(hk, dh, 1)
    return Model("dirac", nk, nk, shift, a, 2, 1, kpts, eps, evec, vel, dip, hk)


def draw_tb4_hoppings(seed: int):
    """Seeded draw of the two 4x4 hopping matrices (eV): magnitudes U[0.2, 1.0],
    phases U[0, 2 pi); draw order |Tx|, arg Tx, |Ty|, arg Ty (PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(2):
        mag = rng.uniform(0.2, 1.0, size=(4, 4))
        ph = rng.uniform(0.0, 2.0 * np.pi, size=(4, 4))
        out.append(mag * np.exp(1j * ph))
    return out[0], out[1]


def tb4_hamiltonian(kpts: np.ndarray, a: float, tx: np.ndarray, ty: np.ndarray,
                    delta: float):
    """H(k) and dH/dk for the four-band model; tx, ty, delta in hartree."""
    h0 = np.diag([delta, delta, -delta, -delta]).astype(np.complex128)
    ex = np.exp(1j * kpts[:, 0] * a)[:, None, None]
    ey = np.exp(1j * kpts[:, 1] * a)[:, None, None]
    txh = tx.conj().T
    tyh = ty.conj().T
    hk = h0[None] + tx[None] * ex + txh[None] * ex.conj() + ty[None] * ey + tyh[None] * ey.conj()
    dhx = 1j * a * (tx[None] * ex - txh[None] * ex.conj())
    dhy = 1j * a * (ty[None] * ey - tyh[None] * ey.conj())
    return hk, np.stack([dhx, dhy])


def load_tb4_table(path: str | None = None) -> dict:
    """The stored four-band model (seed, hoppings, on-site splitting)."""
    path = path or os.path.join(_DATA, "tb4_model.json")
    with open(path) as f:
        tab = json.load(f)
    tab["tx"] = np.array(tab["tx_re"]) + 1j * np.array(tab["tx_im"])
    tab["ty"] = np.array(tab["ty_re"]) + 1j * np.array(tab["ty_im"])
    return tab


def tb4_model(nk: int, a: float = 6.0, shift: float = 0.5, table: dict | None = None) -> Model:
    """Seeded random 4-band model (2 valence + 2 conduction bands) on an nk x nk grid."""
    tab = table or load_tb4_table()
    kpts = mp_grid(nk, nk, a, shift)
    hk, dh = tb4_hamiltonian(kpts, a, tab["tx"] / HARTREE_EV, tab["ty"] / HARTREE_EV,
                             tab["delta_ev"] / HARTREE_EV)
    eps, evec, vel, dip = _bands(hk, dh, 2)
    return Model("tb4", nk, nk, shift, a, 4, 2, kpts, eps, evec, vel, dip, hk)


def multiband_model(nk: int, nb: int = 8, nv: int = 4, seed: int = 3, a: float = 6.0, shift: float = 0.5,
                    delta_ev: float = 3.0, tmin_ev: float = 0.05, tmax_ev: float = 0.2) -> Model:
    """Seeded random nb-band nearest-neighbour model (edge cases with many
    bands): H0 = diag(+delta on nb - nv bands, -delta on nv bands), hoppings
    T_x, T_y with magnitudes U[tmin, tmax] eV and phases U[0, 2 pi) drawn in
    the order |Tx|, arg Tx, |Ty|, arg Ty from PCG64(seed); the small hoppings
    keep the nv lowest bands separated from the others."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ts = []
    for _ in range(2):
        mag = rng.uniform(tmin_ev, tmax_ev, size=(nb, nb))
        ph = rng.uniform(0.0, 2.0 * np.pi, size=(nb, nb))
        ts.append(mag * np.exp(1j * ph) / HARTREE_EV)
    tx, ty = ts
    kpts = mp_grid(nk, nk, a, shift)
    d = delta_ev / HARTREE_EV
    h0 = np.diag([d] * (nb - nv) + [-d] * nv).astype(np.complex128)
    ex = np.exp(1j * kpts[:, 0] * a)[:, None, None]
    ey = np.exp(1j * kpts[:, 1] * a)[:, None, None]
    hk = h0[None] + tx[None] * ex + tx.conj().T[None] * ex.conj() + ty[None] * ey + ty.conj().T[None] * ey.conj()
    dhx = 1j * a * (tx[None] * ex - tx.conj().T[None] * ex.conj())
    dhy = 1j * a * (ty[None] * ey - ty.conj().T[None] * ey.conj())
    eps, evec, vel, dip = _bands(hk, np.stack([dhx, dhy]), nv)
    return Model(f"mb{nb}", nk, nk, shift, a, nb, nv, kpts, eps, evec, vel, dip, hk)


def _haar_unitary(rng: np.random.Generator, n: int) -> np.ndarray:
    """Haar-random n x n unitary (QR of a complex Gaussian, phases of R fixed)."""
    z = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    return q * (d / np.abs(d))[None, :]


def flat_band_model(nk1: int, nk2: int, nb: int = 4, nv: int = 2, gap_ev: float = 2.0, a: float = 6.0,
                    shift: float = 0.5, dip_seed: int | None = None, dip_bohr: float = 1.0,
                    gauge_seed: int | None = None) -> Model:
    """Flat degenerate bands on an nk1 x nk2 grid: nv valence bands at -gap/2 and
    nb - nv conduction bands at +gap/2, H(k) constant, velocity zero.

    dip_seed draws a constant interband dipole d0 in the orbital basis
    (Hermitian, nonzero only between the two subspaces, entries of magnitude
    U[0.2, 1] dip_bohr, phases U[0, 2 pi)); None gives d0 = 0.  gauge_seed
    draws, per k, Haar-random unitaries R_v(k) and R_c(k) within the two
    degenerate subspaces and uses them as the Bloch states, evec_k =
    blockdiag(R_v, R_c), with dip_k = evec_k^H d0 evec_k; None keeps evec = I.
    Draw order (PCG64): d0 magnitudes, d0 phases; then per k R_v, R_c."""
    nk = nk1 * nk2
    g = gap_ev / HARTREE_EV
    kpts = mp_grid(nk1, nk2, a, shift)
    eps = np.tile(np.array([-0.5 * g] * nv + [0.5 * g] * (nb - nv)), (nk, 1))
    hk = np.zeros((nk, nb, nb), dtype=np.complex128)
    hk[:, np.arange(nb), np.arange(nb)] = eps
    d0 = np.zeros((2, nb, nb), dtype=np.complex128)
    if dip_seed is not None:
        rng = np.random.Generator(np.random.PCG64(dip_seed))
        mag = rng.uniform(0.2, 1.0, size=(2, nv, nb - nv)) * dip_bohr
        ph = rng.uniform(0.0, 2.0 * np.pi, size=(2, nv, nb - nv))
        d0[:, :nv, nv:] = mag * np.exp(1j * ph)
        d0[:, nv:, :nv] = d0[:, :nv, nv:].conj().transpose(0, 2, 1)
    evec = np.broadcast_to(np.eye(nb, dtype=np.complex128), (nk, nb, nb)).copy()
    if gauge_seed is not None:
        rng = np.random.Generator(np.random.PCG64(gauge_seed))
        for k in range(nk):
            evec[k, :nv, :nv] = _haar_unitary(rng, nv)
            evec[k, nv:, nv:] = _haar_unitary(rng, nb - nv)
    dip = np.einsum("kan,xab,kbm->xknm", evec.conj(), d0, evec)
    vel = np.zeros_like(dip)
    return Model(f"flat{nb}", nk1, nk2, shift, a, nb, nv, kpts, eps, evec, vel, dip, hk)


def diagonal_band_model(nk1: int, nk2: int, nb: int = 4, nv: int = 2, gap_ev: float = 2.0,
                        width_ev: float = 0.3, a: float = 6.0, shift: float = 0.5) -> Model:
    """Dispersive bands with k-independent Bloch states (evec = I, dipole 0):
    eps_n(k) = c_n + w_n (cos kx a + 0.5 cos ky a), centres 0.2 eV apart within
    each subspace (valence below -gap/2, conduction above +gap/2),
    w_n = width (1 + 0.2 n), so the bands never cross; velocity
    v^a_nn = d eps_n / dk_a (diagonal)."""
    nk = nk1 * nk2
    kpts = mp_grid(nk1, nk2, a, shift)
    g, w, s = gap_ev / HARTREE_EV, width_ev / HARTREE_EV, 0.2 / HARTREE_EV
    cen = np.array([-0.5 * g - (nv - 1 - n) * s for n in range(nv)] + [0.5 * g + n * s for n in range(nb - nv)])
    wid = np.array([w * (1.0 + 0.2 * n) for n in range(nb)])
    cx, cy = np.cos(kpts[:, 0] * a), np.cos(kpts[:, 1] * a)
    sx, sy = np.sin(kpts[:, 0] * a), np.sin(kpts[:, 1] * a)
    eps = cen[None, :] + wid[None, :] * (cx + 0.5 * cy)[:, None]
    vel = np.zeros((2, nk, nb, nb), dtype=np.complex128)
    vel[0][:, np.arange(nb), np.arange(nb)] = -a * wid[None, :] * sx[:, None]
    vel[1][:, np.arange(nb), np.arange(nb)] = -0.5 * a * wid[None, :] * sy[:, None]
    hk = np.zeros((nk, nb, nb), dtype=np.complex128)
    hk[:, np.arange(nb), np.arange(nb)] = eps
    evec = np.broadcast_to(np.eye(nb, dtype=np.complex128), (nk, nb, nb)).copy()
    return Model(f"diag{nb}", nk1, nk2, shift, a, nb, nv, kpts, eps, evec, vel, np.zeros_like(vel), hk)
