"""Diagonal / off-diagonal split and truncated SVD of the kernel (oracle).

Paper, Sec. "SVD analysis of electron-hole kernel":
  * K_0 = K_0^diag + K_0^off, where K_0^diag holds the elements with
    (n1, n2, k) = (n3, n4, k') -- the matrix diagonal, 1/(N_b^2 N_k) of K_0 --
    and K_0^off the rest;
  * K_0^off is replaced by its rank-z truncated SVD, Eq. (svd_diag_offdiag):
    K~_0 = K_0^diag + U~ M~ V~^T.  For a complex kernel the right factor is
    read as V^H (K_off = U diag(s) V^H);
  * Eq. (svd_acc) uses S~ = U~ M~, so the oracle returns US = U_r diag(s_r)
    and Vh = V_r^H.
Rank rules: keep singular values above a fraction of the largest ("rel_cut",
strict >), keep a fraction of all singular values ("fraction"), a fixed
rank ("rank"), or the smallest rank reaching a reconstruction R^2 ("r2",
R^2 = 1 - sum|y - yhat|^2 / sum|y - ybar|^2 over the elements of K_off, with
sum|y - yhat|^2 equal to the discarded sum of s_i^2 by Eckart-Young).
A cut never splits a group of equal singular values (equal to within
1e-9 s_max): the rank is raised to the end of the group, so the truncated
kernel is unique.
"""

from __future__ import annotations

import numpy as np

MULTIPLET_TOL = 1e-9


def split_diag(k: np.ndarray):
    kdiag = np.diag(k).copy()
    koff = k.copy()
    np.fill_diagonal(koff, 0.0)
    return kdiag, koff


def svd_offdiag(koff: np.ndarray, method: str = "svd"):
    """U, s, Vh of K_off with s descending.

    method "svd" is the plain LAPACK SVD.  method "eigh" uses that K_off is
    Hermitian: K_off = Q diag(l) Q^H gives s = |l|, U = Q sign(l), V = Q
    (same factors, used only where a full SVD is too slow on the CPU).
    """
    if method == "svd":
        u, s, vh = np.linalg.svd(koff)
        return u, s, vh
    lam, q = np.linalg.eigh(koff)
    order = np.argsort(-np.abs(lam), kind="stable")
    lam = lam[order]
    q = q[:, order]
    s = np.abs(lam)
    sign = np.where(lam < 0, -1.0, 1.0)
    return q * sign[None, :], s, q.conj().T


def choose_rank(s: np.ndarray, rule: str, value: float, koff_fro2: float | None = None,
                koff_mean_dev2: float | None = None) -> int:
    n = s.shape[0]
    if rule == "rel_cut":
        r = int(np.count_nonzero(s > value * s[0]))
    elif rule == "fraction":
        r = int(max(1, round(value * n)))
    elif rule == "rank":
        r = int(value)
    elif rule == "r2":
        # tail[r] = sum_{i >= r} s_i^2 is the squared residual at rank r
        tail = np.concatenate([np.cumsum((s ** 2)[::-1])[::-1], [0.0]])
        r2 = 1.0 - tail / koff_mean_dev2
        r = int(np.argmax(r2 >= value))
    else:
        raise ValueError(rule)
    r = min(max(r, 0), n)
    while 0 < r < n and s[r - 1] - s[r] <= MULTIPLET_TOL * s[0]:
        r += 1
    return r


def compress(k: np.ndarray, rule: str = "rel_cut", value: float = 1e-3, method: str = "svd"):
    """Truncated factorisation of K: dict(kdiag, US, Vh, s, r, tail_fro, tail_spec)."""
    kdiag, koff = split_diag(k)
    u, s, vh = svd_offdiag(koff, method)
    dev2 = float(np.sum(np.abs(koff - koff.mean()) ** 2))
    r = choose_rank(s, rule, value, koff_mean_dev2=dev2)
    us = u[:, :r] * s[None, :r]
    return {
        "kdiag": kdiag,
        "US": np.ascontiguousarray(us),
        "Vh": np.ascontiguousarray(vh[:r]),
        "s": s,
        "r": r,
        "tail_fro": float(np.sqrt(np.sum(s[r:] ** 2))),
        "tail_spec": float(s[r]) if r < s.shape[0] else 0.0,
    }


def randomized_compress(k: np.ndarray, rank: int, omega: np.ndarray, power_iters: int = 2):
    """Truncated factorisation of K through a randomized range finder.

    Not part of the paper (its SVD is exact); a standard randomized range
    finder with power iterations and a Rayleigh-Ritz step on the Hermitian
    K_off (Halko, Martinsson and Tropp, SIAM Review 53 (2011), Algs. 4.3/4.4
    and 5.3), used when an exact decomposition of K_off is too large:
      Y = K_off Omega;  repeat power_iters times: Q = orth(Y), Y = K_off Q;
      Q = orth(Y);  T = Q^H K_off Q;  T = W diag(l) W^H;
      keep the `rank` largest |l| (never splitting equal values);
      S = (Q W)_r diag(l_r),  V^H = (Q W)_r^H.
    omega: [n][l] test matrix, l >= rank.  Returns the dict of compress().
    """
    kdiag, koff = split_diag(k)
    y = koff @ omega
    for _ in range(power_iters):
        q, _ = np.linalg.qr(y)
        y = koff @ q
    q, _ = np.linalg.qr(y)
    t = q.conj().T @ (koff @ q)
    t = 0.5 * (t + t.conj().T)
    lam, w = np.linalg.eigh(t)
    order = np.argsort(-np.abs(lam), kind="stable")
    lam, w = lam[order], w[:, order]
    s = np.abs(lam)
    r = choose_rank(s, "rank", rank)
    u = q @ w[:, :r]
    return {
        "kdiag": kdiag,
        "US": np.ascontiguousarray(u * lam[None, :r]),
        "Vh": np.ascontiguousarray(u.conj().T),
        "s": s,
        "r": r,
    }


def channel_blocks(k: np.ndarray, nk: int, npair: int):
    """Channel (p, q) of K: the N_k x N_k block K[k P + p, k' P + q] over k, k'
    (paper Sec. "SVD analysis of electron-hole kernel": a channel is a
    transition (n1 n2) -> (n3 n4) between band pairs, over k and k')."""
    kk = k.reshape(nk, npair, nk, npair)
    return {(p, q): np.ascontiguousarray(kk[:, p, :, q]) for p in range(npair) for q in range(npair)}


def compress_channelwise(k: np.ndarray, nk: int, npair: int, rule: str = "fraction", value: float = 0.05):
    """Channel-wise truncated SVD, Eq. (svd-channel-wise): every off-diagonal
    channel (p != q) K^{pq} ~ U~ M~ V~^H with its own rank (the rule applied to
    that channel's singular values, N_k of them; R^2 over that channel's
    elements); the diagonal channels are kept whole, as in the paper's
    "K^{diag-ch} + 5 % K^{off-ch}".  Returns dict(diag {p: [nk][nk]},
    off {(p, q): (S = U M [nk][r], V^H [r][nk], s)}, ranks {(p, q): r})."""
    blocks = channel_blocks(k, nk, npair)
    out = {"diag": {}, "off": {}, "ranks": {}}
    for (p, q), a in blocks.items():
        if p == q:
            out["diag"][p] = a
            out["ranks"][(p, q)] = nk
            continue
        u, s, vh = np.linalg.svd(a)
        dev2 = float(np.sum(np.abs(a - a.mean()) ** 2))
        r = choose_rank(s, rule, value, koff_mean_dev2=dev2)
        out["off"][(p, q)] = (np.ascontiguousarray(u[:, :r] * s[None, :r]), np.ascontiguousarray(vh[:r]), s)
        out["ranks"][(p, q)] = r
    return out
