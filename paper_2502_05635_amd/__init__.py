"""Python binding of libtdagw (MI355X TD-aGW propagation with dense or
SVD-compressed electron-hole kernels).

Argument marshalling only: torch tensors provide device memory and the HIP
stream, every computation runs in the library's HIP kernels.  There is no CPU
fallback; loading fails loudly when the library is missing.
"""

from __future__ import annotations

import ctypes as C
import dataclasses
import os
from dataclasses import dataclass

import numpy as np
import torch  # must precede the library load: it binds to torch's HIP runtime

from . import _abi as abi

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtdagw.so")
_LIB = None


class TdgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tdagw error {code}: {msg}")
        self.code = code


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2502_05635_amd.build`")
        handle = C.CDLL(LIB_PATH)
        for name, (args, res) in abi.SIGNATURES.items():
            fn = getattr(handle, name)
            fn.argtypes = args
            fn.restype = res
        _LIB = handle
    return _LIB


def _ptr(t: torch.Tensor | None):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _cdtype(dtype: str):
    if dtype == "c128":
        return abi.TDG_C128, torch.complex128
    if dtype == "c64":
        return abi.TDG_C64, torch.complex64
    if dtype == "bf16x2":  # two bf16 planes, 8 bytes per element like complex64
        return abi.TDG_BF16X2, torch.complex64
    raise ValueError(dtype)


@dataclass
class Bf16x2Matrix:
    """A complex matrix in BF16 split storage (hi plane, then lo plane);
    `data` only provides the device memory (rows * ld * 8 bytes)."""
    data: torch.Tensor
    rows: int
    cols: int
    ld: int

    def data_ptr(self) -> int:
        return self.data.data_ptr()


def _block(block: str) -> int:
    return {"all": abi.TDG_BLOCK_ALL, "eh": abi.TDG_BLOCK_EH}[block]


def field_array(fields) -> C.Array:
    """tdg_field[B] (host) from a FieldTable or a [B][8] float64 array."""
    rec = fields.as_records() if hasattr(fields, "as_records") else np.asarray(fields, dtype=np.float64)
    arr = (abi.Field * rec.shape[0])()
    C.memmove(arr, np.ascontiguousarray(rec, dtype=np.float64).ctypes.data, rec.nbytes)
    return arr


@dataclass
class DeviceModel:
    """Band-structure input resident on the device (caller-owned tensors)."""
    nk1: int
    nk2: int
    nb: int
    nv: int
    shift: float
    a: float
    eps: torch.Tensor
    evec: torch.Tensor
    dip: torch.Tensor
    vel: torch.Tensor
    links: torch.Tensor | None = None   # [2][nk][nb][nb] from Context.links_build: intraband term on

    @staticmethod
    def from_model(m, device="cuda") -> "DeviceModel":
        as_t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)  # noqa: E731
        return DeviceModel(m.nk1, m.nk2, m.nb, m.nv, m.shift, m.a,
                           as_t(m.eps, torch.float64), as_t(m.evec, torch.complex128),
                           as_t(m.dip, torch.complex128), as_t(m.vel, torch.complex128))

    @property
    def nk(self) -> int:
        return self.nk1 * self.nk2

    def struct(self) -> abi.Model:
        return abi.Model(self.nk1, self.nk2, self.nb, self.nv, self.shift, self.a,
                         self.eps.data_ptr(), self.evec.data_ptr(), self.dip.data_ptr(), self.vel.data_ptr(),
                         self.links.data_ptr() if self.links is not None else None)

    def with_links(self, links: torch.Tensor | None) -> "DeviceModel":
        """The same model with the intraband term switched on (links) or off (None)."""
        return dataclasses.replace(self, links=links)


@dataclass
class LowRankFactors:
    kdiag: torch.Tensor
    us: torch.Tensor        # [N][rank]
    w: torch.Tensor         # [rank][N]  (= V^H)
    sigma: np.ndarray       # all singular values of K_off, descending
    rank: int
    tail_fro: float
    tail_spec: float
    dtype: str


@dataclass
class ChannelFactors:
    """Channel-wise compressed kernel (see tdg_channels)."""
    diag: torch.Tensor      # [P][nk][nk]
    s: torch.Tensor         # [nk P][(P - 1) rmax]
    w: torch.Tensor         # [P][P - 1][rmax][nk]
    rmax: int
    ranks: np.ndarray       # [P][P]
    sigma: np.ndarray       # [P][P][nk]
    dtype: str


class Context:
    """A library context bound to one device and the current torch stream."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self._lib = lib()
        self.device = device
        stream = stream or torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        self._check(self._lib.tdg_create(C.byref(h), device, C.c_void_p(stream.cuda_stream)), None)
        self.h = h

    def set_stream(self, stream: torch.cuda.Stream) -> None:
        """Queue later calls on `stream`; it first waits for the work already
        queued on the previous one (tdg_set_stream)."""
        self._check(self._lib.tdg_set_stream(self.h, C.c_void_p(stream.cuda_stream)))
        self.stream = stream

    def close(self):
        if getattr(self, "h", None):
            self._lib.tdg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, h=...):
        if rc != abi.TDG_OK:
            handle = self.h if h is ... else h
            msg = self._lib.tdg_last_error(handle).decode()
            raise TdgError(rc, msg)

    # --- kernel build / compression -------------------------------------
    def kernel_dim(self, model: DeviceModel, block: str) -> int:
        n = C.c_int64()
        ms = model.struct()
        self._check(self._lib.tdg_kernel_dim(C.byref(ms), _block(block), C.byref(n)))
        return n.value

    def links_build(self, model: DeviceModel) -> torch.Tensor:
        """Parallel-transport links [2][nk][nb][nb] complex128 of the model's
        Bloch states (tdg_links_build); pass them with model.with_links()."""
        out = torch.empty((2, model.nk, model.nb, model.nb), dtype=torch.complex128, device=f"cuda:{self.device}")
        ms = model.struct()
        self._check(self._lib.tdg_links_build(self.h, C.byref(ms), _ptr(out)))
        return out

    def kernel_build(self, model: DeviceModel, r0: float, block: str, dtype: str = "c128",
                     nquad: int = 64, out: torch.Tensor | None = None):
        code, tdt = _cdtype(dtype)
        n = self.kernel_dim(model, block)
        ms = model.struct()
        cs = abi.Coulomb(r0, _block(block), nquad)
        if dtype == "bf16x2":
            ld = (n + 3) // 4 * 4
            mat = Bf16x2Matrix(torch.empty(n * ld, dtype=tdt, device=f"cuda:{self.device}"), n, n, ld)
            self._check(self._lib.tdg_kernel_build(self.h, C.byref(ms), C.byref(cs), code, _ptr(mat), ld))
            return mat
        if out is None:
            out = torch.empty((n, n), dtype=tdt, device=f"cuda:{self.device}")
        self._check(self._lib.tdg_kernel_build(self.h, C.byref(ms), C.byref(cs), code, _ptr(out), out.stride(0)))
        return out

    def kernel_compress(self, K: torch.Tensor, rule: str = "rel_cut", value: float = 1e-3,
                        max_rank: int | None = None, out_dtype: str | None = None) -> LowRankFactors:
        """Truncated SVD of K_off; factors in out_dtype (default: K's dtype;
        "bf16x2" writes split-precision factors with a complex64 K_diag)."""
        kdtype = "c128" if K.dtype == torch.complex128 else "c64"
        kcode, _ = _cdtype(kdtype)
        dtype = out_dtype or kdtype
        code, tdt = _cdtype(dtype)
        n = K.shape[0]
        max_rank = n if max_rank is None else int(max_rank)
        dev = K.device
        kdiag = torch.empty(n, dtype=tdt, device=dev)
        us = torch.empty(n * (max_rank + 3), dtype=tdt, device=dev)
        w = torch.empty(n * max_rank, dtype=tdt, device=dev)
        sigma = np.zeros(n, dtype=np.float64)
        lr = abi.LowRank(n, max_rank, code, 0, kdiag.data_ptr(), us.data_ptr(), w.data_ptr(),
                         sigma.ctypes.data, 0, 0.0, 0.0)
        tr = abi.Trunc(abi.TDG_TRUNC[rule], 0, float(value))
        self._check(self._lib.tdg_kernel_compress(self.h, _ptr(K), K.stride(0), kcode, C.byref(tr), C.byref(lr)))
        return self._factors(kdiag, us, w, sigma, lr, dtype)

    @staticmethod
    def _factors(kdiag, us, w, sigma, lr, dtype) -> LowRankFactors:
        n, r = int(lr.n), int(lr.rank)
        if dtype == "bf16x2":
            return LowRankFactors(kdiag, us, w, sigma, r, lr.tail_fro, lr.tail_spec, dtype)
        return LowRankFactors(kdiag, us[: n * r].view(n, r), w[: n * r].view(r, n), sigma, r,
                              lr.tail_fro, lr.tail_spec, dtype)

    def kernel_compress_randomized(self, K: torch.Tensor, omega_t: torch.Tensor, rule: str = "rank",
                                   value: float = 1.0, power_iters: int = 2, max_rank: int | None = None,
                                   out_dtype: str | None = None) -> LowRankFactors:
        """Randomized range-finder factorisation of K_off.  omega_t is the
        test matrix transposed, a contiguous complex128 device tensor [l][n]
        (row j = test vector j); sigma holds the l Ritz values."""
        kdtype = "c128" if K.dtype == torch.complex128 else "c64"
        kcode, _ = _cdtype(kdtype)
        dtype = out_dtype or kdtype
        code, tdt = _cdtype(dtype)
        n = K.shape[0]
        if omega_t.dtype != torch.complex128 or not omega_t.is_contiguous() or omega_t.shape[1] != n:
            raise ValueError("omega_t must be a contiguous complex128 tensor [l][n]")
        l = omega_t.shape[0]
        max_rank = min(n, l) if max_rank is None else int(max_rank)
        dev = K.device
        kdiag = torch.empty(n, dtype=tdt, device=dev)
        us = torch.empty(n * (max_rank + 3), dtype=tdt, device=dev)
        w = torch.empty(n * max_rank, dtype=tdt, device=dev)
        sigma = np.zeros(l, dtype=np.float64)
        lr = abi.LowRank(n, max_rank, code, 0, kdiag.data_ptr(), us.data_ptr(), w.data_ptr(),
                         sigma.ctypes.data, 0, 0.0, 0.0)
        tr = abi.Trunc(abi.TDG_TRUNC[rule], 0, float(value))
        self._check(self._lib.tdg_kernel_compress_randomized(self.h, _ptr(K), K.stride(0), kcode, C.byref(tr),
                                                             _ptr(omega_t), l, int(power_iters), C.byref(lr)))
        return self._factors(kdiag, us, w, sigma, lr, dtype)

    def kernel_compress_channels(self, K: torch.Tensor, nk: int, npair: int, rule: str = "fraction",
                                 value: float = 0.05, rmax: int | None = None,
                                 out_dtype: str | None = None) -> ChannelFactors:
        """Channel-wise truncated SVD (off-diagonal channels), diagonal channels kept."""
        kdtype = "c128" if K.dtype == torch.complex128 else "c64"
        kcode, _ = _cdtype(kdtype)
        dtype = out_dtype or kdtype
        code, tdt = _cdtype(dtype)
        rmax = (nk + 3) // 4 * 4 if rmax is None else int(rmax)
        rmax = min(rmax, nk // 4 * 4)
        dev = K.device
        diag = torch.empty((npair, nk, nk), dtype=tdt, device=dev)
        s = torch.empty((nk * npair, (npair - 1) * rmax), dtype=tdt, device=dev)
        w = torch.empty((npair, npair - 1, rmax, nk), dtype=tdt, device=dev)
        ranks = np.zeros((npair, npair), dtype=np.int64)
        sigma = np.zeros((npair, npair, nk), dtype=np.float64)
        ch = abi.Channels(nk, npair, code, rmax, diag.data_ptr(), s.data_ptr(), w.data_ptr(), ranks.ctypes.data,
                          sigma.ctypes.data)
        tr = abi.Trunc(abi.TDG_TRUNC[rule], 0, float(value))
        self._check(self._lib.tdg_kernel_compress_channels(self.h, _ptr(K), K.stride(0), kcode, C.byref(tr),
                                                           C.byref(ch)))
        return ChannelFactors(diag, s, w, rmax, ranks, sigma, dtype)

    # --- propagation --------------------------------------------------------
    def _operator(self, op, block: str, n: int) -> abi.Operator:
        if isinstance(op, ChannelFactors):
            code, _ = _cdtype(op.dtype)
            return abi.Operator(abi.TDG_OP_CHANNEL, code, _block(block), 0, n, op.diag.data_ptr(), 0,
                                None, op.s.data_ptr(), op.w.data_ptr(), op.rmax)
        if isinstance(op, LowRankFactors):
            code, _ = _cdtype(op.dtype)
            return abi.Operator(abi.TDG_OP_LOWRANK, code, _block(block), 0, n, None, 0,
                                op.kdiag.data_ptr(), op.us.data_ptr(), op.w.data_ptr(), op.rank)
        if isinstance(op, Bf16x2Matrix):
            return abi.Operator(abi.TDG_OP_DENSE, abi.TDG_BF16X2, _block(block), 0, n, op.data_ptr(), op.ld,
                                None, None, None, 0)
        code, _ = _cdtype("c128" if op.dtype == torch.complex128 else "c64")
        return abi.Operator(abi.TDG_OP_DENSE, code, _block(block), 0, n, op.data_ptr(), op.stride(0),
                            None, None, None, 0)

    def propagate(self, op, model: DeviceModel, block: str, fields, dt: float,
                  rho: torch.Tensor | None = None, init_eq: bool | None = None,
                  diagnostics: bool = True, _entry: str = "tdg_propagate") -> dict:
        """Integrate every instance of `fields`; returns device tensors
        P, J, occ (and tr, herm) of shape [B][max nsteps + 1] and rho(T)."""
        fa = field_array(fields)
        batch = len(fa)
        maxn = max((int(f.nsteps) for f in fa), default=0)
        dev = f"cuda:{self.device}"
        if rho is None:
            rho = torch.empty((batch, model.nk, model.nb, model.nb), dtype=torch.complex128, device=dev)
            init_eq = True if init_eq is None else init_eq
        init_eq = bool(init_eq)
        stride = maxn + 1
        names = ("P", "J", "occ", "tr", "herm") if diagnostics else ("P", "J", "occ")
        # every entry up to an instance's own length is written; only shorter
        # instances leave a tail, which is zeroed
        even = all(int(f.nsteps) == maxn for f in fa)
        buf = (torch.empty if even else torch.zeros)((len(names), batch, stride), dtype=torch.float64, device=dev)
        arrs = {k: buf[i] for i, k in enumerate(names)}
        obs = abi.Obs(arrs["P"].data_ptr(), arrs["J"].data_ptr(), arrs["occ"].data_ptr(),
                      arrs["tr"].data_ptr() if diagnostics else None,
                      arrs["herm"].data_ptr() if diagnostics else None, stride)
        n = self.kernel_dim(model, block)
        opr = self._operator(op, block, n)
        ms = model.struct()
        fn = getattr(self._lib, _entry)
        self._check(fn(self.h, C.byref(opr), C.byref(ms), fa, batch, float(dt), _ptr(rho), int(init_eq),
                       C.byref(obs)))
        arrs["rho"] = rho
        arrs["_obs_struct"] = obs
        return arrs

    def propagate_noalloc(self, op, model: DeviceModel, block: str, fields, dt: float,
                          rho: torch.Tensor | None = None, init_eq: bool | None = None,
                          diagnostics: bool = True) -> dict:
        """propagate() through tdg_propagate_noalloc: the library allocates
        nothing (its workspace is the per-GPU scratch array); the result
        tensors are still allocated here, by torch."""
        return self.propagate(op, model, block, fields, dt, rho, init_eq, diagnostics, "tdg_propagate_noalloc")

    def propagate_adjoint(self, op, model: DeviceModel, block: str, fields, dt: float, gP=None, gJ=None,
                          gocc=None, rho0: torch.Tensor | None = None, checkpoint_every: int = 50,
                          factor_grads: bool = True) -> dict:
        """Gradient of L = sum_n gP_n P(t_n) + gJ_n J(t_n) + gocc_n occ(t_n) (each [B][nsteps + 1]
        or None) by the adjoint RK4 on the device.  Returns dfield [B][4] (d e0, omega, tau, t0),
        dE [B][nsteps][4], drho0 and, for complex128 low-rank factors, dus and dw."""
        fa = field_array(fields)
        batch = len(fa)
        nsteps = int(fa[0].nsteps)
        dev = f"cuda:{self.device}"
        ws = {}
        for key, g in (("gP", gP), ("gJ", gJ), ("gocc", gocc)):
            if g is not None:
                ws[key] = torch.as_tensor(g, dtype=torch.float64).to(dev).reshape(batch, nsteps + 1).contiguous()
        og = abi.ObsGrad(_ptr(ws.get("gP")), _ptr(ws.get("gJ")), _ptr(ws.get("gocc")), nsteps + 1)
        out = {"dfield": torch.zeros((batch, 4), dtype=torch.float64, device=dev),
               "dE": torch.zeros((batch, nsteps, 4), dtype=torch.float64, device=dev),
               "drho0": torch.zeros((batch, model.nk, model.nb, model.nb), dtype=torch.complex128, device=dev)}
        lowrank = isinstance(op, LowRankFactors)
        if lowrank and factor_grads:
            out["dus"] = torch.zeros(tuple(op.us.shape), dtype=torch.complex128, device=dev)
            out["dw"] = torch.zeros(tuple(op.w.shape), dtype=torch.complex128, device=dev)
        gr = abi.Grads(_ptr(out["dfield"]), _ptr(out["dE"]), _ptr(out["drho0"]), _ptr(out.get("dus")),
                       _ptr(out.get("dw")))
        n = self.kernel_dim(model, block)
        opr = self._operator(op, block, n)
        ms = model.struct()
        self._check(self._lib.tdg_propagate_adjoint(self.h, C.byref(opr), C.byref(ms), fa, batch, float(dt),
                                                    _ptr(rho0), int(checkpoint_every), C.byref(og), C.byref(gr)))
        return out

    def observables(self, model: DeviceModel, rho: torch.Tensor, fields) -> torch.Tensor:
        fa = field_array(fields)
        out = torch.zeros((len(fa), 5), dtype=torch.float64, device=rho.device)
        ms = model.struct()
        self._check(self._lib.tdg_observables(self.h, C.byref(ms), _ptr(rho), len(fa), fa, _ptr(out)))
        return out

    def check_numeric(self, result: dict, fields, tr_tol: float = 1e-10, herm_tol: float = 1e-10) -> None:
        fa = field_array(fields)
        self._check(self._lib.tdg_check_numeric(self.h, C.byref(result["_obs_struct"]), len(fa), fa,
                                                tr_tol, herm_tol))

    # --- launch-shape selection ---------------------------------------------
    def set_option(self, option: int, value: int) -> None:
        self._check(self._lib.tdg_set_option(self.h, option, int(value)))

    def last_variant(self) -> str:
        return self._lib.tdg_last_variant(self.h).decode()

    # --- measurement ------------------------------------------------------
    def profile_enable(self, on: bool = True) -> None:
        self._check(self._lib.tdg_profile_enable(self.h, int(on)))

    def profile_read(self, kclass: int = abi.TDG_KCLASS_STAGE):
        ms = C.c_double()
        cnt = C.c_int64()
        self._check(self._lib.tdg_profile_read(self.h, kclass, C.byref(ms), C.byref(cnt)))
        return ms.value, cnt.value


# --- differentiable propagation ---------------------------------------------

def _field_records(params: torch.Tensor, nsteps: int, ex: float, ey: float) -> np.ndarray:
    p = params.detach().to("cpu", torch.float64).numpy()
    rec = np.zeros((p.shape[0], 8))
    rec[:, :4] = p
    rec[:, 4], rec[:, 5], rec[:, 6] = ex, ey, nsteps
    return rec


class _Propagate(torch.autograd.Function):
    """P, J, occ series as functions of the pulse parameters and the low-rank
    factors; backward runs the library's adjoint RK4."""

    @staticmethod
    def forward(fctx, params, us, w, cfg):
        ctx, model, block, kdiag, K, dt, nsteps, ex, ey, every = cfg
        rec = _field_records(params, nsteps, ex, ey)
        op = K if K is not None else LowRankFactors(kdiag, us, w, None, us.shape[1], 0.0, 0.0, "c128")
        res = ctx.propagate(op, model, block, rec, dt, diagnostics=False)
        fctx.cfg = cfg
        fctx.save_for_backward(params, us, w)
        return res["P"], res["J"], res["occ"]

    @staticmethod
    def backward(fctx, gP, gJ, gocc):
        params, us, w = fctx.saved_tensors
        ctx, model, block, kdiag, K, dt, nsteps, ex, ey, every = fctx.cfg
        rec = _field_records(params, nsteps, ex, ey)
        lowrank = K is None
        op = K if not lowrank else LowRankFactors(kdiag, us, w, None, us.shape[1], 0.0, 0.0, "c128")
        want = lowrank and (fctx.needs_input_grad[1] or fctx.needs_input_grad[2])
        g = ctx.propagate_adjoint(op, model, block, rec, dt, gP=gP, gJ=gJ, gocc=gocc, checkpoint_every=every,
                                  factor_grads=want)
        dparams = g["dfield"].to(params.device, params.dtype)
        dus = g["dus"] if want and fctx.needs_input_grad[1] else None
        dw = g["dw"] if want and fctx.needs_input_grad[2] else None
        return dparams, dus, dw, None


def propagate_differentiable(ctx: Context, model: DeviceModel, block: str, params: torch.Tensor, dt: float,
                             nsteps: int, *, factors: LowRankFactors | None = None,
                             us: torch.Tensor | None = None, w: torch.Tensor | None = None,
                             K: torch.Tensor | None = None, ex: float = 1.0, ey: float = 0.0,
                             checkpoint_every: int = 50):
    """Differentiable P, J, occ [B][nsteps + 1] (FP64 on the device).

    params: [B][4] float64 (e0, omega, tau, t0) per instance.  The operator is
    either complex128 low-rank factors (K_diag from `factors`; S and V^H from
    `us`, `w` if given, so gradients can flow into them) or a dense complex128
    K (gradients for the pulse parameters only).  Backward runs the adjoint
    RK4 with a checkpoint every `checkpoint_every` steps."""
    if K is None:
        if factors is None or factors.dtype != "c128":
            raise ValueError("complex128 low-rank factors or a dense complex128 K are required")
        us = factors.us if us is None else us
        w = factors.w if w is None else w
        kdiag = factors.kdiag
    else:
        us = w = torch.zeros(1, dtype=torch.complex128, device=K.device)
        kdiag = None
    cfg = (ctx, model, block, kdiag, K, float(dt), int(nsteps), float(ex), float(ey), int(checkpoint_every))
    return _Propagate.apply(params, us, w, cfg)
