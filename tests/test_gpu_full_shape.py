"""Oracle parity at the full shapes of the batched workloads (GPU only).

60x60 grid (N = 14400): the low-rank batched matrix-core path at 5 % of the
singular values (r = 720), 64 instances in one batch with the tuner choosing
tilings and split-K; eight instances, spread over the amplitudes and lengths,
against the FP64 oracle run with the same (complex64) factors.

120x120 grid (N = 57600): the BF16X2 path with randomized factors at 5 % of N
(r = 2880); two instances against the FP64 oracle run with the FP64 factors
the hi + lo planes were rounded from, and the 4000-step runs against the
device's FP64 low-rank path (P, J and the absorption spectrum).

The short runs move the pulse to their first steps (t0 = 8 dt, tau = 3 dt) so
that the state moves within ~20 steps.  Bound: max_n |X - X_ref| / max_n |X_ref|
<= 1e-4 for P and J (the reduced-precision bar)."""

import numpy as np
import pytest
import torch

import oracle as O
from workloads import HARTREE_EV, FieldTable, get_config

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _log(msg):
    print(msg, flush=True)


def _err(x, ref):
    return float(np.abs(np.asarray(x) - ref).max() / np.abs(ref).max())


@pytest.fixture(scope="module")
def P():
    import paper_2502_05635_amd as P
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return P


def _early(fields: FieldTable, nsteps: np.ndarray, dt: float) -> FieldTable:
    b = fields.batch
    return FieldTable(fields.e0.copy(), fields.omega.copy(), np.full(b, 3.0 * dt), np.full(b, 8.0 * dt),
                      fields.ex.copy(), fields.ey.copy(), np.asarray(nsteps, dtype=np.int64))


def _host_factors(fac) -> dict:
    c = lambda t: t.cpu().numpy().astype(np.complex128)  # noqa: E731
    return {"kdiag": c(fac.kdiag), "US": c(fac.us), "Vh": c(fac.w)}


def test_sweep_lowrank_batched_full_shape_vs_oracle(P):
    """The 60x60 sweep shape (N = 14400, rank 720, 64 instances of 14-24
    steps, retiring unevenly) on the batched path, FP32 and then BF16X2 from
    the same K, each against the FP64 oracle with the FP32 factors on eight
    instances.  BF16X2 runs the tuner's tilings with the split gather written
    by the stage kernel; its factors differ from the FP32 ones only by their
    rounding."""
    cfg = get_config(2)
    m = cfg.model()
    n = cfg.n
    B = cfg.fields.batch
    lengths = 14 + (np.arange(B) * 7) % 11            # 14 .. 24 steps, uneven
    fields = _early(cfg.fields, lengths, cfg.dt)
    ctx = P.Context(0)
    try:
        dm = P.DeviceModel.from_model(m)
        _log(f"{cfg.name}: N={n}, building K and compressing to 5 % (exact eigensolver)")
        K = ctx.kernel_build(dm, cfg.r0, "eh", "c64")
        fac = ctx.kernel_compress(K, "fraction", 0.05)
        assert fac.rank == 720
        _log(f"  batched low rank FP32, B={B}, {lengths.min()}-{lengths.max()} steps, tuner on")
        res = ctx.propagate(fac, dm, "eh", fields, cfg.dt)
        torch.cuda.synchronize()
        variant = ctx.last_variant()
        _log(f"  {variant}")
        assert variant.startswith("batched_mfma_lowrank_f32")
        op = O.LowRankOp.from_factors(_host_factors(fac))
        checked = [0, 9, 18, 27, 36, 45, 54, 63]
        refs = {}
        for b in checked:
            refs[b] = ref = O.propagate(m, op, "eh", fields, cfg.dt, instance=b)
            nsb = int(lengths[b])
            errs = {key: _err(res[key][b, : nsb + 1].cpu().numpy(), ref[key]) for key in ("P", "J", "occ")}
            _log(f"  instance {b} (E0 {fields.e0[b]:.1e}, {nsb} steps): "
                 + ", ".join(f"err_{k} {v:.2e}" for k, v in errs.items()))
            assert abs(ref["occ"][-1]) > 1e-14                      # the pulse does excite
            assert errs["P"] <= TOL and errs["J"] <= TOL, b
        assert torch.isfinite(res["P"]).all()
        del res, fac
        fbf = ctx.kernel_compress(K, "fraction", 0.05, out_dtype="bf16x2")
        assert fbf.rank == 720
        del K
        torch.cuda.empty_cache()
        _log("  batched low rank BF16X2, same instances, tuner on")
        res = ctx.propagate(fbf, dm, "eh", fields, cfg.dt)
        torch.cuda.synchronize()
        variant = ctx.last_variant()
        _log(f"  {variant}")
        assert variant.startswith("batched_mfma_lowrank_bf16x2")
        for b in checked:
            nsb = int(lengths[b])
            errs = {key: _err(res[key][b, : nsb + 1].cpu().numpy(), refs[b][key]) for key in ("P", "J", "occ")}
            _log(f"  instance {b}: " + ", ".join(f"err_{k} {v:.2e}" for k, v in errs.items()))
            assert errs["P"] <= TOL and errs["J"] <= TOL, b
        assert torch.isfinite(res["P"]).all()
    finally:
        ctx.close()


@pytest.fixture(scope="module")
def large_grid(P):
    """120x120: K (26.5 GB complex64), the randomized factors once in
    complex128 and once as BF16 hi + lo planes (same test matrix, so the same
    FP64 factors before rounding)."""
    cfg = get_config(4)
    m = cfg.model()
    n = cfg.n
    r = int(round(0.05 * n))
    l, q = r + 128, 2
    c = P.Context(0)
    dm = P.DeviceModel.from_model(m)
    _log(f"large grid {cfg.name} N={n}: randomized compression rank={r} l={l} power_iters={q}")
    kg = c.kernel_build(dm, cfg.r0, "eh", "c64")
    g = torch.Generator(device="cuda")
    g.manual_seed(2026)
    om = (torch.randn(l, n, dtype=torch.float64, device="cuda", generator=g)
          + 1j * torch.randn(l, n, dtype=torch.float64, device="cuda", generator=g)).contiguous()
    f64 = c.kernel_compress_randomized(kg, om, "rank", r, power_iters=q, out_dtype="c128")
    fbf = c.kernel_compress_randomized(kg, om, "rank", r, power_iters=q, out_dtype="bf16x2")
    assert f64.rank == fbf.rank == r
    del kg, om
    torch.cuda.empty_cache()
    yield cfg, m, dm, c, f64, fbf
    c.close()


def test_large_grid_bf16x2_vs_oracle(P, large_grid):
    """Two instances (weakest and strongest amplitude), ~20 steps with the
    pulse moved early: the BF16X2 batched path against the FP64 oracle with
    the FP64 factors."""
    cfg, m, dm, c, f64, fbf = large_grid
    idx = [0, cfg.fields.batch - 1]
    fields = _early(cfg.fields.subset(idx), [20, 17], cfg.dt)
    _log("  BF16X2 batched, 2 instances, 20 / 17 steps")
    got = c.propagate(fbf, dm, "eh", fields, cfg.dt)
    torch.cuda.synchronize()
    assert "bf16x2" in c.last_variant()
    _log("  FP64 oracle with the FP64 factors (host)")
    op = O.LowRankOp.from_factors(_host_factors(f64))
    for b in range(2):
        ref = O.propagate(m, op, "eh", fields, cfg.dt, instance=b)
        nsb = int(fields.nsteps[b])
        errs = {key: _err(got[key][b, : nsb + 1].cpu().numpy(), ref[key]) for key in ("P", "J", "occ")}
        _log(f"  instance {idx[b]} (E0 {fields.e0[b]:.1e}): " + ", ".join(f"err_{k} {v:.2e}" for k, v in errs.items()))
        assert abs(ref["occ"][-1]) > 1e-14
        assert errs["P"] <= TOL and errs["J"] <= TOL, b


def test_large_grid_bf16x2_vs_fp64_lowrank(P, large_grid):
    """The BF16X2 batched path against the device's FP64 low-rank path over
    the full 4000 steps of two instances, on P(t) over the first half and on
    the absorption spectrum A(w) where the pulse has spectral weight."""
    cfg, m, dm, c, f64, fbf = large_grid
    idx = [0, cfg.fields.batch - 1]              # weakest and strongest amplitude
    fields = cfg.fields.subset(idx)
    _log("  FP64 low-rank reference, 2 instances x 4000 steps")
    ref = c.propagate(f64, dm, "eh", fields, cfg.dt, diagnostics=False)
    _log("  BF16X2 batched, same instances")
    got = c.propagate(fbf, dm, "eh", fields, cfg.dt, diagnostics=False)
    assert "bf16x2" in c.last_variant()
    half = 2001
    worst = {}
    for b in range(2):
        for key in ("P", "J"):
            x = got[key][b].cpu().numpy()
            y = ref[key][b].cpu().numpy()
            e_half = float(np.abs(x[:half] - y[:half]).max() / np.abs(y[:half]).max())
            _log(f"  instance {idx[b]} E0={fields.e0[b]:.1e}: err_{key} first half {e_half:.2e}, "
                 f"full run {_err(x, y):.2e}")
            worst[(b, key)] = e_half
    # absorption of the weak pulse
    p_ref = ref["P"][0].cpu().numpy()
    p_got = got["P"][0].cpu().numpy()
    t = np.arange(p_ref.shape[0]) * cfg.dt
    e = np.array([O.field_at(tt, fields, 0) for tt in t])
    w0 = fields.omega[0]
    om_grid = np.linspace(w0 - 0.15 / HARTREE_EV, w0 + 0.15 / HARTREE_EV, 301)
    eta = 0.05 / HARTREE_EV
    a_ref = O.absorption(p_ref, e, cfg.dt, om_grid, eta)
    a_got = O.absorption(p_got, e, cfg.dt, om_grid, eta)
    e_abs = float(np.abs(a_got - a_ref).max() / np.abs(a_ref).max())
    _log(f"  absorption within +-0.15 eV of the carrier: rel err {e_abs:.2e}")
    assert max(worst.values()) <= TOL
    assert e_abs <= TOL
