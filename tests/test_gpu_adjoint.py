"""Adjoint RK4 on the device against the FP64 oracle's reverse-mode
derivative (same inputs) and against central finite differences of the
device's own forward propagation (GPU only)."""

import contextlib

import numpy as np
import pytest
import torch

import oracle as O
from workloads import FS_AU, HARTREE_EV, FieldTable, dirac_model, get_config, tb4_model
from workloads.configs import R0_STABLE
from workloads.random_matrices import gaussian_test_matrix, hermitian_lowrank_factors

pytestmark = pytest.mark.gpu

A = 6.0
DT = 0.2 * FS_AU
NSTEPS = 40


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def P():
    import paper_2502_05635_amd as P
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return P


@pytest.fixture(scope="module")
def ctx(P):
    c = P.Context(0)
    yield c
    c.close()


def _fields(batch=2):
    e0 = np.array([8e-3, 2e-2])[:batch]
    om = np.array([1.2, 0.8])[:batch] / HARTREE_EV
    tau = np.array([2.0, 3.0])[:batch] * FS_AU
    t0 = np.array([4.0, 3.5])[:batch] * FS_AU
    return FieldTable(e0, om, tau, t0, np.ones(batch), np.zeros(batch), np.full(batch, NSTEPS, dtype=np.int64))


def _weights(batch, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((batch, NSTEPS + 1)) for _ in range(3)]


@contextlib.contextmanager
def _stash(ctx, mode):
    """TDG_OPT_ADJOINT_STASH set to mode for the block, then the default (2)."""
    from paper_2502_05635_amd import _abi as abi
    ctx.set_option(abi.TDG_OPT_ADJOINT_STASH, mode)
    try:
        yield
    finally:
        ctx.set_option(abi.TDG_OPT_ADJOINT_STASH, 2)


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("every,stash", [(1, 1), (7, 1), (64, 1), (7, 2)])
def test_adjoint_lowrank_matches_oracle(P, ctx, every, stash):
    """Seeded Hermitian factors (rank 12) on the 4x4 four-band model, two
    instances, loss weights on P, J and occupation; segments of checkpoint
    spacing 1, 7 (ragged last segment) and beyond the run length, and the
    whole run as one segment (stash mode 2, the default)."""
    m = tb4_model(4, A, 0.5)
    dm = P.DeviceModel.from_model(m)
    n = ctx.kernel_dim(dm, "eh")
    kd, us, vh = hermitian_lowrank_factors(n, 12, 0.03, -0.01, 31)
    f = _fields()
    w = _weights(2, 32)
    _log(f"adjoint low-rank tb4 4x4 N={n} rank 12, checkpoint every {every}, stash mode {stash}")
    fac = P.LowRankFactors(torch.from_numpy(kd).cuda(), torch.from_numpy(us).cuda(), torch.from_numpy(vh).cuda(),
                           None, 12, 0.0, 0.0, "c128")
    with _stash(ctx, stash):
        g = ctx.propagate_adjoint(fac, dm, "eh", f, DT, gP=w[0], gJ=w[1], gocc=w[2], checkpoint_every=every)
    op = O.LowRankOp(kd, us, vh)
    for b in range(2):
        ref = O.propagate_adjoint(m, op, "eh", f, DT, w[0][b], w[1][b], w[2][b], instance=b)
        errs = {"dfield": _rel(g["dfield"][b].cpu().numpy(), ref["dfield"]),
                "dE": _rel(g["dE"][b].cpu().numpy(), ref["dE"]),
                "drho0": _rel(g["drho0"][b].cpu().numpy(), ref["drho0"])}
        _log(f"  instance {b}: " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()))
        assert max(errs.values()) <= 1e-10
    # factor gradients sum over instances
    refs = [O.propagate_adjoint(m, op, "eh", f, DT, w[0][b], w[1][b], w[2][b], instance=b) for b in range(2)]
    e_us = _rel(g["dus"].cpu().numpy(), sum(r["dus"] for r in refs))
    e_w = _rel(g["dw"].cpu().numpy(), sum(r["dvh"] for r in refs))
    _log(f"  dS {e_us:.1e}, dV^H {e_w:.1e}")
    assert e_us <= 1e-10 and e_w <= 1e-10


@pytest.mark.parametrize("block", ["eh", "all"])
def test_adjoint_dense_matches_oracle(P, ctx, block):
    """Dense complex128 kernels built on each side from the same model."""
    m = tb4_model(4, A, 0.5) if block == "eh" else dirac_model(4, 1.0, 1.5, A, 0.5)
    dm = P.DeviceModel.from_model(m)
    kg = ctx.kernel_build(dm, R0_STABLE, block, "c128")
    f = _fields(1)
    w = _weights(1, 33)
    _log(f"adjoint dense {block} N={kg.shape[0]}")
    g = ctx.propagate_adjoint(kg, dm, block, f, DT, gP=w[0], gJ=w[1], gocc=w[2], checkpoint_every=9)
    ref = O.propagate_adjoint(m, O.DenseOp(O.build_kernel(m, R0_STABLE, block)), block, f, DT,
                              w[0][0], w[1][0], w[2][0])
    errs = {"dfield": _rel(g["dfield"][0].cpu().numpy(), ref["dfield"]),
            "dE": _rel(g["dE"][0].cpu().numpy(), ref["dE"]),
            "drho0": _rel(g["drho0"][0].cpu().numpy(), ref["drho0"])}
    _log("  " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()))
    assert max(errs.values()) <= 1e-10


@pytest.mark.parametrize("kind", ["dense", "lowrank"])
def test_adjoint_stash_matches_recompute(P, ctx, kind):
    """Keeping each segment's stage data (TDG_OPT_ADJOINT_STASH 1) and
    rerunning every backward step's forward step (0) are the same arithmetic:
    every gradient agrees bitwise, with a ragged last segment.  The whole run
    as one segment (2, the default) differs only in the order in which the
    factor gradients add up the segments' columns."""
    from paper_2502_05635_amd import _abi as abi
    m = tb4_model(4, A, 0.5)
    dm = P.DeviceModel.from_model(m)
    if kind == "dense":
        op = ctx.kernel_build(dm, R0_STABLE, "eh", "c128")
    else:
        n = ctx.kernel_dim(dm, "eh")
        kd, us, vh = hermitian_lowrank_factors(n, 12, 0.03, -0.01, 31)
        op = P.LowRankFactors(torch.from_numpy(kd).cuda(), torch.from_numpy(us).cuda(), torch.from_numpy(vh).cuda(),
                              None, 12, 0.0, 0.0, "c128")
    f = _fields()
    w = _weights(2, 34)
    out = []
    for stash in (1, 0, 2):
        with _stash(ctx, stash):
            out.append(ctx.propagate_adjoint(op, dm, "eh", f, DT, gP=w[0], gJ=w[1], gocc=w[2], checkpoint_every=7))
    for key, v in out[0].items():
        if v is None:
            continue
        assert torch.equal(v, out[1][key]), key
        if key in ("dus", "dw"):
            assert _rel(out[2][key].cpu().numpy(), v.cpu().numpy()) <= 1e-13, key
        else:
            assert torch.equal(out[2][key], v), key
    for bad in (-1, 3):
        with pytest.raises(P.TdgError):
            ctx.set_option(abi.TDG_OPT_ADJOINT_STASH, bad)


def test_adjoint_whole_run_falls_back_to_segments_when_memory_is_short(P):
    """The default stash mode keeps the whole run's stage data (3.1 GB for the
    24x24, 3000-step workload).  With the device filled to within 1.5 GiB that
    workspace cannot be allocated: the call runs checkpoint segments instead
    and returns exactly the gradients of stash mode 1 (factor gradients
    included, whose summation order differs for one segment).  With the
    memory back it runs as one segment again."""
    from paper_2502_05635_amd import _abi as abi
    cfg = get_config(3)
    dm = P.DeviceModel.from_model(cfg.model())
    fl = cfg.fields
    nsteps = int(fl.nsteps[0])
    gj = np.random.default_rng(5).standard_normal((1, nsteps + 1))
    c = P.Context(0)
    hog = []
    try:
        fac = c.kernel_compress(c.kernel_build(dm, cfg.r0, "eh", "c128"), "fraction", 0.05)
        with _stash(c, 1):
            ref = c.propagate_adjoint(fac, dm, "eh", fl, cfg.dt, gJ=gj, checkpoint_every=50)
        _log(f"  stash mode 1: {c.last_variant()}")
        c.close()
        c = P.Context(0)                               # no workspace held yet
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        # hold all but 1.5 GiB of the device, in pieces of at most 16 GiB
        # (halved whenever one cannot be allocated)
        chunk = 16 << 30
        while chunk >= (64 << 20):
            free, _ = torch.cuda.mem_get_info()
            extra = free - (3 << 29)
            if extra <= (64 << 20):
                break
            try:
                hog.append(torch.empty(min(extra, chunk), dtype=torch.uint8, device="cuda"))
            except torch.cuda.OutOfMemoryError:
                chunk //= 2
        _log(f"  {sum(h.numel() for h in hog) / 2**30:.1f} GiB held, "
             f"{torch.cuda.mem_get_info()[0] / 2**30:.2f} GiB left free")
        g = c.propagate_adjoint(fac, dm, "eh", fl, cfg.dt, gJ=gj, checkpoint_every=50)
        plan = c.last_variant()
        hog.clear()
        torch.cuda.empty_cache()
        _log(f"  short of memory: {plan}")
        assert "60 segments of 50 steps" in plan and "stashed" in plan
        for key, v in ref.items():
            assert torch.equal(g[key], v), key
        c.propagate_adjoint(fac, dm, "eh", fl, cfg.dt, gJ=gj, checkpoint_every=50)
        _log(f"  memory back: {c.last_variant()}")
        assert "one segment" in c.last_variant()
    finally:
        hog.clear()
        torch.cuda.empty_cache()
        c.close()


def test_adjoint_rejects_unsupported(P, ctx):
    m = tb4_model(4, A, 0.5)
    dm = P.DeviceModel.from_model(m)
    kg = ctx.kernel_build(dm, R0_STABLE, "eh", "c64")
    f = _fields()
    with pytest.raises(P.TdgError):                       # FP32 operator
        ctx.propagate_adjoint(kg, dm, "eh", f, DT, gJ=np.ones((2, NSTEPS + 1)))
    uneven = FieldTable(f.e0, f.omega, f.tau, f.t0, f.ex, f.ey, np.array([NSTEPS, NSTEPS - 1]))
    with pytest.raises(P.TdgError):                       # unequal lengths
        ctx.propagate_adjoint(ctx.kernel_build(dm, R0_STABLE, "eh", "c128"), dm, "eh", uneven, DT)


def test_autograd_harmonic_loss_vs_finite_differences(P, ctx):
    """Differentiation workload: 24x24 four-band e-h kernel (N = 2304),
    complex128 factors of the exact truncated SVD at 5 % of N, one 3000-step
    pulse (E0 = 5e-3, omega = 0.8 eV); loss = third-harmonic intensity of J.
    torch.autograd through the adjoint against central differences
    (h = 1e-6 relative) of the device forward, and against the FP64 oracle's
    adjoint for the pulse parameters (factors gauge-independent there)."""
    cfg = get_config(3)
    m = cfg.model()
    dm = P.DeviceModel.from_model(m)
    kg = ctx.kernel_build(dm, cfg.r0, "eh", "c128")
    fac = ctx.kernel_compress(kg, "fraction", 0.05)
    fl = cfg.fields
    nsteps = int(fl.nsteps[0])
    _log(f"autograd {cfg.name} N={cfg.n} rank {fac.rank}, {nsteps} steps, checkpoint every 50")
    base = torch.tensor([[fl.e0[0], fl.omega[0], fl.tau[0], fl.t0[0]]], dtype=torch.float64)
    t = torch.arange(nsteps + 1, dtype=torch.float64, device="cuda") * cfg.dt

    def loss_of(params, us=None, w=None):
        _, j, _ = P.propagate_differentiable(ctx, dm, "eh", params, cfg.dt, nsteps, factors=fac, us=us, w=w)
        om = params[0, 1].to("cuda")
        ph = torch.exp(-1j * 3.0 * om * t)
        a = 3.0 * om * cfg.dt * torch.sum(j[0].to(torch.complex128) * ph)
        return (a.abs() ** 2)

    params = base.clone().requires_grad_(True)
    us = fac.us.clone().requires_grad_(True)
    w = fac.w.clone().requires_grad_(True)
    L = loss_of(params, us, w)
    L.backward()
    grad = params.grad[0].numpy()
    for i, name in enumerate(("e0", "omega", "tau", "t0")):
        h = 1e-6 * abs(float(base[0, i]))
        pp, pm = base.clone(), base.clone()
        pp[0, i] += h
        pm[0, i] -= h
        with torch.no_grad():
            fd = (loss_of(pp).item() - loss_of(pm).item()) / (2 * h)
        _log(f"  dL/d{name}: adjoint {grad[i]:.10e}, central difference {fd:.10e}")
        assert abs(grad[i] - fd) <= 1e-5 * max(abs(fd), 1e-6 * np.abs(grad).max())
    # factor directions
    rng = np.random.default_rng(41)
    for name, tens, g_ in (("S", fac.us, us.grad), ("V^H", fac.w, w.grad)):
        d = torch.from_numpy(rng.standard_normal(tuple(tens.shape)) + 1j * rng.standard_normal(tuple(tens.shape))).cuda()
        eps = 1e-6 * tens.abs().max().item()
        with torch.no_grad():
            lp = loss_of(base, *((tens + eps * d, None) if name == "S" else (None, tens + eps * d))).item()
            lm = loss_of(base, *((tens - eps * d, None) if name == "S" else (None, tens - eps * d))).item()
        fd = (lp - lm) / (2 * eps)
        ad = float(torch.sum((g_.conj() * d).real).item())
        _log(f"  d/d{name} along a seeded direction: adjoint {ad:.10e}, central difference {fd:.10e}")
        assert abs(ad - fd) <= 1e-5 * abs(fd)
    # the oracle's adjoint with its own factors of the same rank
    kf = O.compress(O.build_kernel(m, cfg.r0, "eh"), "fraction", 0.05, method="eigh")
    r = O.propagate(m, O.LowRankOp.from_factors(kf), "eh", fl, cfg.dt)
    _, gj, gw = O.harmonic_loss(r["J"], float(fl.omega[0]), cfg.dt)
    ref = O.propagate_adjoint(m, O.LowRankOp.from_factors(kf), "eh", fl, cfg.dt, gJ=gj)
    ref_grad = ref["dfield"].copy()
    ref_grad[1] += gw
    e = _rel(grad, ref_grad)
    _log(f"  pulse-parameter gradient vs FP64 oracle adjoint: {e:.2e}")
    assert e <= 1e-8
