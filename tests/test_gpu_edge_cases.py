"""Edge cases on the device against the FP64 oracle (GPU only): the largest
band count (8 bands: 16 e-h pairs or 64 pairs per k), rank 1, runs of zero
steps, rejected arguments, and sampled properties of the 120x120 workload."""

import numpy as np
import pytest
import torch

import oracle as O
from workloads import FS_AU, HARTREE_EV, FieldTable, get_config, multiband_model
from workloads.configs import R0_STABLE

pytestmark = pytest.mark.gpu

DT = 0.1 * FS_AU


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


@pytest.fixture(scope="module")
def mb8():
    return multiband_model(4, nb=8, nv=4, seed=3)


def _pulse(nsteps, e0=2e-2, omega_ev=4.5, batch=1):
    t = nsteps * DT
    return FieldTable.stack([FieldTable.single(e0 * (1 + 0.3 * i), omega_ev / HARTREE_EV, t / 6.0, t / 2.0, nsteps)
                             for i in range(batch)])


def _err(x, ref):
    return float(np.abs(np.asarray(x) - ref).max() / np.abs(ref).max())


@pytest.mark.parametrize("block,kind,dtype,tol", [
    ("eh", "dense", "c128", 1e-10), ("eh", "lowrank", "c64", 1e-4),
    ("all", "dense", "c128", 1e-10), ("all", "lowrank", "c64", 1e-4)])
def test_eight_bands_per_instance(P, ctx, mb8, block, kind, dtype, tol):
    dm = P.DeviceModel.from_model(mb8)
    kg = ctx.kernel_build(dm, R0_STABLE, block, dtype)
    ko = O.build_kernel(mb8, R0_STABLE, block)
    assert kg.shape[0] == mb8.nk * (16 if block == "eh" else 64)
    if kind == "dense":
        op, oop = kg, O.DenseOp(ko)
    else:
        op = ctx.kernel_compress(kg, "fraction", 0.25)
        oop = O.LowRankOp.from_factors(O.compress(kg.cpu().numpy().astype(np.complex128), "fraction", 0.25))
    f = _pulse(120)
    _log(f"8 bands {block} {kind} {dtype}: N={kg.shape[0]}, 120 steps")
    res = ctx.propagate(op, dm, block, f, DT)
    ref = O.propagate(mb8, oop, block, f, DT)
    for key in ("P", "J", "occ"):
        e = _err(res[key][0].cpu().numpy(), ref[key])
        _log(f"  err_{key} = {e:.2e}")
        assert e <= tol, key
    assert abs(ref["P"]).max() > 0 and abs(ref["occ"][-1]) > 1e-12     # the pulse does excite


@pytest.mark.parametrize("dtype", ["c64", "bf16x2"])
def test_eight_bands_batched(P, ctx, mb8, dtype):
    """Batched matrix-core path with 8 bands (16 instances per stage block),
    uneven lengths including zero."""
    from paper_2502_05635_amd import _abi as abi
    dm = P.DeviceModel.from_model(mb8)
    kg = ctx.kernel_build(dm, R0_STABLE, "eh", "c64")
    op = ctx.kernel_compress(kg, "rank", 40, out_dtype=dtype)
    oop = O.LowRankOp.from_factors(O.compress(kg.cpu().numpy().astype(np.complex128), "rank", 40))
    lens = [0, 37, 90, 64, 90, 5, 71]
    f = FieldTable.stack([_pulse(n if n else 1, e0=1e-2 * (1 + 0.1 * i)).subset([0]) for i, n in enumerate(lens)])
    f = FieldTable(f.e0, f.omega, f.tau, f.t0, f.ex, f.ey, np.array(lens, dtype=np.int64))
    ctx.set_option(abi.TDG_OPT_BATCHED_MIN, 2)
    try:
        res = ctx.propagate(op, dm, "eh", f, DT)
    finally:
        ctx.set_option(abi.TDG_OPT_BATCHED_MIN, 4)
    assert ctx.last_variant().startswith("batched_mfma")
    worst = 0.0
    for b, nsb in enumerate(lens):
        ref = O.propagate(mb8, oop, "eh", f, DT, instance=b)
        for key in ("P", "J"):
            got = res[key][b, : nsb + 1].cpu().numpy()
            worst = max(worst, float(np.abs(got - ref[key]).max() / max(np.abs(ref[key]).max(), 1e-300)))
    _log(f"  8 bands batched {dtype}: worst err {worst:.2e}")
    assert worst <= 1e-4


def test_eight_bands_channelwise_and_adjoint(P, ctx, mb8):
    """Channel-wise operator with 16 pairs per k (256 channels) and the adjoint
    with 8 bands (one k point per block), FP64 against the oracle."""
    dm = P.DeviceModel.from_model(mb8)
    kg = ctx.kernel_build(dm, R0_STABLE, "eh", "c128")
    k = O.build_kernel(mb8, R0_STABLE, "eh")
    nk, npair = mb8.nk, 16
    fac = ctx.kernel_compress_channels(kg, nk, npair, "rank", 4, rmax=8)
    f = _pulse(60)
    res = ctx.propagate(fac, dm, "eh", f, DT)
    ref = O.propagate(mb8, O.ChannelOp(O.compress_channelwise(k, nk, npair, "rank", 4), nk, npair), "eh", f, DT)
    e = _err(res["P"][0].cpu().numpy(), ref["P"])
    _log(f"  8 bands channel-wise: err_P {e:.2e}")
    assert e <= 1e-10
    rng = np.random.default_rng(3)
    w = rng.standard_normal((1, 61))
    g = ctx.propagate_adjoint(kg, dm, "eh", f, DT, gJ=w, checkpoint_every=16)
    gr = O.propagate_adjoint(mb8, O.DenseOp(k), "eh", f, DT, gJ=w[0])
    e = _err(g["dfield"][0].cpu().numpy(), gr["dfield"])
    _log(f"  8 bands adjoint: dfield err {e:.2e}")
    assert e <= 1e-10


def test_rank_one_and_zero_steps(P, ctx):
    from workloads import tb4_model
    m = tb4_model(4, 6.0, 0.5)
    dm = P.DeviceModel.from_model(m)
    kg = ctx.kernel_build(dm, R0_STABLE, "eh", "c128")
    k = O.build_kernel(m, R0_STABLE, "eh")
    fac = ctx.kernel_compress(kg, "rank", 1)
    assert fac.rank == 1 or fac.rank == int(O.compress(k, "rank", 1)["r"])
    f = _pulse(80)
    res = ctx.propagate(fac, dm, "eh", f, DT)
    ref = O.propagate(m, O.LowRankOp.from_factors(O.compress(k, "rank", 1)), "eh", f, DT)
    assert _err(res["J"][0].cpu().numpy(), ref["J"]) <= 1e-10
    # every instance of zero length: only the observables of rho(0) = rho_eq
    z = FieldTable(f.e0.repeat(3), f.omega.repeat(3), f.tau.repeat(3), f.t0.repeat(3), np.ones(3), np.zeros(3),
                   np.zeros(3, dtype=np.int64))
    res = ctx.propagate(kg, dm, "eh", z, DT)
    o = O.observables(m, O.rho_equilibrium(m), 1.0, 0.0)
    for key in ("P", "J", "occ"):
        np.testing.assert_allclose(res[key][:, 0].cpu().numpy(), o[key], rtol=0, atol=1e-15)
    assert torch.equal(res["rho"], torch.from_numpy(O.rho_equilibrium(m)).cuda().expand(3, -1, -1, -1))


def test_rejected_arguments(P, ctx):
    from workloads import tb4_model
    m = tb4_model(4, 6.0, 0.5)
    dm = P.DeviceModel.from_model(m)
    kg = ctx.kernel_build(dm, R0_STABLE, "eh", "c128")
    with pytest.raises(P.TdgError):                       # an empty batch
        ctx.propagate(kg, dm, "eh", np.zeros((0, 8)), DT)
    bad = P.DeviceModel.from_model(m)
    bad.nb = 9                                            # beyond the supported band count
    with pytest.raises(P.TdgError):
        ctx.propagate(kg, bad, "eh", _pulse(4), DT)


def test_large_grid_sampled_kernel_and_ritz_pairs(P):
    """120x120 workload (N = 57600): sampled kernel elements against the
    element-by-element definition, and the Rayleigh-Ritz properties of the
    randomized factors, which hold whatever the range finder captured: the
    Ritz vectors (rows of V^H) are orthonormal, each Rayleigh quotient
    v^H K_off v equals its Ritz value, and each residual K_off v - l v is
    orthogonal to every kept Ritz vector (Galerkin condition)."""
    cfg = get_config(4)
    m = cfg.model()
    c = P.Context(0)
    try:
        dm = P.DeviceModel.from_model(m)
        kg = c.kernel_build(dm, cfg.r0, "eh", "c64")
        n = kg.shape[0]
        rng = np.random.default_rng(8)
        idx = rng.integers(0, n, size=(200, 2))
        idx = np.vstack([idx, [[0, 0], [n - 1, n - 1], [0, n - 1], [n - 1, 0]]])
        vals = kg[torch.from_numpy(idx[:, 0]).cuda(), torch.from_numpy(idx[:, 1]).cuda()].cpu().numpy()
        ref = np.array([O.kernel_element(m, cfg.r0, "eh", i, j) for i, j in idx])
        scale = abs(O.kernel_element(m, cfg.r0, "eh", 0, 0))
        e = float(np.abs(vals - ref).max() / scale)
        _log(f"  120x120 sampled kernel elements: {e:.2e}")
        assert e <= 1e-7
        r, l = 64, 192
        g = torch.Generator(device="cuda")
        g.manual_seed(77)
        om = (torch.randn(l, n, dtype=torch.float64, device="cuda", generator=g)
              + 1j * torch.randn(l, n, dtype=torch.float64, device="cuda", generator=g)).contiguous()
        fac = c.kernel_compress_randomized(kg, om, "rank", r, power_iters=3, out_dtype="c128")
        del om
        w = fac.w                                         # [r][n]: row j = u_j^H
        gram = (w.conj() @ w.T)
        e_orth = float((gram - torch.eye(r, dtype=gram.dtype, device=gram.device)).abs().max())
        kd = kg.diagonal().to(torch.complex128)
        smax = float(fac.sigma[0])
        worst_rq = worst_gal = worst_res = 0.0
        for j in range(8):
            v = w[j].conj()
            kv = (kg @ v.to(torch.complex64)).to(torch.complex128) - kd * v
            lam_j = complex((v.conj() @ fac.us[:, j]).item())        # S column j = l_j u_j
            rq = complex((v.conj() @ kv).item())
            res = kv - lam_j * v
            worst_rq = max(worst_rq, abs(rq - lam_j) / smax)
            worst_gal = max(worst_gal, float((w @ res).abs().max()) / smax)
            worst_res = max(worst_res, float(res.norm()) / smax)
        _log(f"  Ritz vectors orthonormal to {e_orth:.1e}; Rayleigh quotients {worst_rq:.1e}, "
             f"Galerkin {worst_gal:.1e}, residuals <= {worst_res:.3f} of s_max")
        assert e_orth <= 1e-10
        assert worst_rq <= 1e-5 and worst_gal <= 1e-5      # FP32 products with K
        assert worst_res <= 0.1
    finally:
        c.close()
