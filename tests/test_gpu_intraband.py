"""Intraband field coupling on the device (tdg_links_build and a model with
links) against the FP64 oracle on the same seeded inputs (GPU only).

The links are computed independently on each side (Newton polar iteration on
the device, SVD in the oracle) and compared element by element; propagation
with the intraband term is compared on P, J, occupation, the grid-averaged
trace diagnostic and the final state, with the tolerances of the other
parity tests: 1e-10 (FP64 operators), 1e-4 (FP32 operators).
"""

import numpy as np
import pytest
import torch

import oracle as O
from workloads import (FS_AU, HARTREE_EV, FieldTable, dirac_model, flat_band_model, multiband_model,
                       tb4_model)
from workloads.configs import R0_STABLE, get_config

pytestmark = pytest.mark.gpu

A = 6.0
DT = 0.05 * FS_AU


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
def tb4_6():
    return tb4_model(6, A, 0.5)


@pytest.fixture(scope="module")
def k_tb4_6(tb4_6):
    return O.build_kernel(tb4_6, R0_STABLE, "eh")


def _with_links(P, ctx, m):
    dm = P.DeviceModel.from_model(m)
    return dm.with_links(ctx.links_build(dm))


def _drho(m, seed, scale=1e-2):
    """Hermitian perturbation whose per-k traces differ (grid mean zero)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((m.nk, m.nb, m.nb)) + 1j * rng.standard_normal((m.nk, m.nb, m.nb))
    d = 0.5 * scale * (z + z.conj().transpose(0, 2, 1))
    d[:, 0, 0] -= np.mean(np.einsum("knn->k", d))
    return d


def _two_polarisations(nsteps, e0=5e-3, omega_ev=1.5):
    t = nsteps * DT
    return FieldTable.stack([
        FieldTable.single(e0, omega_ev / HARTREE_EV, t / 10.0, t / 2.0, nsteps, ex=0.8, ey=0.6),
        FieldTable.single(0.7 * e0, 1.1 * omega_ev / HARTREE_EV, t / 8.0, t / 2.5, nsteps, ex=0.0, ey=-1.0),
    ])


def _compare(res, refs, tol, rho_tol):
    for b, ref in enumerate(refs):
        ns = len(ref["P"]) - 1
        for key in ("P", "J", "occ"):
            got = res[key][b, : ns + 1].cpu().numpy()
            scale = max(np.abs(ref[key] - ref[key][0]).max(), np.abs(ref[key]).max(), 1e-300)
            e = float(np.abs(got - ref[key]).max() / scale)
            _log(f"  instance {b} err_{key} = {e:.2e}")
            assert e <= tol, (b, key)
        tr = res["tr"][b, : ns + 1].cpu().numpy()
        assert np.abs(tr - ref["tr"]).max() <= max(10 * tol * 1e-3, 1e-13), (b, "tr")
        got = res["rho"][b].cpu().numpy()
        assert np.abs(got - ref["rho"]).max() <= rho_tol, (b, "rho")


@pytest.mark.parametrize("kind", ["tb4", "multiband8", "dirac", "flat_rotated"])
def test_links_match_oracle(P, ctx, kind):
    m = {"tb4": lambda: tb4_model(6, A, 0.5),
         "multiband8": lambda: multiband_model(6, nb=8, nv=4),
         "dirac": lambda: dirac_model(6, 1.0, 1.5, A, 0.5),
         "flat_rotated": lambda: flat_band_model(8, 6, dip_seed=5, gauge_seed=7, a=A)}[kind]()
    _log(f"links {kind} {m.nk1}x{m.nk2}, nb = {m.nb}")
    lg = ctx.links_build(P.DeviceModel.from_model(m)).cpu().numpy()
    lo = O.transport_links(m)
    e = float(np.abs(lg - lo).max())
    _log(f"  max |L_gpu - L_oracle| = {e:.2e}")
    assert e <= 1e-12


def test_links_singular_block_reported(P, ctx):
    """Bloch states whose valence subspace at odd i1 is the conduction
    subspace at even i1: the block overlap vanishes and the build says so."""
    m = flat_band_model(4, 4, a=A)
    swap = np.zeros((4, 4), dtype=np.complex128)
    for n in range(4):
        swap[(n + 2) % 4, n] = 1.0
    i1 = np.arange(m.nk) // m.nk2
    m.evec[i1 % 2 == 1] = swap
    with pytest.raises(P.TdgError) as e:
        ctx.links_build(P.DeviceModel.from_model(m))
    assert "singular" in str(e.value)


def test_drift_fp64_matches_oracle(P, ctx):
    """Flat bands, no interaction: the pure drift of a perturbed state, two
    instances with different polarisations, against the oracle."""
    m = flat_band_model(8, 6, nb=4, nv=2, gap_ev=0.5, a=A)
    dm = _with_links(P, ctx, m)
    n = m.nk * 4
    k0 = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
    fields = FieldTable.stack([FieldTable.single(2e-3, 0.0, 80.0, 240.0, 400, ex=0.8, ey=0.6),
                               FieldTable.single(2e-3, 0.0, 60.0, 150.0, 400, ex=0.0, ey=-1.0)])
    rho0 = O.rho_equilibrium(m) + _drho(m, 5)
    _log("drift, flat 8x6, dense zero kernel c128, 2 instances, 400 steps")
    res = ctx.propagate(k0, dm, "eh", fields, 0.5, rho=torch.from_numpy(np.stack([rho0, rho0])).cuda(),
                        init_eq=False)
    refs = [O.propagate(m, O.DenseOp(np.zeros((n, n), complex)), "eh", fields, 0.5, instance=b, rho0=rho0,
                        links=O.transport_links(m)) for b in range(2)]
    _compare(res, refs, 1e-10, 1e-12)


@pytest.mark.parametrize("kind,dtype,tol", [("dense", "c128", 1e-10), ("lowrank", "c128", 1e-10),
                                            ("dense", "c64", 1e-4), ("lowrank", "c64", 1e-4),
                                            ("channel", "c64", 1e-4)])
def test_tb4_intraband_per_instance_path(P, ctx, tb4_6, k_tb4_6, kind, dtype, tol):
    from paper_2502_05635_amd import _abi as abi
    dm = _with_links(P, ctx, tb4_6)
    kg = ctx.kernel_build(dm, R0_STABLE, "eh", dtype)
    nk, NP = tb4_6.nk, 4
    if kind == "dense":
        op, oop = kg, O.DenseOp(k_tb4_6)
    elif kind == "lowrank":
        op = ctx.kernel_compress(kg, "fraction", 0.3)
        oop = O.LowRankOp.from_factors(O.compress(k_tb4_6, "fraction", 0.3))
    else:
        op = ctx.kernel_compress_channels(kg, nk, NP, "fraction", 0.2, rmax=12)
        oop = O.ChannelOp(O.compress_channelwise(k_tb4_6, nk, NP, "fraction", 0.2), nk, NP)
    fields = _two_polarisations(200)
    rho0 = O.rho_equilibrium(tb4_6) + _drho(tb4_6, 9, 1e-3)
    ctx.set_option(abi.TDG_OPT_BATCHED_MIN, 1 << 20)
    try:
        _log(f"tb4 6x6 intraband {kind} {dtype}, 2 instances, 200 steps")
        res = ctx.propagate(op, dm, "eh", fields, DT, rho=torch.from_numpy(np.stack([rho0, rho0])).cuda(),
                            init_eq=False)
    finally:
        ctx.set_option(abi.TDG_OPT_BATCHED_MIN, 4)
    assert not ctx.last_variant().startswith("batched")
    links = O.transport_links(tb4_6)
    refs = [O.propagate(tb4_6, oop, "eh", fields, DT, instance=b, rho0=rho0, links=links) for b in range(2)]
    _compare(res, refs, tol, 1e-10 if dtype == "c128" else 1e-5)


@pytest.mark.parametrize("model_kind", ["tb4", "multiband8"])
def test_intraband_per_instance_uneven_lengths(P, ctx, model_kind):
    """Per-instance path (FP64) with the intraband term and instances of
    uneven length, one of zero steps: each stage reads the neighbours from
    one stage-state buffer and writes the other, and a finished instance is
    observed from the buffer its last step wrote.  The 8-band model stages
    8 nb^2 = 512 neighbour entries per k (eight 64-lane copies)."""
    from paper_2502_05635_amd import _abi as abi
    m = tb4_model(6, A, 0.5) if model_kind == "tb4" else multiband_model(6, nb=8, nv=4)
    dm = _with_links(P, ctx, m)
    kg = ctx.kernel_build(dm, R0_STABLE, "eh", "c128")
    ko = O.build_kernel(m, R0_STABLE, "eh")
    if model_kind == "tb4":
        op = ctx.kernel_compress(kg, "fraction", 0.3)
        oop = O.LowRankOp.from_factors(O.compress(ko, "fraction", 0.3))
    else:
        op, oop = kg, O.DenseOp(ko)
    tabs = []
    for i, ns in enumerate((0, 37, 121, 160)):
        t = max(ns, 1) * DT
        tabs.append(FieldTable.single(3e-3, 1.4 / HARTREE_EV, max(t / 10.0, 0.5 * FS_AU), t / 2.0, ns,
                                      ex=np.cos(0.9 * i), ey=np.sin(0.9 * i)))
    fields = FieldTable.stack(tabs)
    ctx.set_option(abi.TDG_OPT_BATCHED_MIN, 1 << 20)
    try:
        _log(f"{model_kind} intraband per-instance FP64, lengths 0/37/121/160")
        res = ctx.propagate(op, dm, "eh", fields, DT)
    finally:
        ctx.set_option(abi.TDG_OPT_BATCHED_MIN, 4)
    assert not ctx.last_variant().startswith("batched")
    links = O.transport_links(m)
    refs = [O.propagate(m, oop, "eh", fields, DT, instance=b, links=links) for b in range(4)]
    _compare(res, refs, 1e-10, 1e-10)


@pytest.mark.parametrize("kind", ["dense", "lowrank", "lowrank_bf16x2"])
def test_tb4_intraband_batched_path(P, ctx, tb4_6, k_tb4_6, kind):
    """Uneven batch through the matrix-core path with the intraband term."""
    from paper_2502_05635_amd import _abi as abi
    dm = _with_links(P, ctx, tb4_6)
    kg = ctx.kernel_build(dm, R0_STABLE, "eh", "c64")
    if kind == "dense":
        op, oop = kg, O.DenseOp(k_tb4_6)
    else:
        op = ctx.kernel_compress(kg, "rank", 37, out_dtype="bf16x2" if kind.endswith("bf16x2") else None)
        oop = O.LowRankOp.from_factors(O.compress(k_tb4_6, "rank", 37))
    rng = np.random.default_rng(21)
    tabs = []
    for i in range(6):
        ns = int(rng.integers(1, 200))
        t = ns * DT
        tabs.append(FieldTable.single(10 ** rng.uniform(-3, -2), rng.uniform(0.5, 3.0) / HARTREE_EV,
                                      max(t / 10.0, 0.5 * FS_AU), t / 2.0, ns, ex=np.cos(0.7 * i),
                                      ey=np.sin(0.7 * i)))
    fields = FieldTable.stack(tabs)
    ctx.set_option(abi.TDG_OPT_BATCHED_MIN, 2)
    try:
        _log(f"tb4 6x6 intraband batched {kind}, 6 uneven instances")
        res = ctx.propagate(op, dm, "eh", fields, DT)
    finally:
        ctx.set_option(abi.TDG_OPT_BATCHED_MIN, 4)
    assert ctx.last_variant().startswith("batched_mfma")
    links = O.transport_links(tb4_6)
    refs = [O.propagate(tb4_6, oop, "eh", fields, DT, instance=b, links=links) for b in range(6)]
    tol = 2e-3 if kind.endswith("bf16x2") else 1e-4
    _compare(res, refs, tol, 1e-4)


@pytest.mark.parametrize("links", [False, True])
@pytest.mark.parametrize("tiling", [1, 3, 4])
def test_bf16x2_split_gather_written_by_stage_kernel(P, ctx, tb4_6, k_tb4_6, links, tiling):
    """40 uneven instances (64 per stage-kernel block): with BF16X2 tiling 1,
    3 or 4 the batched stage kernel writes the next projection's split operand
    itself, Hermitian-packed state without the intraband term, full state
    with it.  Four instances against the FP64 oracle; all of them against the
    same run on tiling 0, which splits X in the product (the tilings differ
    only in summation order)."""
    from paper_2502_05635_amd import _abi as abi
    dm = _with_links(P, ctx, tb4_6) if links else P.DeviceModel.from_model(tb4_6)
    kg = ctx.kernel_build(dm, R0_STABLE, "eh", "c64")
    op = ctx.kernel_compress(kg, "rank", 37, out_dtype="bf16x2")
    rng = np.random.default_rng(33)
    tabs = []
    for i in range(40):
        ns = int(rng.integers(20, 90))
        t = ns * DT
        tabs.append(FieldTable.single(10 ** rng.uniform(-3, -2), rng.uniform(0.5, 3.0) / HARTREE_EV,
                                      max(t / 10.0, 0.5 * FS_AU), t / 2.0, ns, ex=np.cos(0.3 * i),
                                      ey=np.sin(0.3 * i)))
    fields = FieldTable.stack(tabs)
    try:
        ctx.set_option(abi.TDG_OPT_GEMM_VARIANT, tiling)
        res = ctx.propagate(op, dm, "eh", fields, DT)
        assert f"tilings {tiling}/{tiling}" in ctx.last_variant()
        ctx.set_option(abi.TDG_OPT_GEMM_VARIANT, 0)
        ref0 = ctx.propagate(op, dm, "eh", fields, DT)
        assert "tilings 0/0" in ctx.last_variant()
    finally:
        ctx.set_option(abi.TDG_OPT_GEMM_VARIANT, -1)
    for key in ("P", "J", "occ"):
        a, b = res[key].cpu().numpy(), ref0[key].cpu().numpy()
        assert np.abs(a - b).max() <= 1e-5 * np.abs(b).max(), key
    oop = O.LowRankOp.from_factors(O.compress(k_tb4_6, "rank", 37))
    lk = O.transport_links(tb4_6) if links else None
    idx = [0, 13, 27, 39]
    refs = [O.propagate(tb4_6, oop, "eh", fields, DT, instance=b, links=lk) for b in idx]
    sub = {k: res[k][idx] for k in ("P", "J", "occ", "tr", "rho")}
    _compare(sub, refs, 2e-3, 1e-4)


def test_intraband_graph_replay_matches_direct(P, ctx, tb4_6):
    from paper_2502_05635_amd import _abi as abi
    dm = _with_links(P, ctx, tb4_6)
    op = ctx.kernel_compress(ctx.kernel_build(dm, R0_STABLE, "eh", "c64"), "rank", 37)
    fields = FieldTable.stack([FieldTable.single(3e-3, 1.5 / HARTREE_EV, 8.0 * FS_AU, 4.0 * FS_AU, 60 + 15 * i,
                                                 ex=np.cos(0.4 * i), ey=np.sin(0.4 * i)) for i in range(5)])
    ctx.set_option(abi.TDG_OPT_BATCHED_MIN, 2)
    ctx.set_option(abi.TDG_OPT_GEMM_VARIANT, 0)
    try:
        ctx.set_option(abi.TDG_OPT_GRAPHS, 0)
        a = ctx.propagate(op, dm, "eh", fields, DT)
        ctx.set_option(abi.TDG_OPT_GRAPHS, 1)
        for rep in range(2):
            b = ctx.propagate(op, dm, "eh", fields, DT)
            torch.cuda.synchronize()
            assert "graphs" in ctx.last_variant()
            for key in ("P", "J", "occ", "tr", "herm", "rho"):
                assert torch.equal(a[key], b[key]), (rep, key)
    finally:
        ctx.set_option(abi.TDG_OPT_GRAPHS, 0)
        ctx.set_option(abi.TDG_OPT_GEMM_VARIANT, -1)
        ctx.set_option(abi.TDG_OPT_BATCHED_MIN, 4)


def test_observables_grid_trace_with_links(P, ctx, tb4_6):
    dm = _with_links(P, ctx, tb4_6)
    rho = O.rho_equilibrium(tb4_6) + _drho(tb4_6, 4)
    rho[:, 1, 1] += 1e-3                                   # grid-mean trace deviation 1e-3
    f = FieldTable.single(1e-3, 0.05, 100.0, 200.0, 10, ex=0.6, ey=0.8)
    out = ctx.observables(dm, torch.from_numpy(rho[None]).cuda(), f).cpu().numpy()[0]
    ref = O.observables(tb4_6, rho, 0.6, 0.8, grid_trace=True)
    for i, key in enumerate(("P", "J", "occ", "tr", "herm")):
        assert abs(out[i] - ref[key]) <= 1e-13 * max(1.0, abs(ref[key])), key
    assert abs(out[3] - 1e-3) < 1e-12


def test_adjoint_with_links_matches_oracle(P, ctx):
    """Adjoint RK4 with the intraband term: field-parameter gradients, dL/dE
    and dL/drho0 against the oracle's adjoint (itself pinned by central
    differences), low-rank FP64 operator, two instances."""
    m = tb4_model(4, A, 0.5)
    dm = _with_links(P, ctx, m)
    kg = ctx.kernel_build(dm, R0_STABLE, "eh", "c128")
    fac = ctx.kernel_compress(kg, "rank", 12)
    oop = O.LowRankOp.from_factors(O.compress(O.build_kernel(m, R0_STABLE, "eh"), "rank", 12))
    ns, dt = 40, 0.2 * FS_AU
    fields = FieldTable.stack([
        FieldTable.single(8e-3, 1.2 / HARTREE_EV, 2.0 * FS_AU, 4.0 * FS_AU, ns, ex=0.6, ey=0.8),
        FieldTable.single(6e-3, 0.9 / HARTREE_EV, 1.5 * FS_AU, 3.0 * FS_AU, ns, ex=-1.0, ey=0.0)])
    rng = np.random.default_rng(17)
    gP, gJ, gocc = (rng.standard_normal((2, ns + 1)) for _ in range(3))
    _log("adjoint with links, tb4 4x4 low rank c128, 2 instances, 40 steps, checkpoints every 7")
    g = ctx.propagate_adjoint(fac, dm, "eh", fields, dt, gP=gP, gJ=gJ, gocc=gocc, checkpoint_every=7,
                              factor_grads=False)
    links = O.transport_links(m)
    for b in range(2):
        ref = O.propagate_adjoint(m, oop, "eh", fields, dt, gP[b], gJ[b], gocc[b], instance=b, links=links)
        for key in ("dfield", "dE", "drho0"):
            got = g[key][b].cpu().numpy()
            e = float(np.abs(got - ref[key]).max() / np.abs(ref[key]).max())
            _log(f"  instance {b} {key}: {e:.2e}")
            assert e <= 1e-9, (b, key)


def test_full_size_intraband_lowrank_fp32(P, ctx):
    """The 36x36 e-h workload (N = 5184) with the intraband term, FP32 low-rank
    operator at 5 %, the first 200 steps of a pulse centred in them, against
    the FP64 oracle with its own kernel, SVD and links."""
    cfg = get_config(1)
    m = cfg.model()
    dm = _with_links(P, ctx, m)
    kg = ctx.kernel_build(dm, R0_STABLE, "eh", "c64")
    fac = ctx.kernel_compress(kg, "fraction", 0.05)
    t = 200 * cfg.dt
    f = FieldTable.single(5e-3, 1.5 / HARTREE_EV, t / 10.0, t / 2.0, 200, ex=0.8, ey=0.6)
    _log(f"36x36 intraband low rank FP32, rank {fac.rank}, 200 steps")
    res = ctx.propagate(fac, dm, "eh", f, cfg.dt)
    _log("  oracle: kernel, SVD, links, 200 steps")
    ko = O.build_kernel(m, R0_STABLE, "eh")
    oop = O.LowRankOp.from_factors(O.compress(ko, "fraction", 0.05, method="eigh"))
    ref = O.propagate(m, oop, "eh", f, cfg.dt, links=O.transport_links(m))
    _compare(res, [ref], 1e-4, 1e-5)
