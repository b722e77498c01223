"""Batched (block-diagonal, one launch) forward and adjoint on the GPU."""
import json
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.helpers import azint, norm_err, oracle_matrix

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_batch(insts, dtype, dev, tile=None, layout="band"):
    """Plans of one fixed tiling (pieces of 2048 nonzeros unless `tile` says
    otherwise: a batch cuts each instance as its plan would, but for the
    balanced rounds of tile_nnz 0, which are one plan's) and their batch."""
    az = azint()
    plans = []
    tile = dict(tile or {})
    tile.setdefault("tile_nnz", 2048)
    for inst in insts:
        g = inst.geom
        p = az.Plan(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), dtype=dtype,
                    layout=layout)
        p.set_tiling(**tile)
        plans.append(p)
    return plans, az.Batch(plans, device=dev)


def flat_images(insts, dtype):
    return np.concatenate([i.raw.reshape(-1) for i in insts]).astype(dtype)


def small_batch(n=40, seed=21):
    return synth.batch(n, 1.0, 2e4, seed, grad=True)


@pytest.mark.parametrize("layout,stage", [("ring", "tile"), ("ring", "gather"),
                                          ("ring", "scatter"), ("pixel", "tile"),
                                          ("tile", "tile"), ("band", "tile"),
                                          ("run", "tile"), ("run", "fuse")])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batch_equals_per_instance_and_oracle(dtype, layout, stage, dev):
    say("batch vs per instance", dtype, layout, stage)
    az = azint()
    insts = small_batch()
    plans, batch = make_batch(insts, dtype, dev, layout=layout, tile=dict(stage=stage))
    npd = np.float64 if dtype == torch.float64 else np.float32
    x = torch.from_numpy(flat_images(insts, npd)).to(dev)
    I, W, U = batch.forward(x, empty=-3.0)
    Il, Wl, Ul = batch.forward(x, empty=-3.0, loop=True)
    raw = torch.from_numpy(np.concatenate([i.raw.reshape(-1) for i in insts])).to(dev)
    Ir, Wr, Ur = batch.forward_raw(raw, empty=-3.0)
    torch.cuda.synchronize()
    # identical tiles per instance -> identical bits
    assert torch.equal(I, Il) and torch.equal(W, Wl) and torch.equal(U, Ul)
    assert torch.equal(I, Ir) and torch.equal(W, Wr) and torch.equal(U, Ur)
    po, bo = batch.pix_off, batch.bin_off
    for k, (inst, plan) in enumerate(zip(insts, plans)):
        plan.upload(dev)
        plan.set_tiling(stage=stage)
        xs = x[po[k]:po[k + 1]].contiguous()
        Ik, Wk, Uk = plan.integrate(xs, empty=-3.0)
        assert torch.equal(Ik, I[bo[k]:bo[k + 1]]), k
        assert torch.equal(Uk, U[bo[k]:bo[k + 1]]), k
        g = inst.geom
        m = oracle_matrix(g.h, g.w, g.center_y, g.center_x, inst.npt)
        xv = inst.raw.reshape(-1).astype(np.float64)
        if dtype == torch.float32:
            m["coef"] = m["coef"].astype(np.float32).astype(np.float64)
        Io, Wo, Uo = oracle.integrate(m, xv, empty=-3.0)
        _, Wa, _ = oracle.integrate(m, np.abs(xv))
        tol = 1e-12 if dtype == torch.float64 else 2.0 ** -22
        Ig = I[bo[k]:bo[k + 1]].double().cpu().numpy()
        Wg = W[bo[k]:bo[k + 1]].double().cpu().numpy()
        assert norm_err(Wg, Wo, Wa) <= tol, k
        sI = np.where(Uo > 0, Wa / np.where(Uo > 0, Uo, 1.0), 0.0)
        assert norm_err(Ig, Io, sI) <= tol, k


@pytest.mark.parametrize("grid", [8, 64, 1024, 0])
@pytest.mark.parametrize("tiling", [(2048, 256, 2, 1), (256, 64, 0, 16), (8192, 512, 3, 16),
                                    (1024, 128, 4, 4), (1024, 64, 5, 16), (512, 64, 6, 2)])
def test_persistent_grid_same_bits(grid, tiling, dev):
    """The tile sums do not depend on which workgroup computes a tile."""
    say("persistent", grid, tiling)
    insts = small_batch(30, 5)
    _, batch = make_batch(insts, torch.float64, dev)
    x = torch.from_numpy(flat_images(insts, np.float64)).to(dev)
    kw = dict(tile_nnz=tiling[0], block=tiling[1], variant=tiling[2], band=tiling[3])
    batch.set_tiling(grid=0, **kw)
    ref = batch.forward(x)
    batch.set_tiling(grid=grid, **kw)
    got = batch.forward(x)
    torch.cuda.synchronize()
    for a, b in zip(ref, got):
        assert torch.equal(a, b)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batch_backward(dtype, dev):
    say("batch backward", dtype)
    insts = small_batch(25, 9)
    plans, batch = make_batch(insts, dtype, dev)
    npd = np.float64 if dtype == torch.float64 else np.float32
    x = torch.from_numpy(flat_images(insts, npd)).to(dev)
    gI = torch.from_numpy(np.concatenate([i.grad for i in insts]).astype(npd)).to(dev)
    I, W, U = batch.forward(x)
    gx = batch.backward(U, gI)
    torch.cuda.synchronize()
    po, bo = batch.pix_off, batch.bin_off
    for k, plan in enumerate(plans):
        plan.upload(dev)
        gk = plan.backward(U[bo[k]:bo[k + 1]].contiguous(), gI[bo[k]:bo[k + 1]].contiguous())
        assert torch.equal(gk, gx[po[k]:po[k + 1]]), k
        inst = insts[k]
        g = inst.geom
        m = oracle_matrix(g.h, g.w, g.center_y, g.center_x, inst.npt)
        if dtype == torch.float32:
            m["coef"] = m["coef"].astype(np.float32).astype(np.float64)
        Uk = U[bo[k]:bo[k + 1]].double().cpu().numpy()
        gik = inst.grad.astype(npd).astype(np.float64)
        ref = oracle.integrate_vjp(m, Uk, gik)
        scale = oracle.integrate_vjp(m, Uk, np.abs(gik))
        tol = 1e-12 if dtype == torch.float64 else 2.0 ** -22
        assert norm_err(gx[po[k]:po[k + 1]].double().cpu().numpy(), ref, scale) <= tol, k


@pytest.mark.parametrize("layout", ["ring", "tile", "band", "run"])
def test_graph_replays_match_eager(layout, dev):
    """A captured forward+backward replays the same bits every time, with
    eager work and synchronisations in between."""
    say("graph replay", layout)
    insts = small_batch(20, 13)
    _, batch = make_batch(insts, torch.float64, dev, layout=layout)
    batch.set_tiling(tile_nnz=1024, block=256, grid=512)
    x = torch.from_numpy(flat_images(insts, np.float64)).to(dev)
    gI = torch.from_numpy(np.concatenate([i.grad for i in insts])).to(dev)
    I0, W0, U0 = batch.forward(x)
    gx0 = batch.backward(U0, gI)
    I, W, U = (torch.full_like(I0, np.nan) for _ in range(3))
    gx = torch.full_like(gx0, np.nan)
    graph = batch.graph(x, I, W, U, grad_I=gI, grad_x=gx)
    for rep in range(4):
        for t in (I, W, U, gx):
            t.fill_(np.nan)
        graph.launch()
        torch.cuda.synchronize()
        assert torch.equal(I, I0) and torch.equal(W, W0) and torch.equal(U, U0), rep
        assert torch.equal(gx, gx0), rep
        _ = (x * 2).sum().item()   # unrelated eager work between replays


def test_plan_graph(dev):
    say("plan graph")
    az = azint()
    inst = synth.instance(20000, 3)
    g = inst.geom
    plan = az.Plan(g.h, g.w, inst.npt, device=dev)
    raw = torch.from_numpy(inst.raw.reshape(-1)).to(dev)
    I0, W0, U0 = plan.integrate_raw(raw)
    I, W, U = (torch.empty_like(I0) for _ in range(3))
    graph = plan.graph(raw, I, W, U)
    for _ in range(3):
        I.zero_()
        graph.launch()
        torch.cuda.synchronize()
        assert torch.equal(I, I0) and torch.equal(W, W0) and torch.equal(U, U0)


def test_graph_keeps_its_owner_alive(dev):
    """A graph records its plan's (or batch's) device matrices and work
    buffers: dropping the caller's last reference to the owner must not free
    them while the graph lives."""
    say("graph owner")
    import gc
    az = azint()
    inst = synth.instance(20000, 5)
    g = inst.geom
    plan = az.Plan(g.h, g.w, inst.npt, device=dev)
    raw = torch.from_numpy(inst.raw.reshape(-1)).to(dev)
    I0, W0, U0 = plan.integrate_raw(raw)
    I, W, U = (torch.empty_like(I0) for _ in range(3))
    graph = plan.graph(raw, I, W, U)
    assert any(k is plan for k in graph._keep)
    del plan
    insts = small_batch(12, 19)
    _, batch = make_batch(insts, torch.float64, dev)
    x = torch.from_numpy(flat_images(insts, np.float64)).to(dev)
    Ib0, Wb0, Ub0 = batch.forward(x)
    Ib, Wb, Ub = (torch.empty_like(Ib0) for _ in range(3))
    bgraph = batch.graph(x, Ib, Wb, Ub)
    assert any(k is batch for k in bgraph._keep)
    del batch, _
    gc.collect()
    # other allocations that could reuse freed memory
    junk = [torch.full((1 << 20,), 7.0, dtype=torch.float64, device=dev) for _ in range(8)]
    for _ in range(2):
        graph.launch()
        bgraph.launch()
        torch.cuda.synchronize()
        assert torch.equal(I, I0) and torch.equal(W, W0) and torch.equal(U, U0)
        assert torch.equal(Ib, Ib0) and torch.equal(Wb, Wb0) and torch.equal(Ub, Ub0)
    del junk


def test_autotune_picks_valid_config(dev, tmp_path):
    say("autotune")
    az = azint()
    insts = small_batch(60, 17)
    _, batch = make_batch(insts, torch.float64, dev)
    x = torch.from_numpy(flat_images(insts, np.float64)).to(dev)
    ref = [t.clone() for t in batch.forward(x)]
    cache = tmp_path / "tune.json"
    rep = az.autotune(batch, x, cache_path=str(cache))
    best = rep["best"]
    assert batch.tiling()["tile_nnz"] == best["tile_nnz"]
    assert len(rep["candidates"]) >= 5
    got = batch.forward(x)
    torch.cuda.synchronize()
    for a, b in zip(ref, got):
        assert torch.allclose(a, b, rtol=1e-12, atol=0)
    # a second call is served from the cache
    batch.set_tiling(tile_nnz=64, block=64, grid=0)
    rep2 = az.autotune(batch, x, cache_path=str(cache))
    assert rep2["best"] == best and batch.tiling()["tile_nnz"] == best["tile_nnz"]
    assert json.loads(cache.read_text())


@pytest.mark.parametrize("layout", ["run", "band", "tile", "ring"])
def test_c3_full_batch_sampled(layout, dev):
    """The 4096-instance workload at full size, in the benchmark's launch
    configuration: batched forward == per-instance loop bit for bit, 12
    sampled instances against the oracle, conservation over all."""
    say("c3 full")
    c = synth.C3
    insts = synth.batch(c["count"], c["lo"], c["hi"], c["seed"])
    plans, batch = make_batch(insts, torch.float64, dev, layout=layout)
    batch.set_tiling(grid=0)
    x = torch.from_numpy(flat_images(insts, np.float64)).to(dev)
    I, W, U = batch.forward(x)
    Il, Wl, Ul = batch.forward(x, loop=True)
    torch.cuda.synchronize()
    assert torch.equal(I, Il) and torch.equal(W, Wl) and torch.equal(U, Ul)
    Ih = I.cpu().numpy()
    Uh = U.cpu().numpy()
    Wh = W.cpu().numpy()
    po, bo = batch.pix_off, batch.bin_off
    xh = x.cpu().numpy()
    for k in range(len(insts)):
        assert abs(Uh[bo[k]:bo[k + 1]].sum() - (po[k + 1] - po[k])) <= 1e-9 * (po[k + 1] - po[k])
        xs = np.abs(xh[po[k]:po[k + 1]]).sum()
        assert abs(Wh[bo[k]:bo[k + 1]].sum() - xh[po[k]:po[k + 1]].sum()) <= 1e-12 * xs
    for k in np.random.default_rng(0).choice(len(insts), 12, replace=False):
        inst = insts[k]
        g = inst.geom
        m = oracle_matrix(g.h, g.w, g.center_y, g.center_x, inst.npt)
        xv = inst.raw.reshape(-1).astype(np.float64)
        Io, Wo, Uo = oracle.integrate(m, xv)
        _, Wa, _ = oracle.integrate(m, np.abs(xv))
        sI = np.where(Uo > 0, Wa / np.where(Uo > 0, Uo, 1.0), 0.0)
        sl = slice(bo[k], bo[k + 1])
        assert norm_err(Wh[sl], Wo, Wa) <= 1e-12, k
        assert norm_err(Uh[sl], Uo, Uo) <= 1e-12, k
        assert norm_err(Ih[sl], Io, sI) <= 1e-12, k
        assert np.all(Ih[sl][Uo == 0] == 0.0) and np.all(Wh[sl][Uo == 0] == 0.0), k


@pytest.mark.parametrize("R,piece", [(4, 512), (8, 2048), (16, 256), (8, 64)])
def test_band_batch_retile(R, piece, dev):
    """Band batches rebuild their bands from the device copy of the matrix
    when the band rows or piece size change; results stay exact and the
    per-instance loop agrees bit for bit."""
    say("band retile", R, piece)
    insts = small_batch(24, 31)
    plans, batch = make_batch(insts, torch.float64, dev, layout="band")
    x = torch.from_numpy(flat_images(insts, np.float64)).to(dev)
    batch.set_tiling(band=R, tile_nnz=piece)
    I, W, U = batch.forward(x)
    Il, Wl, Ul = batch.forward(x, loop=True)
    torch.cuda.synchronize()
    assert torch.equal(I, Il) and torch.equal(W, Wl) and torch.equal(U, Ul)
    po, bo = batch.pix_off, batch.bin_off
    for k in (0, 7, 23):
        inst = insts[k]
        g = inst.geom
        m = oracle_matrix(g.h, g.w, g.center_y, g.center_x, inst.npt)
        xv = inst.raw.reshape(-1).astype(np.float64)
        Io, Wo, Uo = oracle.integrate(m, xv)
        _, Wa, _ = oracle.integrate(m, xv)
        assert norm_err(W[bo[k]:bo[k + 1]].cpu().numpy(), Wo, Wa) <= 1e-12, k
        assert norm_err(U[bo[k]:bo[k + 1]].cpu().numpy(), Uo, Uo) <= 1e-12, k


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_band_fused_correction(dtype, dev):
    """The band kernel with cast and correction in its gather (stage
    "fuse"): against the FP64 oracle and within one rounding per pixel of
    the two-pass results for a plan with all four corrections (the gather
    multiplies by the reciprocal of norm); bit for bit for a batch of raw
    frames without corrections (a plain cast either way)."""
    import oracle
    from tests.test_gpu_forward import TOL32_F64, TOL64, check
    say("band fuse", dtype)
    az = azint()
    npd = np.float64 if dtype == torch.float64 else np.float32
    inst = synth.instance_hw(130, 170, 5, npt=110, corrections=True)
    g = inst.geom
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a).reshape(-1).astype(npd)).to(dev)
    plans = []
    for stage in ("gather", "fuse"):
        p = az.Plan(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), dtype=dtype,
                    device=dev, stage=stage)
        p.set_corrections(t(inst.dark), t(inst.flat), t(inst.solid), t(inst.polar))
        plans.append(p)
    # correction bytes per pixel: none kept by the two-pass stage; 12-byte
    # records for float64 with an integer dark, 8-byte float pairs for float32
    assert plans[0].correction_bytes() == 0
    assert plans[1].correction_bytes() == (12 if dtype == torch.float64 else 8)
    raw = torch.from_numpy(inst.raw.reshape(-1)).to(dev)
    a = plans[0].integrate_raw(raw)
    b = plans[1].integrate_raw(raw)
    torch.cuda.synchronize()
    m = oracle.build_matrix(h=g.h, w=g.w, pixel_y=g.pixel_y, pixel_x=g.pixel_x,
                            center_y=g.center_y, center_x=g.center_x, dist=g.dist,
                            wavelength=g.wavelength, npt=inst.npt)
    f = lambda v: np.ascontiguousarray(v).reshape(-1).astype(npd).astype(np.float64)
    x = oracle.correct(inst.raw.reshape(-1).astype(np.float64), f(inst.dark), f(inst.flat),
                       f(inst.solid), f(inst.polar))
    tol = TOL64 if dtype == torch.float64 else TOL32_F64
    check(b, m, x, tol, what="fused")
    check(a, m, x, tol, what="two pass")
    # switching the stage after the corrections builds the pairs then
    plans[0].set_tiling(stage="fuse")
    assert plans[0].correction_bytes() == plans[1].correction_bytes()
    c = plans[0].integrate_raw(raw)
    torch.cuda.synchronize()
    for u, v in zip(b, c):
        assert torch.equal(u, v)
    insts = small_batch(30, 23)
    _, b0 = make_batch(insts, dtype, dev)
    _, b1 = make_batch(insts, dtype, dev, tile=dict(stage="fuse"))
    rawb = torch.from_numpy(np.concatenate([i.raw.reshape(-1) for i in insts])).to(dev)
    for u, v in zip(b0.forward_raw(rawb), b1.forward_raw(rawb)):
        assert torch.equal(u, v)
    # graph capture of the one-kernel path
    I0, W0, U0 = b
    I, W, U = (torch.full_like(I0, np.nan) for _ in range(3))
    graph = plans[1].graph(raw, I, W, U)
    for _ in range(3):
        graph.launch()
        torch.cuda.synchronize()
        assert torch.equal(I, I0) and torch.equal(W, W0) and torch.equal(U, U0)


def test_batch_of_run_plans(dev):
    """A batch of run-layout plans keeps the run encoding: bit for bit the
    plan-by-plan results, within the FP64 tolerance of the oracle, and the
    raw-frame form equals the corrected-image form for uncorrected frames.
    Plans of the band and run layouts do not mix in one batch."""
    import oracle
    from tests.test_gpu_forward import TOL64, check
    say("batch of run plans")
    insts = small_batch(24, 33)
    plans, br = make_batch(insts, torch.float64, dev, layout="run")
    x = flat_images(insts, np.float64)
    I, W, U = br.forward(torch.from_numpy(x).to(dev))
    raw = torch.from_numpy(np.concatenate([i.raw.reshape(-1) for i in insts])).to(dev)
    Ir, Wr, Ur = br.forward_raw(raw)
    torch.cuda.synchronize()
    assert torch.equal(I, Ir) and torch.equal(W, Wr) and torch.equal(U, Ur)
    po = bo = 0
    for plan, inst in zip(plans, insts):
        g = inst.geom
        plan.upload(dev)
        xk = inst.raw.reshape(-1).astype(np.float64)
        out = plan.integrate(torch.from_numpy(xk).to(dev))
        n = inst.npt
        for a, b in zip((I, W, U), out):
            assert torch.equal(a[bo:bo + n], b)
        m = oracle.build_matrix(h=g.h, w=g.w, pixel_y=g.pixel_y, pixel_x=g.pixel_x,
                                center_y=g.center_y, center_x=g.center_x, dist=g.dist,
                                wavelength=g.wavelength, npt=n)
        check(out, m, xk, TOL64, what=f"instance {g.h}x{g.w}")
        bo += n
        po += g.npix
    az = azint()
    mixed = [az.Plan(10, 12, 6, layout="run"), az.Plan(10, 12, 6, layout="band")]
    with pytest.raises(az.AzintError):
        az.Batch(mixed, device=dev)


def test_c5_full_batch_sampled(dev):
    """The 1024-instance float32 workload at full size (1.4e8 pixels) in the
    benchmark's launch configuration (default layout, autotuned tiling):
    the batched forward equals the per-instance loop bit for bit and
    conserves every instance; sampled instances' forward and adjoint match
    the FP64 oracle to the float32 tolerance."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    from tests.test_gpu_forward import TOL32_F64
    say("c5 full")
    az = azint()
    c = synth.C5
    insts = synth.batch(c["count"], c["lo"], c["hi"], c["seed"], grad=True)

    def mk(inst):
        g = inst.geom
        return az.Plan(g.h, g.w, inst.npt, center=(g.center_y, g.center_x),
                       dtype=torch.float32)

    with ThreadPoolExecutor(16) as ex:
        plans = list(ex.map(mk, insts))
    batch = az.Batch(plans, device=dev)
    x = torch.from_numpy(flat_images(insts, np.float32)).to(dev)
    az.autotune(batch, x)
    say("  tiling", batch.tiling())
    I, W, U = batch.forward(x)
    Il, Wl, Ul = batch.forward(x, loop=True)
    gI = torch.from_numpy(np.concatenate([i.grad for i in insts]).astype(np.float32)).to(dev)
    gx = batch.backward(U, gI)
    torch.cuda.synchronize()
    assert torch.equal(I, Il) and torch.equal(W, Wl) and torch.equal(U, Ul)
    Wh, Uh, gh = W.double().cpu().numpy(), U.double().cpu().numpy(), gx.double().cpu().numpy()
    xh = x.double().cpu().numpy()
    po, bo = batch.pix_off, batch.bin_off
    for k in range(len(insts)):
        n = po[k + 1] - po[k]
        assert abs(Uh[bo[k]:bo[k + 1]].sum() - n) <= 1e-5 * n, k
        xs = xh[po[k]:po[k + 1]].sum()
        assert abs(Wh[bo[k]:bo[k + 1]].sum() - xs) <= 1e-5 * xs, k
    sizes = np.diff(po)
    picks = list(np.random.default_rng(5).choice(len(insts), 6, replace=False))
    picks.append(int(np.argmax(sizes)))
    for k in picks:
        inst = insts[k]
        g = inst.geom
        m = oracle_matrix(g.h, g.w, g.center_y, g.center_x, inst.npt)
        xv = xh[po[k]:po[k + 1]]
        Io, Wo, Uo = oracle.integrate(m, xv)
        assert norm_err(Wh[bo[k]:bo[k + 1]], Wo, Wo) <= TOL32_F64, k
        assert norm_err(Uh[bo[k]:bo[k + 1]], Uo, Uo) <= TOL32_F64, k
        gk = inst.grad.astype(np.float32).astype(np.float64)
        ref = oracle.integrate_vjp(m, Uo, gk)
        scale = oracle.integrate_vjp(m, Uo, np.abs(gk))
        assert norm_err(gh[po[k]:po[k + 1]], ref, scale) <= TOL32_F64, k


@pytest.mark.parametrize("band", [4, 16])
@pytest.mark.parametrize("dtype,accum", [(torch.float64, "f64"), (torch.float32, "kahan32")])
def test_lane_and_wavefront_reductions_agree(dtype, accum, band, dev):
    """A launch whose bins all have at most 8 band partials finishes them one
    lane per bin; otherwise one wavefront per bin.  Both combine a bin's
    partials in the same order, so a batch holding an image with long bands
    (more than 8 partials per bin: the wavefront form for the whole batch)
    equals, bit for bit, each of the other images integrated alone (the lane
    form), over bins with 1 to 8 partials."""
    say("lane vs wavefront reduction", dtype, accum)
    az = azint()
    # band 16 cuts the 100 x 100 image's bands into 9 pieces: a smaller one there
    geoms = [(300, 300, 20), (100, 100, 50) if band == 4 else (96, 96, 50), (64, 64, 40),
             (70, 50, 45)]
    tile = 512
    plans = []
    for h, w, n in geoms:
        p = az.Plan(h, w, n, center=(h / 2 + 0.3, w / 2 - 0.7), dtype=dtype, accum=accum,
                    layout="run")
        p.set_tiling(tile_nnz=tile, band=band)
        plans.append(p)
    counts = [p.run_schedule(tile)["bin_count"] for p in plans]
    assert counts[0].max() > 8
    assert all(c.max() <= 8 for c in counts[1:])
    if band == 4:
        assert set(np.concatenate(counts[1:]).tolist()) == set(range(1, 9))
    batch = az.Batch(plans, device=dev)
    batch.set_tiling(tile_nnz=tile)
    assert batch.tiling()["tile_nnz"] == tile
    rng = np.random.default_rng(41)
    npd = np.float64 if dtype == torch.float64 else np.float32
    xs = [rng.uniform(-5.0, 1000.0, size=h * w).astype(npd) for h, w, _ in geoms]
    I, W, U = batch.forward(torch.from_numpy(np.concatenate(xs)).to(dev), empty=-2.0)
    torch.cuda.synchronize()
    bo = batch.bin_off
    for k, (plan, x) in enumerate(zip(plans, xs)):
        plan.upload(dev)
        assert plan.tiling()["tile_nnz"] == tile
        out = plan.integrate(torch.from_numpy(x).to(dev), empty=-2.0)
        for a, b in zip((I, W, U), out):
            assert torch.equal(a[bo[k]:bo[k + 1]], b), (k, geoms[k])
