"""GPU forward path vs the FP64 oracle, element by element (C-ABI calls)."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.helpers import azint, norm_err, oracle_matrix

pytestmark = pytest.mark.gpu

TOL64 = 1e-12          # FP64: normalised by sum_p A_bp |x_p| per bin
TOL32_SAME = 2.0 ** -22  # FP32 storage, FP64 accumulation, vs oracle on the same FP32 inputs
TOL32_F64 = 1e-6       # FP32 storage vs the FP64 oracle on FP64 inputs
TOLK32 = 4e-7          # FP32 storage, Kahan float sums, vs oracle on the same FP32 inputs


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def scales(m, x):
    """Per-bin scales: sum A|x| for W and I (the latter / U), U for U."""
    _, Wabs, U = oracle.integrate(m, np.abs(x))
    sI = np.where(U > 0, Wabs / np.where(U > 0, U, 1.0), 0.0)
    return sI, Wabs, U


def check(out, m, x, tol, empty=0.0, what=""):
    I, W, U = (t.double().cpu().numpy() for t in out)
    Io, Wo, Uo = oracle.integrate(m, x, empty=empty)
    sI, sW, sU = scales(m, x)
    eI, eW, eU = norm_err(I, Io, sI), norm_err(W, Wo, sW), norm_err(U, Uo, sU)
    empty_bins = Uo == 0
    if np.isnan(empty):
        assert np.all(np.isnan(I[empty_bins])), what
    else:
        assert np.all(I[empty_bins] == empty), what
    assert np.all(W[empty_bins] == 0) and np.all(U[empty_bins] == 0), what
    assert eI <= tol and eW <= tol and eU <= tol, (what, eI, eW, eU)
    return eI, eW, eU


GEOMS = [
    # h, w, center_y, center_x, npt, unit, split, range
    (100, 100, 50.0, 50.0, 100, "r_m", "bbox", None),
    (37, 53, 10.25, 40.5, 61, "r_m", "bbox", None),
    (64, 48, -5.0, 70.0, 40, "r_m", "bbox", None),
    (31, 29, 15.5, 14.5, 300, "r_m", "bbox", None),
    (45, 45, 22.5, 22.5, 7, "r_m", "bbox", None),
    (50, 60, 25.0, 30.0, 37, "r_m", "bbox", (5e-4, 2.5e-3)),
    (50, 60, 25.3, 30.7, 37, "r_m", "none", None),
    (1, 1, 0.5, 0.5, 4, "r_m", "bbox", None),
    (1, 17, 0.5, 8.5, 5, "r_m", "bbox", None),
    (257, 263, 128.5, 131.5, 256, "r_m", "bbox", None),
    (300, 200, 10.0, 190.0, 150, "2th_deg", "bbox", None),
    (120, 130, 60.2, 64.9, 140, "r_m", "full", None),
    (90, 70, -10.0, 35.0, 80, "q_nm", "full", None),
]
# tile_nnz, block, variant, grid, band
TILINGS = [(2048, 256, 3, 0, 1, 2), (1024, 64, 3, 0, 16, 0), (2048, 256, 2, 0, 1, 1),
           (64, 64, 0, 0, 16, 2), (256, 128, 1, 0, 4, 0), (1024, 512, 3, 64, 16, 1),
           (16384, 256, 4, 0, 1, 2), (128, 64, 5, 8, 16, 0), (4096, 512, 6, 0, 2, 1),
           (512, 256, 3, 2048, 1, 2), (0, 256, 5, 0, 32, 4)]


def tiling_kw(t):
    return dict(zip(("tile_nnz", "block", "variant", "grid", "band", "stage"), t))


@pytest.mark.parametrize("layout", ["ring", "pixel", "tile", "band", "run"])
@pytest.mark.parametrize("tiling", TILINGS, ids=lambda t: "t{}b{}v{}g{}n{}s{}".format(*t))
@pytest.mark.parametrize("g", GEOMS, ids=lambda g: f"{g[0]}x{g[1]}-{g[5]}-{g[6]}-{g[4]}")
def test_forward_f64(g, tiling, layout, dev):
    h, w, cy, cx, npt, unit, split, rng = g
    say("forward f64", g, tiling, layout)
    az = azint()
    plan = az.Plan(h, w, npt, center=(cy, cx), unit=unit, split=split, range=rng,
                   layout=layout, device=dev, **tiling_kw(tiling))
    m = oracle_matrix(h, w, cy, cx, npt, 1e-4, 1e-4, unit, split, rng)
    x = np.random.default_rng(h * w + npt).uniform(-2.0, 1000.0, size=h * w)
    out = plan.integrate(torch.from_numpy(x).to(dev), empty=-1.5)
    torch.cuda.synchronize()
    check(out, m, x, TOL64, empty=-1.5, what=str(g))


def test_c1_workload(dev):
    """The smallest workload: 100x100 float64, seed 0, npt 100."""
    say("c1")
    az = azint()
    inst = synth.instance(synth.C1["n"], synth.C1["seed"])
    g = inst.geom
    plan = az.Plan(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), device=dev)
    m = oracle_matrix(g.h, g.w, g.center_y, g.center_x, inst.npt)
    x = inst.raw.reshape(-1).astype(np.float64)
    raw = torch.from_numpy(inst.raw.reshape(-1)).to(dev)
    out = plan.integrate_raw(raw)
    torch.cuda.synchronize()
    check(out, m, x, TOL64, what="c1")
    # identical bits through the corrected-image entry point and on a rerun
    out2 = plan.integrate(torch.from_numpy(x).to(dev))
    out3 = plan.integrate(torch.from_numpy(x).to(dev))
    torch.cuda.synchronize()
    for a, b, c in zip(out, out2, out3):
        assert torch.equal(a, b) and torch.equal(b, c)


@pytest.mark.parametrize("raw_dtype", [np.int32, np.uint16, np.int16, np.uint32, np.float32,
                                       np.float64])
def test_correction_map_bit_exact(raw_dtype, dev):
    """(raw - dark) / ((flat*solid)*polar) in FP64 is correctly rounded on both
    sides, so the GPU map equals the oracle bit for bit."""
    say("correction", raw_dtype)
    az = azint()
    inst = synth.instance_hw(61, 67, 5, npt=40, corrections=True)
    g = inst.geom
    plan = az.Plan(g.h, g.w, 40, device=dev)
    hi = np.iinfo(raw_dtype).max if np.issubdtype(raw_dtype, np.integer) else 1 << 20
    raw_np = np.random.default_rng(2).integers(0, min(hi, 1 << 20), size=g.npix).astype(raw_dtype)
    raw = torch.from_numpy(raw_np).to(dev)
    t = lambda a: torch.from_numpy(a.reshape(-1)).to(dev)
    for combo in [(1, 1, 1, 1), (1, 0, 0, 0), (0, 1, 1, 0), (0, 0, 0, 1), (0, 0, 0, 0)]:
        arrs = [a if on else None for a, on in zip((inst.dark, inst.flat, inst.solid, inst.polar), combo)]
        plan.set_corrections(*(None if a is None else t(a) for a in arrs))
        x = plan.correct(raw).cpu().numpy()
        ref = oracle.correct(raw_np, *arrs)
        assert np.array_equal(x, ref), combo


@pytest.mark.parametrize("layout,stage", [("ring", "tile"), ("ring", "gather"),
                                          ("ring", "scatter"), ("pixel", "tile"),
                                          ("tile", "tile"), ("band", "tile"),
                                          ("band", "fuse"), ("ring", "fuse"),
                                          ("run", "fuse"), ("run", "gather")])
def test_raw_pipeline_with_corrections(layout, stage, dev):
    say("raw pipeline with corrections", layout, stage)
    az = azint()
    inst = synth.instance_hw(211, 190, 7, npt=160, corrections=True)
    g = inst.geom
    plan = az.Plan(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), layout=layout,
                   stage=stage, device=dev)
    t = lambda a: torch.from_numpy(a.reshape(-1)).to(dev)
    plan.set_corrections(t(inst.dark), t(inst.flat), t(inst.solid), t(inst.polar))
    out = plan.integrate_raw(t(inst.raw))
    torch.cuda.synchronize()
    m = oracle_matrix(g.h, g.w, g.center_y, g.center_x, inst.npt)
    x = oracle.correct(inst.raw, inst.dark, inst.flat, inst.solid, inst.polar)
    check(out, m, x, TOL64, what="corrected")
    # the same through the corrected-image entry point (a separate pass
    # brings the row-major image into the layout)
    xd = plan.correct(t(inst.raw))
    assert np.array_equal(xd.cpu().numpy(), x)
    out2 = plan.integrate(xd)
    torch.cuda.synchronize()
    if layout in ("band", "run") and stage == "fuse":
        # the fused gather multiplies by the reciprocal of norm: one rounding
        # per pixel away from the corrected image's quotient
        check(out2, m, x, TOL64, what="corrected image")
    else:
        for a, b in zip(out, out2):
            assert torch.equal(a, b)


@pytest.mark.parametrize("layout", ["band", "run"])
def test_fused_correction_record_and_pair_same_bits(layout, dev):
    """A float64 plan keeps (dark, 1/norm) as 12-byte records when every dark
    value is a float and as 16-byte pairs otherwise.  Changing dark only on a
    pixel that feeds no bin switches the form and must leave every bit of
    the result unchanged; both results match the oracle."""
    say("correction record vs pair")
    az = azint()
    inst = synth.instance_hw(151, 140, 8, npt=120, corrections=True)
    g = inst.geom
    rng_r = (4e-4, 6e-3)  # the inner disc of radius 4e-4 m feeds no bin
    plan = az.Plan(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), range=rng_r,
                   layout=layout, stage="fuse", device=dev)
    colptr = plan.export_csc()[2]
    empty_pix = np.flatnonzero(np.diff(colptr) == 0)
    assert empty_pix.size > 0
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).to(dev)
    dark_f = inst.dark.reshape(-1).copy()          # integers: floats
    dark_d = dark_f.copy()
    dark_d[empty_pix[0]] = 0.1                      # not a float
    outs, sizes, forms = [], [], []
    for dark in (dark_f, dark_d):
        plan.set_corrections(t(dark), t(inst.flat), t(inst.solid), t(inst.polar))
        sizes.append(plan.device_bytes())
        forms.append(plan.correction_bytes())
        outs.append(plan.integrate_raw(t(inst.raw)))
        torch.cuda.synchronize()
    assert forms == [12, 16]
    assert sizes[1] - sizes[0] == 4 * g.npix      # pairs are 4 bytes longer per pixel
    for a, b in zip(*outs):
        assert torch.equal(a, b)
    m = oracle_matrix(g.h, g.w, g.center_y, g.center_x, inst.npt, 1e-4, 1e-4, "r_m", "bbox",
                      rng_r)
    for dark, out in zip((dark_f, dark_d), outs):
        x = oracle.correct(inst.raw.reshape(-1), dark, inst.flat.reshape(-1),
                           inst.solid.reshape(-1), inst.polar.reshape(-1))
        check(out, m, x, TOL64, what="record/pair")


@pytest.mark.parametrize("layout", ["ring", "pixel", "tile", "band", "run"])
@pytest.mark.parametrize("accum", ["f64", "kahan32"])
@pytest.mark.parametrize("tiling", [(2048, 256, 2, 0, 1, 2), (64, 64, 0, 0, 16, 0),
                                    (512, 512, 3, 0, 16, 1), (1024, 128, 1, 256, 4, 2),
                                    (8192, 256, 4, 0, 1, 0), (1024, 64, 5, 0, 16, 1),
                                    (2048, 128, 6, 16, 16, 2)])
def test_forward_f32(accum, tiling, layout, dev):
    say("forward f32", accum, tiling, layout)
    az = azint()
    h, w, npt = 240, 250, 230
    plan = az.Plan(h, w, npt, center=(119.3, 125.8), dtype=torch.float32, accum=accum,
                   layout=layout, device=dev, **tiling_kw(tiling))
    m = oracle_matrix(h, w, 119.3, 125.8, npt)
    x64 = np.random.default_rng(3).integers(0, 1 << 20, size=h * w).astype(np.float64)
    out = plan.integrate(torch.from_numpy(x64.astype(np.float32)).to(dev))
    torch.cuda.synchronize()
    m32 = dict(m)
    m32["coef"] = m["coef"].astype(np.float32).astype(np.float64)
    tol = TOL32_SAME if accum == "f64" else TOLK32
    check(out, m32, x64, tol, what=f"f32 {accum} same inputs")
    check(out, m, x64, TOL32_F64, what=f"f32 {accum} vs f64 oracle")


def test_kahan32_long_rows_within_bound(dev):
    """Few wide bins: rows of ~10^5 terms.  The Kahan float sums (Section
    5.2.2) stay within their bound of the FP64 sums, and closer to them than
    plain float32 sums of the same products taken in row order on the host
    (the uncompensated sum the paper's compensation is there to improve)."""
    say("kahan long rows")
    az = azint()
    h, w, npt = 400, 400, 6
    plan = az.Plan(h, w, npt, dtype=torch.float32, accum="kahan32", tile_nnz=16384, block=256,
                   device=dev)
    m = oracle_matrix(h, w, 200.0, 200.0, npt)
    x = np.random.default_rng(4).integers(0, 1 << 20, size=h * w).astype(np.float64)
    out = plan.integrate(torch.from_numpy(x.astype(np.float32)).to(dev))
    m32 = dict(m)
    m32["coef"] = m["coef"].astype(np.float32).astype(np.float64)
    check(out, m32, x, TOLK32, what="kahan")
    _, Wo, _ = oracle.integrate(m32, x)
    Wk = out[1].double().cpu().numpy()
    c32 = m["data"].astype(np.float32)
    prod = c32 * x[m["indices"]].astype(np.float32)
    plain = np.array([np.add.accumulate(prod[m["indptr"][b]:m["indptr"][b + 1]],
                                        dtype=np.float32)[-1] for b in range(npt)])
    err_k = np.abs(Wk - Wo) / np.abs(Wo)
    err_p = np.abs(plain.astype(np.float64) - Wo) / np.abs(Wo)
    assert err_k.max() < err_p.max(), (err_k, err_p)


def test_empty_and_degenerate(dev):
    say("empty and degenerate")
    az = azint()
    # a range that holds no pixel: every bin is empty
    plan = az.Plan(20, 20, 16, range=(1.0, 2.0), device=dev)
    assert plan.nnz == 0
    x = torch.rand(400, dtype=torch.float64, device=dev)
    I, W, U = plan.integrate(x, empty=np.nan)
    assert torch.isnan(I).all() and (W == 0).all() and (U == 0).all()
    # many more bins than pixels: most bins empty, the rest exact
    plan = az.Plan(6, 5, 500, center=(3.0, 2.5), device=dev)
    m = oracle_matrix(6, 5, 3.0, 2.5, 500)
    xv = np.arange(30, dtype=np.float64) + 1.0
    out = plan.integrate(torch.from_numpy(xv).to(dev), empty=np.nan)
    check(out, m, xv, TOL64, empty=np.nan, what="sparse bins")
    # outputs W / U may be omitted
    I_only = torch.empty(500, dtype=torch.float64, device=dev)
    az.lib().azi_integrate1d(plan.handle, torch.from_numpy(xv).to(dev).data_ptr(),
                             I_only.data_ptr(), None, None, 0.0, None)
    torch.cuda.synchronize()
    Io, _, Uo = oracle.integrate(m, xv)
    nz = Uo > 0
    assert np.allclose(I_only.cpu().numpy()[nz], Io[nz], rtol=1e-12, atol=0)


def _sampled_bins_oracle(g, npt, x, bins):
    """Oracle values of a few bins of a large image, computed from only the
    pixels whose radial box overlaps them."""
    lo, hi, _ = oracle.pixel_extents(g.h, g.w, g.pixel_y, g.pixel_x, g.center_y, g.center_x,
                                     g.dist, g.wavelength, "r_m")
    pmin, pmax = float(lo.min()), float(hi.max())
    delta = (pmax - pmin) / npt
    out = {}
    for b in bins:
        e0, e1 = pmin + (b - 1) * delta, pmin + (b + 2) * delta
        sel = np.nonzero((hi >= e0) & (lo <= e1))[0]
        pix, bb, coef = oracle.bbox_entries(lo[sel], hi[sel], npt, pmin, pmax)
        keep = bb == b
        m = dict(npt=npt, pix=sel[pix[keep]], bins=np.zeros(keep.sum(), dtype=np.int64),
                 coef=coef[keep])
        out[b] = (oracle.integrate(dict(m, npt=1), x), oracle.integrate(dict(m, npt=1), np.abs(x)))
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_c2_full_size_sampled(dtype, dev):
    # default plan settings: the launch configuration the benchmark times
    """The ~1e7-pixel workload at full size, in the launch configuration the
    benchmark times: 24 sampled bins against the oracle, plus conservation
    over all bins."""
    say("c2 full size", dtype)
    az = azint()
    inst = synth.instance(synth.C2["n"], synth.C2["seed"])
    g = inst.geom
    tdt = torch.float64 if dtype == "f64" else torch.float32
    plan = az.Plan(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), dtype=tdt, device=dev)
    raw = torch.from_numpy(inst.raw.reshape(-1)).to(dev)
    I, W, U = plan.integrate_raw(raw)
    torch.cuda.synchronize()
    I, W, U = (t.double().cpu().numpy() for t in (I, W, U))
    x = inst.raw.reshape(-1).astype(np.float64)
    bins = np.unique(np.r_[0, 1, 2, inst.npt - 1, inst.npt - 2,
                           np.random.default_rng(0).choice(inst.npt, 19, replace=False)])
    ref = _sampled_bins_oracle(g, inst.npt, x, bins)
    tol = TOL64 if dtype == "f64" else TOL32_F64
    for b, ((Io, Wo, Uo), (_, Wa, _)) in ref.items():
        assert abs(W[b] - Wo[0]) <= tol * Wa[0], (b, W[b], Wo[0])
        assert abs(U[b] - Uo[0]) <= tol * Uo[0], (b, U[b], Uo[0])
        assert abs(I[b] - Io[0]) <= tol * Wa[0] / Uo[0], (b, I[b], Io[0])
    assert abs(U.sum() - g.npix) <= (1e-12 if dtype == "f64" else 1e-6) * g.npix
    assert abs(W.sum() - x.sum()) <= (1e-12 if dtype == "f64" else 1e-6) * x.sum()


def test_tile_layout_grid_keeps_bits(dev):
    """Persistent launches of the blocked kernel give the same bits."""
    say("tile layout grid")
    az = azint()
    plan = az.Plan(700, 650, 600, center=(350.2, 320.9), layout="tile", device=dev)
    x = torch.from_numpy(np.random.default_rng(9).uniform(0, 9, 700 * 650)).to(dev)
    ref = [t.clone() for t in plan.integrate(x)]
    for block, grid in ((128, 0), (512, 0), (256, 8), (256, 100), (128, 2048)):
        plan.set_tiling(block=block, grid=grid)
        got = plan.integrate(x)
        torch.cuda.synchronize()
        for a, b in zip(ref, got):
            assert torch.equal(a, b), (block, grid)


@pytest.mark.parametrize("variant", range(7))
def test_schedule_changes_keep_bits(variant, dev):
    """Persistent launches and the staging mode only change which workgroup
    computes a tile or how the image reaches the layout, so every output bit
    stays the same for a given tile size, band and variant."""
    say("schedule bits", variant)
    az = azint()
    plan = az.Plan(700, 650, 600, center=(350.2, 320.9), device=dev, tile_nnz=512, block=64,
                   variant=variant, band=4, grid=0, layout="ring")
    x = torch.from_numpy(np.random.default_rng(9).uniform(0, 9, 700 * 650)).to(dev)
    ref = [t.clone() for t in plan.integrate(x)]
    # the staging mode changes only how the image reaches the ring layout
    for grid, stage in ((0, 2), (0, 0), (2048, 1), (512, 2), (8, 0)):
        plan.set_tiling(grid=grid, stage=stage)
        got = plan.integrate(x)
        torch.cuda.synchronize()
        for a, b in zip(ref, got):
            assert torch.equal(a, b), (variant, grid, stage)


def test_layout_switch_and_errors(dev):
    """Changing the layout re-uploads; both give the oracle's values; the
    layout cannot change under live corrections, and the refused call
    leaves the plan in its layout, still integrating correctly."""
    say("layout switch")
    az = azint()
    plan = az.Plan(90, 80, 70, center=(45.5, 40.1), layout="pixel", device=dev)
    m = oracle_matrix(90, 80, 45.5, 40.1, 70)
    x = np.random.default_rng(2).uniform(0, 10, 90 * 80)
    xd = torch.from_numpy(x).to(dev)
    check(plan.integrate(xd), m, x, TOL64, what="pixel")
    plan.set_layout("ring")
    assert plan.layout() == "ring"
    check(plan.integrate(xd), m, x, TOL64, what="ring")
    plan.set_corrections(dark=torch.zeros(90 * 80, dtype=torch.float64, device=dev))
    for other in ("pixel", "run", "band", "tile"):
        with pytest.raises(az.AzintError, match="before the corrections"):
            plan.set_layout(other)
        assert plan.layout() == "ring"
    check(plan.integrate(xd), m, x, TOL64, what="ring after refused switch")
    raw = torch.from_numpy(np.round(x * 100).astype(np.int32)).to(dev)
    check(plan.integrate_raw(raw), m, np.round(x * 100), TOL64, what="raw after refused switch")


@pytest.mark.parametrize("R", [4, 8, 16])
@pytest.mark.parametrize("piece,block,grid", [(2048, 256, 0), (64, 128, 0), (512, 512, 2048),
                                              (16384, 256, 8)])
def test_band_layout_shapes(R, piece, block, grid, dev):
    say("band shapes", R, piece, block, grid)
    az = azint()
    plan = az.Plan(300, 280, 250, center=(150.2, 139.7), layout="band", device=dev,
                   band=R, tile_nnz=piece, block=block, grid=grid)
    m = oracle_matrix(300, 280, 150.2, 139.7, 250)
    x = np.random.default_rng(R + piece).uniform(-1, 50, 300 * 280)
    check(plan.integrate(torch.from_numpy(x).to(dev), empty=7.0), m, x, TOL64, empty=7.0,
          what="band")


@pytest.mark.parametrize("piece,grid", [(4096, 0), (64, 0), (128, 8), (16384, 2048), (1024, 64),
                                        (0, 0), (0, 96)])
@pytest.mark.parametrize("g", [(300, 280, 150.2, 139.7, 250, "r_m", "bbox"),
                               (1, 17, 0.5, 8.5, 5, "r_m", "bbox"),
                               (64, 48, -5.0, 70.0, 40, "r_m", "bbox"),
                               (120, 130, 60.2, 64.9, 140, "r_m", "full"),
                               (50, 60, 25.3, 30.7, 37, "r_m", "none"),
                               (20, 20, 10.0, 10.0, 1, "r_m", "bbox"),
                               (90, 70, -10.0, 35.0, 80, "q_nm", "full")],
                         ids=lambda g: f"{g[0]}x{g[1]}-{g[5]}-{g[6]}-{g[4]}")
def test_run_layout_shapes(g, piece, grid, dev):
    """The run encoding of the band layout (a word per pixel run within a
    band, coefficients slot-major per 64 runs) against the oracle, for
    pieces from one group of 64 runs to 8192 runs and persistent grids, and
    within FP64 rounding of the per-entry band encoding; piece 0: the
    balanced pieces the library sizes for the device."""
    h, w, cy, cx, npt, unit, split = g
    say("run shapes", g, piece, grid)
    az = azint()
    plan = az.Plan(h, w, npt, center=(cy, cx), unit=unit, split=split, layout="run", device=dev,
                   tile_nnz=piece, grid=grid)
    band = az.Plan(h, w, npt, center=(cy, cx), unit=unit, split=split, layout="band", device=dev)
    m = oracle_matrix(h, w, cy, cx, npt, 1e-4, 1e-4, unit, split)
    x = np.random.default_rng(h + piece).uniform(-1, 50, h * w)
    xt = torch.from_numpy(x).to(dev)
    out = plan.integrate(xt, empty=7.0)
    again = plan.integrate(xt, empty=7.0)
    ref = band.integrate(xt, empty=7.0)
    torch.cuda.synchronize()
    check(out, m, x, TOL64, empty=7.0, what="run")
    for a, b in zip(out, again):
        assert torch.equal(a, b)
    _, Wabs, Uo = oracle.integrate(m, np.abs(x))
    assert norm_err(out[1].cpu().numpy(), ref[1].cpu().numpy(), Wabs) <= 2 * TOL64
    assert norm_err(out[2].cpu().numpy(), ref[2].cpu().numpy(), Uo) <= 2 * TOL64


def test_run_layout_c2_full_size(dev):
    """The 10-Mpixel float64 workload in the run layout, raw frame with
    corrections as the benchmark runs it: sampled bins against the oracle
    one by one, every bin against the per-entry band encoding, and
    conservation."""
    say("run c2")
    az = azint()
    inst = synth.instance(synth.C2["n"], synth.C2["seed"], corrections=True)
    g = inst.geom
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).to(dev)
    plans = {}
    for layout in ("run", "band"):
        p = az.Plan(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), layout=layout,
                    device=dev)
        p.set_corrections(t(inst.dark), t(inst.flat), t(inst.solid), t(inst.polar))
        plans[layout] = p
    raw = t(inst.raw)
    I, W, U = (a.cpu().numpy() for a in plans["run"].integrate_raw(raw))
    Ib, Wb, Ub = (a.cpu().numpy() for a in plans["band"].integrate_raw(raw))
    x = oracle.correct(inst.raw.reshape(-1), inst.dark.reshape(-1), inst.flat.reshape(-1),
                       inst.solid.reshape(-1), inst.polar.reshape(-1))
    assert np.all(np.abs(U - Ub) <= 2 * TOL64 * Ub)
    assert np.all(np.abs(W - Wb) <= 2 * TOL64 * np.abs(Wb))
    assert abs(U.sum() - g.npix) <= 1e-12 * g.npix
    assert abs(W.sum() - x.sum()) <= 1e-12 * np.abs(x).sum()
    bins = np.unique(np.r_[0, 1, inst.npt - 1, np.random.default_rng(2).choice(inst.npt, 13,
                                                                                  replace=False)])
    for b, ((Io, Wo, Uo), (_, Wa, _)) in _sampled_bins_oracle(g, inst.npt, x, bins).items():
        assert abs(W[b] - Wo[0]) <= TOL64 * Wa[0], (b, W[b], Wo[0])
        assert abs(U[b] - Uo[0]) <= TOL64 * Uo[0], (b, U[b], Uo[0])
        assert abs(I[b] - Io[0]) <= TOL64 * Wa[0] / Uo[0], (b, I[b], Io[0])


def test_c2_full_split_full_size(dev):
    """Full pixel splitting (Section 4.2) of the 10-Mpixel frame in the
    default layout, as the benchmark times it: conservation over all bins,
    and three sampled bins against the oracle's polygon clipping of the
    pixels whose radial box reaches them."""
    say("c2 full split")
    az = azint()
    inst = synth.instance(synth.C2["n"], synth.C2["seed"])
    g = inst.geom
    plan = az.Plan(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), split="full", device=dev)
    x = inst.raw.reshape(-1).astype(np.float64)
    I, W, U = (a.cpu().numpy() for a in plan.integrate(torch.from_numpy(x).to(dev)))
    assert abs(U.sum() - g.npix) <= 1e-9 * g.npix
    assert abs(W.sum() - x.sum()) <= 1e-9 * x.sum()
    geo = (g.h, g.w, g.pixel_y, g.pixel_x, g.center_y, g.center_x, g.dist, g.wavelength)
    lo, hi, rc = oracle.pixel_extents(*geo, "r_m")
    pmin, pmax = oracle.default_range(lo, hi, rc, "full")
    corners = oracle.pixel_corners(*geo, "r_m")
    delta = (pmax - pmin) / inst.npt
    for b in (1, 700, 2900):
        say("  bin", b)
        sel = np.nonzero((hi >= pmin + (b - 1) * delta) & (lo <= pmin + (b + 2) * delta))[0]
        pix, bins, coef = oracle.full_entries(corners[sel], lo[sel], hi[sel], inst.npt, pmin,
                                              pmax)
        keep = bins == b
        xs = x[sel[pix[keep]]]
        Wo, Uo, Wa = (coef[keep] * xs).sum(), coef[keep].sum(), (coef[keep] * np.abs(xs)).sum()
        assert abs(W[b] - Wo) <= TOL64 * Wa, (b, W[b], Wo)
        assert abs(U[b] - Uo) <= TOL64 * Uo, (b, U[b], Uo)
        assert abs(I[b] - Wo / Uo) <= TOL64 * Wa / Uo, (b, I[b], Wo / Uo)


def _random_geometries(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        h, w = int(rng.integers(1, 260)), int(rng.integers(1, 260))
        # beam on the detector, on a pixel corner, or outside it
        kind = rng.integers(0, 3)
        if kind == 0:
            cy, cx = rng.uniform(0, h), rng.uniform(0, w)
        elif kind == 1:
            cy, cx = float(rng.integers(0, h + 1)), float(rng.integers(0, w + 1))
        else:
            cy, cx = rng.uniform(-h, 2 * h), rng.uniform(-w, 2 * w)
        npt = int(rng.integers(1, 400))
        split = ["bbox", "bbox", "full", "none"][int(rng.integers(0, 4))]
        unit = ["r_m", "r_m", "r_mm"][int(rng.integers(0, 3))]
        tile = int(rng.choice([64, 512, 4096, 16384]))
        block = int(rng.choice([128, 256]))
        out.append((h, w, cy, cx, npt, split, unit, tile, block))
    return out


@pytest.mark.parametrize("g", _random_geometries(24, 2024),
                         ids=lambda g: f"{g[0]}x{g[1]}-{g[5]}-{g[4]}-t{g[7]}b{g[8]}")
def test_run_layout_random_geometries(g, dev):
    """Seeded random detectors (sizes 1-259, the beam on, at a corner of or
    away from the detector, 1-399 bins, every split, radial units, several
    tilings) in the default run layout against the oracle, for a corrected
    image and for the raw pipeline with corrections."""
    h, w, cy, cx, npt, split, unit, tile, block = g
    say("random", g)
    az = azint()
    plan = az.Plan(h, w, npt, center=(cy, cx), split=split, unit=unit, device=dev,
                   tile_nnz=tile, block=block)
    assert plan.layout() == "run"
    m = oracle_matrix(h, w, cy, cx, npt, 1e-4, 1e-4, unit, split)
    rng = np.random.default_rng(h * 1000 + w)
    x = rng.uniform(-5.0, 100.0, size=h * w)
    check(plan.integrate(torch.from_numpy(x).to(dev), empty=-2.0), m, x, TOL64, empty=-2.0,
          what=str(g))
    raw = rng.integers(0, 1 << 16, size=h * w).astype(np.int32)
    dark = rng.integers(0, 50, size=h * w).astype(np.float64)
    flat = rng.uniform(0.9, 1.1, size=h * w)
    t = lambda a: torch.from_numpy(a).to(dev)
    plan.set_corrections(dark=t(dark), flat=t(flat))
    out = plan.integrate_raw(t(raw))
    torch.cuda.synchronize()
    check(out, m, oracle.correct(raw.astype(np.float64), dark, flat), TOL64, what=f"raw {g}")


@pytest.mark.parametrize("kind", ["1d", "2d", "1d-corrected"])
def test_plan_autotune(kind, dev):
    """The plan autotuner tries layouts and tilings on the plan's own image,
    keeps the fastest, reports every candidate, and the tuned plan still
    matches the oracle.  With corrections set, only tilings of the current
    layout are tried."""
    say("plan autotune", kind)
    az = azint()
    h, w, cy, cx = 200, 190, 95.2, 100.6
    na = 36 if kind == "2d" else None
    plan = az.Plan(h, w, 60 if na else 150, npt_azim=na, center=(cy, cx), device=dev)
    rng = np.random.default_rng(21)
    x = rng.uniform(0.0, 100.0, size=h * w)
    xt = torch.from_numpy(x).to(dev)
    start = plan.layout()
    if kind == "1d-corrected":
        plan.set_corrections(dark=torch.zeros(h * w, dtype=torch.float64, device=dev))
    rep = plan.autotune(xt)
    layouts = {c["layout"] for c in rep["candidates"]}
    assert len(rep["candidates"]) >= 3
    assert rep["best"]["ms"] == min(c["ms"] for c in rep["candidates"])
    assert plan.layout() == rep["best"]["layout"]
    assert plan.tiling()["tile_nnz"] == rep["best"]["tile_nnz"]
    if kind == "1d-corrected":
        assert layouts == {start}
    else:
        assert len(layouts) >= 2
    if na:
        m = oracle.build_matrix2d(h=h, w=w, pixel_y=1e-4, pixel_x=1e-4, center_y=cy,
                                  center_x=cx, dist=0.1, wavelength=1e-10, npt_rad=60,
                                  npt_azim=na, unit="r_m", split="bbox")
    else:
        m = oracle_matrix(h, w, cy, cx, 150)
    out = plan.integrate(xt, empty=-1.0)
    torch.cuda.synchronize()
    check(out, m, x, TOL64, empty=-1.0, what=f"tuned {kind}")
