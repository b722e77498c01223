"""Matrix-free (fused) layout vs the FP64 oracle and vs the stored-matrix
layouts (C-ABI calls).

The fused kernel recomputes the bounding-box coefficients from the geometry
per frame with the plan builder's operations, so its sums are the stored
matrix's sums in another order: equal to the band layout's within FP64
rounding, and to the oracle within the FP64 tolerance.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.helpers import azint, norm_err, oracle_matrix
from tests.test_gpu_forward import TOL32_F64, TOL32_SAME, TOL64, TOLK32, check

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


GEOMS = [
    # h, w, center_y, center_x, npt, unit, split, range
    (100, 100, 50.0, 50.0, 100, "r_m", "bbox", None),
    (37, 53, 10.25, 40.5, 61, "r_m", "bbox", None),
    (64, 48, -5.0, 70.0, 40, "r_m", "bbox", None),       # beam off the detector
    (31, 29, 15.5, 14.5, 300, "r_m", "bbox", None),      # windows wider than one pass
    (45, 45, 22.5, 22.5, 7, "r_m", "bbox", None),
    (50, 60, 25.0, 30.0, 37, "r_m", "bbox", (5e-4, 2.5e-3)),  # clipped range
    (50, 60, 25.3, 30.7, 37, "r_m", "none", None),
    (1, 1, 0.5, 0.5, 4, "r_m", "bbox", None),
    (1, 17, 0.5, 8.5, 5, "r_m", "bbox", None),
    (257, 263, 128.5, 131.5, 256, "r_m", "bbox", None),
    (40, 130, 20.0, -3.0, 200, "r_mm", "bbox", None),    # beam left of the detector
    (300, 200, 10.0, 190.0, 150, "2th_deg", "bbox", None),
    (90, 70, -10.0, 35.0, 80, "q_nm", "bbox", None),
]


@pytest.mark.parametrize("grid", [0, 64])
@pytest.mark.parametrize("g", GEOMS, ids=lambda g: f"{g[0]}x{g[1]}-{g[5]}-{g[6]}-{g[4]}")
def test_fused_f64(g, grid, dev):
    h, w, cy, cx, npt, unit, split, rng = g
    say("fused f64", g, grid)
    az = azint()
    plan = az.Plan(h, w, npt, center=(cy, cx), unit=unit, split=split, range=rng,
                   layout="fused", device=dev, grid=grid)
    band = az.Plan(h, w, npt, center=(cy, cx), unit=unit, split=split, range=rng, device=dev)
    m = oracle_matrix(h, w, cy, cx, npt, 1e-4, 1e-4, unit, split, rng)
    x = np.random.default_rng(h * w + npt).uniform(-2.0, 1000.0, size=h * w)
    xt = torch.from_numpy(x).to(dev)
    out = plan.integrate(xt, empty=-1.5)
    ref = band.integrate(xt, empty=-1.5)
    again = plan.integrate(xt, empty=-1.5)
    torch.cuda.synchronize()
    check(out, m, x, TOL64, empty=-1.5, what=str(g))
    for a, b in zip(out, again):
        assert torch.equal(a, b)
    # the band layout sums the same coefficients in another order
    _, Wabs, Ub = oracle.integrate(m, np.abs(x))
    assert norm_err(out[1].cpu().numpy(), ref[1].cpu().numpy(), Wabs) <= 2 * TOL64
    assert norm_err(out[2].cpu().numpy(), ref[2].cpu().numpy(), Ub) <= 2 * TOL64


@pytest.mark.parametrize("accum", ["f64", "kahan32"])
def test_fused_f32(accum, dev):
    h, w, cy, cx, npt = 150, 170, 70.3, 85.9, 120
    say("fused f32", accum)
    az = azint()
    plan = az.Plan(h, w, npt, center=(cy, cx), dtype=torch.float32, accum=accum,
                   layout="fused", device=dev)
    m = oracle_matrix(h, w, cy, cx, npt)
    x = np.random.default_rng(9).uniform(0.0, 1000.0, size=h * w).astype(np.float32)
    out = plan.integrate(torch.from_numpy(x).to(dev))
    torch.cuda.synchronize()
    x64 = x.astype(np.float64)
    m32 = dict(m, data=m["data"].astype(np.float32).astype(np.float64),
               coef=m["coef"].astype(np.float32).astype(np.float64))
    check(out, m32, x64, TOL32_SAME if accum == "f64" else TOLK32, what="f32 same inputs")
    check(out, m, x64, TOL32_F64, what="f32 vs f64 oracle")


@pytest.mark.parametrize("raw_dtype", [np.int32, np.uint16, np.float64])
def test_fused_raw_pipeline_one_kernel(raw_dtype, dev):
    """Cast, correction and integration in the one fused kernel."""
    h, w, cy, cx, npt = 200, 190, 95.2, 100.6, 150
    say("fused raw", raw_dtype)
    az = azint()
    rng = np.random.default_rng(10)
    raw = rng.integers(0, 1 << 16, size=h * w).astype(raw_dtype)
    dark = rng.integers(0, 64, size=h * w).astype(np.float64)
    flat = rng.uniform(0.95, 1.05, size=h * w)
    solid = rng.uniform(0.9, 1.0, size=h * w)
    polar = rng.uniform(0.5, 1.0, size=h * w)
    t = lambda a: torch.from_numpy(a).to(dev)
    plan = az.Plan(h, w, npt, center=(cy, cx), layout="fused", device=dev)
    plan.set_corrections(dark=t(dark), flat=t(flat), solid=t(solid), polar=t(polar))
    band = az.Plan(h, w, npt, center=(cy, cx), device=dev)
    band.set_corrections(dark=t(dark), flat=t(flat), solid=t(solid), polar=t(polar))
    out = plan.integrate_raw(t(raw))
    staged = (plan.stage(t(raw)), plan.integrate_staged())[1]
    ref = band.integrate_raw(t(raw))
    torch.cuda.synchronize()
    m = oracle_matrix(h, w, cy, cx, npt)
    xc = oracle.correct(raw.astype(np.float64), dark, flat, solid, polar)
    check(out, m, xc, TOL64, what="fused raw")
    check(staged, m, xc, TOL64, what="fused staged")
    check(ref, m, xc, TOL64, what="band raw")


def test_fused_backward_and_errors(dev):
    az = azint()
    h, w, npt = 80, 90, 60
    plan = az.Plan(h, w, npt, layout="fused", device=dev)
    m = oracle_matrix(h, w, h / 2, w / 2, npt)
    rng = np.random.default_rng(11)
    x = rng.uniform(0, 1, size=h * w)
    g = rng.standard_normal(npt)
    t = lambda a: torch.from_numpy(a).to(dev)
    _, _, U = plan.integrate(t(x))
    gx = plan.backward(U, t(g)).cpu().numpy()
    _, _, Uo = oracle.integrate(m, x)
    ref = oracle.integrate_vjp(m, Uo, g, None)
    assert norm_err(gx, ref, oracle.integrate_vjp(m, Uo, np.abs(g), None)) <= 1e-12
    full = az.Plan(20, 20, 10, split="full")
    with pytest.raises(az.AzintError):
        full.set_layout("fused")
    two = az.Plan(20, 20, 10, npt_azim=8)
    with pytest.raises(az.AzintError):
        two.set_layout("fused")
    with pytest.raises(az.AzintError):
        az.Batch([az.Plan(10, 10, 5, layout="fused")], device=dev)


def test_fused_c2_full_size(dev):
    """The 10-Mpixel workload in float64, the configuration the benchmark
    times: sampled bins against the oracle (one by one), every bin against
    the band layout's sums of the same coefficients, and conservation."""
    from tests.test_gpu_forward import _sampled_bins_oracle
    say("fused c2")
    az = azint()
    inst = synth.instance(synth.C2["n"], synth.C2["seed"])
    g = inst.geom
    plan = az.Plan(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), layout="fused",
                   device=dev)
    band = az.Plan(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), device=dev)
    x = inst.raw.reshape(-1).astype(np.float64)
    xt = torch.from_numpy(x).to(dev)
    I, W, U = (a.cpu().numpy() for a in plan.integrate(xt))
    Ib, Wb, Ub = (a.cpu().numpy() for a in band.integrate(xt))
    assert np.all(np.abs(U - Ub) <= 2 * TOL64 * Ub)
    assert np.all(np.abs(W - Wb) <= 2 * TOL64 * np.abs(Wb))
    assert abs(U.sum() - g.npix) <= 1e-12 * g.npix
    assert abs(W.sum() - x.sum()) <= 1e-12 * x.sum()
    bins = np.unique(np.r_[0, 1, inst.npt - 1, np.random.default_rng(1).choice(inst.npt, 13,
                                                                                  replace=False)])
    for b, ((Io, Wo, Uo), (_, Wa, _)) in _sampled_bins_oracle(g, inst.npt, x, bins).items():
        assert abs(W[b] - Wo[0]) <= TOL64 * Wa[0], (b, W[b], Wo[0])
        assert abs(U[b] - Uo[0]) <= TOL64 * Uo[0], (b, U[b], Uo[0])
        assert abs(I[b] - Io[0]) <= TOL64 * Wa[0] / Uo[0], (b, I[b], Io[0])


@pytest.mark.parametrize("layout", ["fused", "pixel"])
def test_plan_graph_replays(layout, dev):
    """The raw pipeline captured in a HIP graph (the fused layout's one
    kernel, and a 2-D plan in its default layout for the pixel case)
    replays the eager bits every time, with eager work in between."""
    say("plan graph", layout)
    az = azint()
    rng = np.random.default_rng(14)
    h, w = 160, 150
    raw = torch.from_numpy(rng.integers(0, 1 << 20, size=h * w).astype(np.int32)).to(dev)
    dark = torch.from_numpy(rng.integers(0, 64, size=h * w).astype(np.float64)).to(dev)
    if layout == "fused":
        plan = az.Plan(h, w, 120, layout="fused", device=dev)
    else:
        plan = az.Plan(h, w, 60, npt_azim=36, device=dev)
    plan.set_corrections(dark=dark)
    I0, W0, U0 = plan.integrate_raw(raw)
    I, W, U = (torch.full_like(I0, np.nan) for _ in range(3))
    graph = plan.graph(raw, I, W, U)
    for rep in range(4):
        for t in (I, W, U):
            t.fill_(np.nan)
        graph.launch()
        torch.cuda.synchronize()
        assert torch.equal(I, I0) and torch.equal(W, W0) and torch.equal(U, U0), rep
        _ = (raw * 2).sum().item()
