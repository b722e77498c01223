"""Two-dimensional integration on the GPU vs the FP64 oracle (C-ABI calls).

The per-frame kernels are the one-dimensional ones run over a matrix whose
rows are (azimuthal wedge, radial bin) pairs; these tests check every device
layout, the raw pipeline with corrections, the adjoint and batches on such
matrices, and at the 10-Mpixel detector size the properties that hold at any
size (conservation, and the azimuthal marginal equal to the 1-D profile).
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.helpers import azint, norm_err
from tests.test_gpu_forward import TOL32_F64, TOL64, check

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle2d(h, w, cy, cx, nr, na, unit="r_m", split="bbox"):
    return oracle.build_matrix2d(h=h, w=w, pixel_y=1e-4, pixel_x=1e-4, center_y=cy,
                                 center_x=cx, dist=0.1, wavelength=1e-10, npt_rad=nr,
                                 npt_azim=na, unit=unit, split=split)


GEOMS = [
    # h, w, center_y, center_x, npt_rad, npt_azim, unit, split
    (120, 130, 60.2, 64.9, 60, 36, "r_m", "bbox"),
    (128, 128, 64.0, 64.0, 64, 360, "r_m", "bbox"),    # beam on a pixel corner
    (100, 90, -20.0, 45.0, 50, 72, "r_m", "bbox"),     # beam above the detector
    (64, 64, 32.5, 140.0, 30, 360, "r_m", "bbox"),     # rows across the +-pi cut
    (96, 80, 40.3, 39.6, 40, 90, "2th_deg", "bbox"),
    (120, 130, 60.2, 64.9, 60, 36, "r_m", "none"),
    (100, 110, 50.4, 55.1, 45, 24, "r_m", "full"),
    (64, 64, 32.5, 140.0, 30, 360, "q_nm", "full"),
    (1, 17, 0.5, 8.5, 5, 4, "r_m", "bbox"),
]
SLIVER = 1e-12


def check_slivers(out, m, x, tol, empty, what):
    """As check(), for units where a library transcendental (atan, sin) may
    differ from the oracle's by an ulp: a corner within an ulp of a bin edge
    can then leave a sliver of area (U <= 1e-12) in a bin the oracle leaves
    empty, or the reverse.  Such bins must hold only that sliver; every other
    bin is compared to the FP64 tolerance."""
    I, W, U = (t.double().cpu().numpy() for t in out)
    Io, Wo, Uo = oracle.integrate(m, x, empty=empty)
    _, Wabs, _ = oracle.integrate(m, np.abs(x))
    thin = (Uo <= SLIVER) | (U <= SLIVER)
    assert np.all(np.abs(U[thin] - Uo[thin]) <= SLIVER), what
    assert np.all(np.abs(W[thin] - Wo[thin]) <= SLIVER * np.abs(x).max()), what
    keep = ~thin
    sI = Wabs[keep] / Uo[keep]
    assert norm_err(I[keep], Io[keep], sI) <= tol, what
    assert norm_err(W[keep], Wo[keep], Wabs[keep]) <= tol, what
    assert norm_err(U[keep], Uo[keep], Uo[keep]) <= tol, what
    assert np.all(I[(U == 0)] == empty), what


TILINGS = [dict(), dict(tile_nnz=256, block=64, variant=0, band=1),
           dict(tile_nnz=4096, block=512, variant=6, grid=128, band=8),
           dict(tile_nnz=0, band=16)]


@pytest.mark.parametrize("layout", ["band", "tile", "ring", "pixel", "run"])
@pytest.mark.parametrize("tiling", range(len(TILINGS)))
@pytest.mark.parametrize("g", GEOMS, ids=lambda g: f"{g[0]}x{g[1]}-{g[7]}-{g[6]}-{g[5]}")
def test_forward2d_f64(g, tiling, layout, dev):
    h, w, cy, cx, nr, na, unit, split = g
    say("2d forward f64", g, tiling, layout)
    az = azint()
    plan = az.Plan(h, w, nr, npt_azim=na, center=(cy, cx), unit=unit, split=split,
                   layout=layout, device=dev, **TILINGS[tiling])
    m = oracle2d(h, w, cy, cx, nr, na, unit, split)
    x = np.random.default_rng(h * w + na).uniform(-2.0, 1000.0, size=h * w)
    out = plan.integrate(torch.from_numpy(x).to(dev), empty=-1.5)
    torch.cuda.synchronize()
    if unit in ("r_m", "r_mm"):
        check(out, m, x, TOL64, empty=-1.5, what=str(g))
    else:
        check_slivers(out, m, x, TOL64, -1.5, str(g))


def test_forward2d_f32_and_raw_pipeline(dev):
    """float32 storage (FP64 accumulation) against the FP64 oracle, and the
    raw-frame pipeline with dark / flat / solid-angle / polarisation."""
    h, w, cy, cx, nr, na = 150, 140, 70.3, 75.8, 70, 90
    say("2d f32 + raw", h, w, nr, na)
    az = azint()
    m = oracle2d(h, w, cy, cx, nr, na)
    rng = np.random.default_rng(11)
    x = rng.uniform(0.0, 1000.0, size=h * w)
    p32 = az.Plan(h, w, nr, npt_azim=na, center=(cy, cx), dtype=torch.float32, device=dev)
    out = p32.integrate(torch.from_numpy(x.astype(np.float32)).to(dev))
    torch.cuda.synchronize()
    check(out, m, x, TOL32_F64, what="f32")

    raw = rng.integers(0, 1 << 20, size=h * w).astype(np.int32)
    dark = rng.integers(0, 64, size=h * w).astype(np.float64)
    flat = rng.uniform(0.95, 1.05, size=h * w)
    solid = rng.uniform(0.9, 1.0, size=h * w)
    polar = rng.uniform(0.5, 1.0, size=h * w)
    p64 = az.Plan(h, w, nr, npt_azim=na, center=(cy, cx), device=dev)
    t = lambda a: torch.from_numpy(a).to(dev)
    p64.set_corrections(dark=t(dark), flat=t(flat), solid=t(solid), polar=t(polar))
    out = p64.integrate_raw(t(raw))
    torch.cuda.synchronize()
    xc = oracle.correct(raw.astype(np.float64), dark, flat, solid, polar)
    check(out, m, xc, TOL64, what="raw")


def test_backward2d_vs_oracle(dev):
    h, w, cy, cx, nr, na = 90, 100, 44.6, 50.2, 40, 72
    say("2d backward", h, w, nr, na)
    az = azint()
    plan = az.Plan(h, w, nr, npt_azim=na, center=(cy, cx), device=dev)
    m = oracle2d(h, w, cy, cx, nr, na)
    rng = np.random.default_rng(12)
    x = rng.uniform(0, 1, size=h * w)
    gI = rng.standard_normal(nr * na)
    gW = rng.standard_normal(nr * na)
    _, _, U = oracle.integrate(m, x)
    t = lambda a: torch.from_numpy(a).to(dev)
    _, _, Ud = plan.integrate(t(x))
    gx = plan.backward(Ud, t(gI), t(gW)).cpu().numpy()
    ref = oracle.integrate_vjp(m, U, gI, gW)
    scale = oracle.integrate_vjp(m, U, np.abs(gI), np.abs(gW))
    assert norm_err(gx, ref, scale) <= 1e-12


@pytest.mark.parametrize("layout", ["band", "tile", "ring"])
def test_batch2d_equals_plans_and_oracle(layout, dev):
    """Uneven two-dimensional instances in one batch: bitwise equal to the
    plan-by-plan results and within tolerance of the oracle."""
    say("2d batch", layout)
    az = azint()
    shapes = [(40, 50, 20.1, 24.7, 20, 36), (64, 30, 10.0, 29.0, 35, 8),
              (7, 9, 3.5, 4.5, 5, 4), (100, 100, 49.2, 50.9, 50, 360)]
    plans = [az.Plan(h, w, nr, npt_azim=na, center=(cy, cx), layout=layout)
             for (h, w, cy, cx, nr, na) in shapes]
    batch = az.Batch(plans, device=dev)
    rng = np.random.default_rng(13)
    xs = [rng.uniform(0, 100, size=h * w) for (h, w, *_r) in shapes]
    I, W, U = batch.forward(torch.from_numpy(np.concatenate(xs)).to(dev))
    torch.cuda.synchronize()
    off = 0
    for plan, s, x in zip(plans, shapes, xs):
        plan.upload(dev)
        out = plan.integrate(torch.from_numpy(x).to(dev))
        n = plan.npt
        for a, b in zip((I, W, U), out):
            assert torch.equal(a[off:off + n], b)
        check(out, oracle2d(*s), x, TOL64, what=str(s))
        off += n


def test_c2_detector_2d_properties(dev):
    """The 10-Mpixel detector (3162 x 3163) in 1000 radial bins x 360 wedges:
    every pixel is conserved (sum U = npix, sum W = sum x), and summing the
    map over the wedges gives the 1-D profile of the same image within FP64
    rounding (the 1-D path is checked against the oracle at this size)."""
    say("c2 2d properties")
    az = azint()
    inst = synth.instance(synth.C2["n"], synth.C2["seed"])
    g = inst.geom
    nr, na = 1000, 360
    p2 = az.Plan(g.h, g.w, nr, npt_azim=na, center=(g.center_y, g.center_x), device=dev)
    p1 = az.Plan(g.h, g.w, nr, center=(g.center_y, g.center_x), device=dev)
    x = torch.from_numpy(inst.raw.reshape(-1).astype(np.float64)).to(dev)
    I2, W2, U2 = p2.integrate(x)
    I1, W1, U1 = p1.integrate(x)
    torch.cuda.synchronize()
    W2 = W2.cpu().numpy().reshape(na, nr)
    U2 = U2.cpu().numpy().reshape(na, nr)
    W1, U1 = W1.cpu().numpy(), U1.cpu().numpy()
    xs = float(x.sum().item())
    assert abs(U2.sum() - g.h * g.w) <= 1e-9 * g.h * g.w
    assert abs(W2.sum() - xs) <= 1e-9 * xs
    assert np.abs(U2.sum(axis=0) - U1).max() <= 1e-9 * U1.max()
    assert np.abs(W2.sum(axis=0) - W1).max() <= 1e-9 * W1.max()
    I2 = I2.cpu().numpy().reshape(na, nr)
    assert np.all(np.isfinite(I2)) and np.all(I2[U2 == 0] == 0)
