"""Device plan builder vs the host plan builder and the FP64 oracle.

The device builder computes per-pixel extents and entries with the same IEEE
operations as the host builder and orders them with a stable radix sort, so
its matrix must equal the host builder's bit for bit wherever every step is
correctly rounded (radius units, bounding box or no split), and to rounding
where a library transcendental (atan2, atan, sin) enters.
"""
import sys
import time

import numpy as np
import pytest
import torch

import synth
from tests.helpers import azint, oracle_matrix
from tests.test_gpu_forward import TOL64, check

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dense(csr, shape):
    import scipy.sparse as sp
    return sp.csr_matrix(csr, shape=shape).toarray()


GEOMS = [
    # h, w, center_y, center_x, npt, unit, split, range, dtype
    (100, 100, 50.0, 50.0, 100, "r_m", "bbox", None, "f64"),
    (37, 53, 10.25, 40.5, 61, "r_m", "bbox", None, "f64"),
    (64, 48, -5.0, 70.0, 40, "r_mm", "bbox", None, "f32"),
    (31, 29, 15.5, 14.5, 300, "r_m", "bbox", None, "f64"),     # bins finer than pixels
    (50, 60, 25.0, 30.0, 37, "r_m", "bbox", (5e-4, 2.5e-3), "f64"),  # clipped range
    (50, 60, 25.3, 30.7, 37, "r_m", "none", None, "f64"),
    (1, 1, 0.5, 0.5, 4, "r_m", "bbox", None, "f64"),
    (1, 17, 0.5, 8.5, 5, "r_m", "bbox", None, "f32"),
    (20, 20, 10.0, 10.0, 1, "r_m", "bbox", None, "f64"),       # one bin
    (257, 263, 128.5, 131.5, 256, "r_m", "bbox", None, "f64"),
    (120, 130, 60.2, 64.9, 140, "r_m", "full", None, "f64"),
    (300, 200, 10.0, 190.0, 150, "2th_deg", "bbox", None, "f64"),
    (90, 70, -10.0, 35.0, 80, "q_nm", "full", None, "f64"),
]
EXACT = lambda g: g[5] in ("r_m", "r_mm") and g[6] in ("bbox", "none")


@pytest.mark.parametrize("g", GEOMS, ids=lambda g: f"{g[0]}x{g[1]}-{g[5]}-{g[6]}-{g[4]}-{g[8]}")
def test_device_plan_equals_host_plan(g, dev):
    h, w, cy, cx, npt, unit, split, rng, dt = g
    say("device build", g)
    az = azint()
    dtype = torch.float64 if dt == "f64" else torch.float32
    kw = dict(center=(cy, cx), unit=unit, split=split, range=rng, dtype=dtype)
    hp = az.Plan(h, w, npt, layout="band", band=4, **kw)   # the device builder's layout
    dp = az.Plan.on_device(h, w, npt, device=dev, **kw)
    ih, idv = hp.info(), dp.info()
    assert idv["npt"] == npt and idv["npix"] == h * w
    assert idv["range"] == ih["range"] or not EXACT(g)
    dh, dd = hp.export_csr(), dp.export_csr()
    ch, cd = hp.export_csc(), dp.export_csc()
    if EXACT(g):
        for a, b in zip(dh + ch, dd + cd):
            assert np.array_equal(a, b)
    else:
        A = dense(dh, (npt, h * w))
        B = dense(dd, (npt, h * w))
        assert np.abs(A - B).max() <= (1e-13 if unit == "r_m" else 1e-9)
    # the device-built plan integrates like the oracle (and, where the
    # matrices are equal, bitwise like the host-built plan in the same layout)
    x = np.random.default_rng(h * w).uniform(-2.0, 1000.0, size=h * w)
    xt = torch.from_numpy(x.astype(np.float64 if dt == "f64" else np.float32)).to(dev)
    hp.upload(dev)
    out_d = dp.integrate(xt, empty=-1.5)
    out_h = hp.integrate(xt, empty=-1.5)
    torch.cuda.synchronize()
    if EXACT(g):
        for a, b in zip(out_d, out_h):
            assert torch.equal(a, b)
    if dt == "f64" and unit == "r_m":
        check(out_d, oracle_matrix(h, w, cy, cx, npt, 1e-4, 1e-4, unit, split, rng), x, TOL64,
              empty=-1.5, what=str(g))


def test_device_plan_layout_switch_and_backward(dev):
    """A device-built plan switched to the other layouts (through its host
    copy) and differentiated gives the host-built plan's results."""
    say("device build layouts")
    az = azint()
    h, w, npt = 150, 170, 120
    dp = az.Plan.on_device(h, w, npt, device=dev)
    hp = az.Plan(h, w, npt, band=4, device=dev)   # the device-built plan's tiling
    x = torch.from_numpy(np.random.default_rng(5).uniform(0, 10, size=h * w)).to(dev)
    for layout in ("pixel", "ring", "tile", "band", "run"):
        dp.set_layout(layout)
        hp.set_layout(layout)
        a, b = dp.integrate(x), hp.integrate(x)
        torch.cuda.synchronize()
        for u, v in zip(a, b):
            assert torch.equal(u, v), layout
    g = torch.from_numpy(np.random.default_rng(6).standard_normal(npt)).to(dev)
    _, _, U = dp.integrate(x)
    assert torch.equal(dp.backward(U, g), hp.backward(U, g))


def test_device_plan_c2_size(dev):
    """The 10-Mpixel detector: the device builder reproduces the host
    builder's matrix bit for bit; both build times are printed."""
    say("device build c2")
    az = azint()
    inst = synth.instance(synth.C2["n"], synth.C2["seed"])
    g = inst.geom
    t0 = time.perf_counter()
    hp = az.Plan(g.h, g.w, inst.npt, center=(g.center_y, g.center_x))
    t1 = time.perf_counter()
    dp = az.Plan.on_device(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), device=dev)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    say(f"host build {t1 - t0:.3f} s, device build {t2 - t1:.3f} s")
    for a, b in zip(hp.export_csr() + hp.export_csc(), dp.export_csr() + dp.export_csc()):
        assert np.array_equal(a, b)


GEOMS2D = [
    # h, w, center_y, center_x, npt_rad, npt_azim, unit, split, dtype
    (100, 100, 50.0, 50.0, 40, 36, "r_m", "bbox", "f64"),
    (64, 48, -5.0, 70.0, 30, 8, "r_m", "bbox", "f64"),       # beam off the detector
    (37, 53, 10.25, 40.5, 25, 12, "r_m", "none", "f64"),
    (120, 130, 60.2, 64.9, 50, 24, "r_m", "full", "f64"),
    (90, 70, -10.0, 35.0, 40, 16, "q_nm", "full", "f64"),
    (31, 29, 15.5, 14.5, 20, 2, "r_m", "bbox", "f32"),       # two wedges: raw wedges tie
    (45, 45, 22.5, 22.5, 15, 3, "2th_deg", "bbox", "f64"),
    (1, 17, 0.5, 8.5, 5, 4, "r_mm", "bbox", "f64"),
]


@pytest.mark.parametrize("g", GEOMS2D, ids=lambda g: f"{g[0]}x{g[1]}-{g[6]}-{g[7]}-{g[4]}x{g[5]}")
def test_device_plan2d_matches_host_and_oracle(g, dev):
    """Two-dimensional plans built on the device: the same rows and
    coefficients as the host builder up to the device atan2's last bits (a
    wedge-edge coefficient to rounding, a sliver entry of a few ulps that one
    side keeps and the other does not), and integration like the oracle."""
    h, w, cy, cx, nr, na, unit, split, dt = g
    say("device build 2d", g)
    az = azint()
    dtype = torch.float64 if dt == "f64" else torch.float32
    kw = dict(npt_azim=na, center=(cy, cx), unit=unit, split=split, dtype=dtype)
    hp = az.Plan(h, w, nr, device=dev, **kw)
    dp = az.Plan.on_device(h, w, nr, device=dev, **kw)
    assert dp.shape() == hp.shape() == (nr, na)
    assert dp.layout() == "pixel"
    ih, idv = hp.info(), dp.info()
    assert idv["npt"] == nr * na and idv["npix"] == h * w
    if unit in ("r_m", "r_mm"):
        assert idv["range"] == ih["range"]
    dh, dd = hp.export_csr(), dp.export_csr()
    A = dense(dh, (nr * na, h * w))
    B = dense(dd, (nr * na, h * w))
    tol = 1e-12 if unit in ("r_m", "r_mm") else 1e-9
    assert np.abs(A - B).max() <= tol
    # entries on one side only are slivers
    only = (A != 0) ^ (B != 0)
    assert np.abs(A[only]).max(initial=0.0) <= tol and np.abs(B[only]).max(initial=0.0) <= tol
    # entries both keep agree to rounding, absolutely (a share cut close to
    # a wedge edge is the difference of nearby values, so its relative error
    # is larger); bit for bit where no corner's atan2 differs
    both = (A != 0) & (B != 0)
    say(f"entries bit-equal: {(A[both] == B[both]).mean():.4f}, one side only: {only.sum()}")
    # per-pixel entries stay in ascending rows (the CSC export)
    _, rows, colptr = dp.export_csc()
    for p in range(h * w):
        r = rows[colptr[p]:colptr[p + 1]]
        assert np.all(np.diff(r) >= 0), p
    # integration: like the oracle (the host-built plan is checked against
    # it elsewhere), and like the host-built plan
    m = az_oracle2d(h, w, cy, cx, nr, na, unit, split)
    x = np.random.default_rng(h * w + na).uniform(-2.0, 1000.0, size=h * w)
    xt = torch.from_numpy(x.astype(np.float64 if dt == "f64" else np.float32)).to(dev)
    out = dp.integrate(xt, empty=-1.5)
    torch.cuda.synchronize()
    tolI = TOL64 if dt == "f64" else 1e-6
    xo = x if dt == "f64" else x.astype(np.float32).astype(np.float64)
    if unit in ("r_m", "r_mm") and split != "full":
        check(out, m, xo, tolI, empty=-1.5, what=str(g))
    else:
        # full splitting clips the quadrilateral by the wedges in differences
        # of corner azimuths (~1e-3 rad across a pixel) taken from atan2
        # values of order 1, and 2theta / q pass through atan and sin: an ulp
        # of the device functions against the C library's moves a coefficient
        # by up to ~1e-12 relative and can add or drop a sliver entry (which
        # can turn an empty bin into a non-empty one).  The matrix is held to
        # the host builder's above; the integration is checked against the
        # oracle's sums over the device-built matrix itself.
        data, idx, ptr = dd
        md = dict(npt=nr * na, pix=idx.astype(np.int64),
                  bins=np.repeat(np.arange(nr * na), np.diff(ptr)),
                  coef=data.astype(np.float64))
        check(out, md, xo, tolI, empty=-1.5, what=str(g))


def az_oracle2d(h, w, cy, cx, nr, na, unit, split):
    import oracle
    return oracle.build_matrix2d(h=h, w=w, pixel_y=1e-4, pixel_x=1e-4, center_y=cy, center_x=cx,
                                 dist=0.1, wavelength=1e-10, npt_rad=nr, npt_azim=na, unit=unit,
                                 split=split)


def test_device_plan2d_c2_size(dev):
    """The 10-Mpixel detector in 1000 x 360 bins: the device-built plan
    integrates like the host-built one and both build times are printed.
    Every coefficient of the two plans agrees to 1e-12 absolutely (the small
    cases above), so a bin's U and W may differ by 1e-12 per entry of the bin
    (times the largest pixel value for W): relatively more than the FP64
    tolerance in bins near the beam, whose U is a few small shares."""
    say("device build 2d c2")
    az = azint()
    inst = synth.instance(synth.C2["n"], synth.C2["seed"])
    g = inst.geom
    t0 = time.perf_counter()
    hp = az.Plan(g.h, g.w, 1000, npt_azim=360, center=(g.center_y, g.center_x), device=dev)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dp = az.Plan.on_device(g.h, g.w, 1000, npt_azim=360, center=(g.center_y, g.center_x),
                           device=dev)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    say(f"2-D host build + upload {t1 - t0:.3f} s, device build {t2 - t1:.3f} s, "
        f"nnz host {hp.nnz} device {dp.nnz}")
    assert abs(dp.nnz - hp.nnz) <= 1e-4 * hp.nnz
    x = torch.from_numpy(inst.raw.reshape(-1).astype(np.float64)).to(dev)
    Ih, Wh, Uh = (a.cpu().numpy() for a in hp.integrate(x))
    Id, Wd, Ud = (a.cpu().numpy() for a in dp.integrate(x))
    torch.cuda.synchronize()
    nb = np.diff(hp.export_csr()[2]).astype(np.float64)
    xmax = float(inst.raw.max())
    nz = Uh > 0
    assert np.array_equal(nz, Ud > 0)
    assert np.all(np.abs(Ud - Uh) <= 1e-12 * nb)
    assert np.all(np.abs(Wd - Wh) <= 1e-12 * nb * xmax)
    # bins away from the beam (U of at least one whole pixel share) agree
    # to the FP64 tolerance
    big = Uh >= 1.0
    assert big.sum() > 100_000
    assert np.max(np.abs(Ud - Uh)[big] / Uh[big]) <= TOL64
    say(f"largest relative U difference {np.max(np.abs(Ud - Uh)[nz] / Uh[nz]):.2e}")
