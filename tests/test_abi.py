"""C-ABI library on the CPU: exports, host plan builder vs the oracle, tile
schedule, argument errors.  No kernel runs here."""
import ctypes
import os
import re

import numpy as np
import pytest
import torch

import oracle
from tests.helpers import ROOT, azint, oracle_matrix

HEADER = os.path.join(ROOT, "include", "azint.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(azi_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    az = azint()
    L = ctypes.CDLL(az.LIB_PATH)
    names = declared_symbols()
    assert len(names) >= 30
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # the Python binding declares a signature for every one of them
    assert set(names) == set(az._SIGS), set(names) ^ set(az._SIGS)
    assert az.lib().azi_version() == 1


GEOMS = [
    # h, w, center_y, center_x, npt, pixel(y, x), unit, split, range
    (100, 100, 50.0, 50.0, 100, (1e-4, 1e-4), "r_m", "bbox", None),
    (37, 53, 10.25, 40.5, 61, (1e-4, 1e-4), "r_m", "bbox", None),
    (64, 48, -5.0, 70.0, 40, (1.5e-4, 1e-4), "r_m", "bbox", None),
    (31, 29, 15.5, 14.5, 300, (1e-4, 1e-4), "r_m", "bbox", None),    # bins finer than pixels
    (45, 45, 22.5, 22.5, 7, (1e-4, 1e-4), "r_m", "bbox", None),      # wide bins
    (50, 60, 25.0, 30.0, 37, (1e-4, 1e-4), "r_m", "bbox", (5e-4, 2.5e-3)),  # clipped range
    (50, 60, 25.3, 30.7, 37, (1e-4, 1e-4), "r_m", "none", None),
    (33, 20, 3.0, 2.0, 25, (1e-4, 1e-4), "r_mm", "bbox", None),
    (1, 1, 0.5, 0.5, 4, (1e-4, 1e-4), "r_m", "bbox", None),          # one pixel
    (1, 17, 0.5, 8.5, 5, (1e-4, 1e-4), "r_m", "bbox", None),         # one row
]


@pytest.mark.parametrize("g", GEOMS, ids=lambda g: f"{g[0]}x{g[1]}-{g[6]}-{g[7]}-{g[4]}")
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_plan_matrix_bit_exact_vs_oracle(g, dtype):
    h, w, cy, cx, npt, (py, px), unit, split, rng = g
    az = azint()
    plan = az.Plan(h, w, npt, pixel=(py, px), center=(cy, cx), unit=unit, split=split,
                   range=rng, dtype=dtype)
    m = oracle_matrix(h, w, cy, cx, npt, py, px, unit, split, rng)
    info = plan.info()
    assert info["npt"] == npt and info["npix"] == h * w and info["nnz"] == m["data"].size
    assert info["range"] == (m["pmin"], m["pmax"])
    data, indices, indptr = plan.export_csr()
    assert np.array_equal(indptr, m["indptr"])
    assert np.array_equal(indices, m["indices"])
    ref = m["data"] if dtype == torch.float64 else m["data"].astype(np.float32)
    assert np.array_equal(data, ref)
    cdata, bins, colptr = plan.export_csc()
    order = np.lexsort((m["bins"], m["pix"]))
    assert np.array_equal(bins, m["bins"][order])
    assert np.array_equal(cdata, m["coef"][order].astype(data.dtype))
    assert np.array_equal(colptr, np.r_[0, np.cumsum(np.bincount(m["pix"], minlength=h * w))])
    assert np.array_equal(plan.positions(), oracle.positions(npt, m["pmin"], m["pmax"]))


@pytest.mark.parametrize("unit", ["2th_deg", "2th_rad", "q_nm"])
def test_transcendental_units_match_up_to_edges(unit):
    """With atan/sin the host libm and numpy may round a value 1 ulp apart;
    then a pixel edge lying on a bin edge may move by one bin.  Everything
    else matches exactly."""
    az = azint()
    h, w, npt = 80, 70, 90
    plan = az.Plan(h, w, npt, center=(40.0, 35.0), unit=unit)
    m = oracle_matrix(h, w, 40.0, 35.0, npt, 1e-4, 1e-4, unit, "bbox", None)
    lo_r, hi_r = plan.info()["range"]
    assert abs(lo_r - m["pmin"]) <= 2 * np.spacing(abs(m["pmin"]) + 1e-300)
    assert abs(hi_r - m["pmax"]) <= 2 * np.spacing(m["pmax"])
    data, indices, indptr = plan.export_csr()
    import scipy.sparse as sp
    A = sp.csr_matrix((data, indices, indptr), shape=(npt, h * w)).toarray()
    B = sp.csr_matrix((m["data"], m["indices"], m["indptr"]), shape=(npt, h * w)).toarray()
    assert np.abs(A - B).max() <= 1e-9


def _piece_cut(a, b, k, pieces):
    if k <= 0:
        return a
    if k >= pieces:
        return b
    return max(a, (a + ((b - a) * k) // pieces) & ~3)


@pytest.mark.parametrize("tile_nnz,band", [(64, 1), (256, 16), (1024, 16), (1024, 1),
                                           (2048, 3), (8192, 16), (2048, 64), (512, 4)])
def test_tile_schedule_covers_every_nonzero_once(tile_nnz, band):
    """Every nonzero lands in exactly one tile, every row is written exactly
    once (directly or by the fix-up of its pieces), every partial slot is
    filled exactly once."""
    az = azint()
    plan = az.Plan(300, 280, 250, center=(150.2, 139.7))
    _, _, indptr = plan.export_csr()
    nnz = int(indptr[-1])
    tiles, splits = plan.tile_schedule(tile_nnz=tile_nnz, band=band)
    covered = np.zeros(nnz, dtype=np.int64)
    rows = np.zeros(plan.npt, dtype=np.int64)
    slots = {}
    for r0, r1, z0, z1, part, ip0, mode, k in tiles.tolist():
        assert r1 > r0 and ip0 == r0
        if mode == 0:      # one row or a piece of one
            assert r1 == r0 + 1 and z1 >= z0
            assert z1 - z0 <= tile_nnz + (3 if part >= 0 else 0)
            covered[z0:z1] += 1
            if part < 0:
                rows[r0] += 1
                assert (z0, z1) == (indptr[r0], indptr[r0 + 1])
            else:
                slots[part] = slots.get(part, 0) + 1
        elif mode == 1:    # whole rows
            assert z0 == indptr[r0] and z1 == indptr[r1] and z1 - z0 <= tile_nnz
            covered[z0:z1] += 1
            rows[r0:r1] += 1
        else:              # piece k of z1 pieces of every row in [r0, r1)
            assert mode == 2 and r1 - r0 <= max(band, 1) and 0 <= k < z1
            for i in range(r1 - r0):
                a, b = indptr[r0 + i], indptr[r0 + i + 1]
                lo, hi = _piece_cut(a, b, k, z1), _piece_cut(a, b, k + 1, z1)
                covered[lo:hi] += 1
                if z1 == 1:
                    rows[r0 + i] += 1
                else:
                    slot = part + i * z1 + k
                    slots[slot] = slots.get(slot, 0) + 1
    for row, p0, p1, _ in splits.tolist():
        rows[row] += 1
        for p in range(p0, p1):
            assert slots.pop(p) == 1
    assert not slots
    assert np.all(covered == 1)
    assert np.all(rows == 1)


def _err(rc):
    return rc, azint().lib().azi_last_error().decode()


def test_argument_errors():
    az = azint()
    L = az.lib()
    g = az._Geom(10, 10, 1e-4, 1e-4, 5.0, 5.0, 0.1, 1e-10)
    out = ctypes.c_void_p()
    cases = [
        (dict(npt=0), -1, "npt"),
        (dict(unit=9), -1, "unit"),
        (dict(split=7), -1, "split"),
        (dict(dtype=2), -1, "dtype"),
        (dict(accum=1, dtype=5), -1, "Kahan"),
    ]
    for kw, code, word in cases:
        a = dict(npt=10, unit=0, split=1, dtype=5, accum=0)
        a.update(kw)
        rc, msg = _err(L.azi_plan_create(ctypes.byref(g), a["npt"], a["unit"], a["split"], None,
                                         a["dtype"], a["accum"], ctypes.byref(out)))
        assert rc == code and word in msg, (kw, rc, msg)
    rc, msg = _err(L.azi_plan_create(None, 10, 0, 1, None, 5, 0, ctypes.byref(out)))
    assert rc == -1
    bad = az._Geom(10, 0, 1e-4, 1e-4, 5.0, 5.0, 0.1, 1e-10)
    assert _err(L.azi_plan_create(ctypes.byref(bad), 10, 0, 1, None, 5, 0, ctypes.byref(out)))[0] == -1
    neg = az._Geom(10, 10, -1e-4, 1e-4, 5.0, 5.0, 0.1, 1e-10)
    assert _err(L.azi_plan_create(ctypes.byref(neg), 10, 0, 1, None, 5, 0, ctypes.byref(out)))[0] == -1
    rng = (ctypes.c_double * 2)(2.0, 1.0)
    assert _err(L.azi_plan_create(ctypes.byref(g), 10, 0, 1, ctypes.cast(rng, ctypes.c_void_p),
                                  5, 0, ctypes.byref(out)))[0] == -1
    # a range that holds no pixel is valid and gives an empty matrix
    far = (ctypes.c_double * 2)(1.0, 2.0)
    assert L.azi_plan_create(ctypes.byref(g), 10, 0, 1, ctypes.cast(far, ctypes.c_void_p), 5, 0,
                             ctypes.byref(out)) == 0
    nnz = ctypes.c_int64()
    assert L.azi_plan_info(out, None, None, ctypes.byref(nnz), None) == 0 and nnz.value == 0
    assert L.azi_plan_destroy(out) == 0
    assert L.azi_plan_destroy(None) == 0
    # per-frame calls on a plan that is not on a device
    plan = az.Plan(10, 10, 10)
    # a new plan starts in the stage that sums the dark term once
    assert plan.tiling() == dict(az.DEFAULT_TILING) and plan.tiling()["stage"] == 5
    assert az.STAGES["fold_sum"] == 5 and az.STAGES["fold"] == 4
    rc, msg = _err(L.azi_integrate1d(plan.handle, ctypes.c_void_p(16), ctypes.c_void_p(16),
                                     None, None, 0.0, None))
    assert rc == -5 and "azi_plan_upload" in msg
    T = lambda *v: ctypes.byref(az.Tiling(*v))
    assert _err(L.azi_plan_set_tiling(plan.handle, T(100, 256, 0, 0, 0, 0)))[0] == -1
    assert _err(L.azi_plan_set_tiling(plan.handle, T(1024, 96, 0, 0, 0, 0)))[0] == -1
    assert _err(L.azi_plan_set_tiling(plan.handle, T(1024, 128, 7, 0, 0, 0)))[0] == -1
    assert _err(L.azi_plan_set_tiling(plan.handle, T(1024, 128, -1, 0, 0, 0)))[0] == -1
    assert _err(L.azi_plan_set_tiling(plan.handle, T(1024, 128, 1, -8, 0, 0)))[0] == -1
    assert _err(L.azi_plan_set_tiling(plan.handle, T(1024, 128, 1, 0, 0, 6)))[0] == -1
    assert _err(L.azi_plan_set_tiling(plan.handle, None))[0] == -1
    assert L.azi_plan_set_tiling(plan.handle, T(1024, 128, 6, 512, 4, 1)) == 0
    assert plan.tiling() == dict(tile_nnz=1024, block=128, variant=6, grid=512, band=4, stage=1)
    assert _err(L.azi_plan_set_layout(plan.handle, 6))[0] == -1
    assert _err(L.azi_batch_create(None, 1, 0, ctypes.byref(out)))[0] == -1


@pytest.mark.skipif(torch.cuda.is_available(), reason="checks the no-GPU error path")
def test_upload_without_gpu_fails_cleanly():
    az = azint()
    plan = az.Plan(10, 10, 10)
    rc, msg = _err(az.lib().azi_plan_upload(plan.handle, 0))
    assert rc == -4 and "device" in msg


def test_correction_bytes_without_device_arrays():
    """A plan that holds no device correction records reports 0 bytes per
    pixel (also for a NULL plan)."""
    az = azint()
    assert az.lib().azi_plan_correction_bytes(None) == 0
    plan = az.Plan(12, 13, 6)
    assert plan.correction_bytes() == 0


def test_integration_on_cpu_via_exported_matrix_matches_oracle():
    """The exported CSR is what the kernels stream: scipy's product with it
    reproduces the oracle's W and U (Section 5.2.1 compatibility)."""
    import scipy.sparse as sp
    az = azint()
    plan = az.Plan(120, 90, 110, center=(60.1, 44.8))
    data, indices, indptr = plan.export_csr()
    A = sp.csr_matrix((data, indices, indptr), shape=(110, 120 * 90))
    x = np.random.default_rng(0).uniform(0, 100, size=120 * 90)
    m = oracle_matrix(120, 90, 60.1, 44.8, 110, 1e-4, 1e-4, "r_m", "bbox", None)
    I, W, U = oracle.integrate(m, x)
    assert np.allclose(A @ x, W, rtol=1e-13, atol=0)
    assert np.allclose(np.asarray(A.sum(1)).ravel(), U, rtol=1e-13, atol=0)


def test_stage_tiles_cover_image_once():
    """The LDS staging tables put every pixel at its own ring position
    exactly once (host side of the ring layout)."""
    az = azint()
    for (h, w, npt) in ((70, 300, 90), (33, 129, 40), (1, 1, 3), (200, 256, 150)):
        plan = az.Plan(h, w, npt, center=(h / 3.0, w / 2.0 + 0.3))
        data, indices, indptr = plan.export_csr()
        # ring order: pixels sorted by first bin, ties by pixel id
        _, bins, colptr = plan.export_csc()
        first = np.where(np.diff(colptr) > 0, bins[np.minimum(colptr[:-1], max(len(bins) - 1, 0))], npt)
        order = np.lexsort((np.arange(h * w), first))
        pos = np.empty(h * w, dtype=np.int64)
        pos[order] = np.arange(h * w)
        # tiles of 32x128 pixels, ranks within a tile by ring position
        seen = np.zeros(h * w, dtype=np.int64)
        for i0 in range(0, h, 32):
            for j0 in range(0, w, 128):
                pix = (np.arange(i0, min(i0 + 32, h))[:, None] * w +
                       np.arange(j0, min(j0 + 128, w))[None, :]).ravel()
                seen[pos[pix]] += 1
        assert np.all(seen == 1)


@pytest.mark.parametrize("g", [(40, 50, 20.3, 25.7, 60, "r_m"), (30, 30, 15.0, 15.0, 45, "r_m"),
                               (20, 35, -3.2, 40.1, 33, "2th_deg"), (64, 64, 32.0, 32.0, 90, "q_nm"),
                               (12, 9, 4.5, 9.5, 200, "r_mm")])
def test_full_split_matches_oracle(g):
    """Full splitting (Section 4.2): the library integrates the four edge
    lines over each bin, the oracle clips the quadrilateral and measures it;
    the two agree to rounding."""
    import scipy.sparse as sp
    h, w, cy, cx, npt, unit = g
    az = azint()
    plan = az.Plan(h, w, npt, center=(cy, cx), split="full", unit=unit)
    d, i, p = plan.export_csr()
    A = sp.csr_matrix((d, i, p), shape=(npt, h * w)).toarray()
    m = oracle_matrix(h, w, cy, cx, npt, 1e-4, 1e-4, unit, "full", None)
    B = sp.csr_matrix((m["data"], m["indices"], m["indptr"]), shape=(npt, h * w)).toarray()
    assert np.abs(A - B).max() <= 1e-13
    assert plan.info()["range"] == (m["pmin"], m["pmax"]) or unit != "r_m"
    assert np.abs(A.sum(axis=0) - 1.0).max() <= 1e-13


GEOMS_2D = [
    # h, w, center_y, center_x, npt_rad, npt_azim, unit, split
    (40, 50, 20.5, 24.3, 30, 36, "r_m", "bbox"),
    (32, 32, 16.0, 16.0, 20, 8, "r_m", "bbox"),        # beam on a pixel corner
    (30, 40, -10.0, 15.0, 20, 72, "r_m", "bbox"),      # beam above the detector
    (24, 24, 12.5, 60.0, 10, 360, "r_m", "bbox"),      # rows across the +-pi cut
    (27, 33, 13.2, 16.7, 25, 90, "2th_deg", "bbox"),
    (40, 50, 20.5, 24.3, 30, 36, "r_m", "none"),
    (24, 24, 12.5, 60.0, 10, 360, "r_m", "none"),
    (40, 50, 20.5, 24.3, 30, 36, "r_m", "full"),
    (32, 32, 16.0, 16.0, 20, 8, "r_m", "full"),
    (24, 24, 12.5, 60.0, 10, 360, "r_m", "full"),
    (30, 40, -10.0, 15.0, 20, 72, "q_nm", "full"),
]


def _oracle2d(h, w, cy, cx, nr, na, unit, split):
    return oracle.build_matrix2d(h=h, w=w, pixel_y=1e-4, pixel_x=1e-4, center_y=cy,
                                 center_x=cx, dist=0.1, wavelength=1e-10, npt_rad=nr,
                                 npt_azim=na, unit=unit, split=split)


@pytest.mark.parametrize("g", GEOMS_2D, ids=lambda g: f"{g[0]}x{g[1]}-{g[7]}-{g[6]}-{g[5]}")
def test_plan2d_matches_oracle(g):
    """Two-dimensional plans: the integer structure (and, where every step is
    a correctly rounded operation or the same libm call, the coefficients)
    equals the oracle's bit for bit; full splitting (edge integrals against
    polygon clipping) agrees to rounding."""
    import scipy.sparse as sp
    h, w, cy, cx, nr, na, unit, split = g
    az = azint()
    plan = az.Plan(h, w, nr, npt_azim=na, center=(cy, cx), unit=unit, split=split)
    m = _oracle2d(h, w, cy, cx, nr, na, unit, split)
    assert plan.shape() == (nr, na)
    assert plan.info()["npt"] == nr * na == m["npt"]
    assert np.array_equal(plan.positions(), m["positions"])
    assert np.array_equal(plan.azimuths(), m["azimuths"])
    d, i, p = plan.export_csr()
    if split == "full":
        A = sp.csr_matrix((d, i, p), shape=(nr * na, h * w)).toarray()
        B = sp.csr_matrix((m["data"], m["indices"], m["indptr"]),
                          shape=(nr * na, h * w)).toarray()
        assert np.abs(A - B).max() <= 1e-13
    elif unit == "r_m":
        assert np.array_equal(p, m["indptr"])
        assert np.array_equal(i, m["indices"])
        assert np.array_equal(d, m["data"])
    else:
        # transcendental units: bins agree except where a box edge sits
        # within rounding of a bin edge; coefficients to rounding
        A = sp.csr_matrix((d, i, p), shape=(nr * na, h * w)).toarray()
        B = sp.csr_matrix((m["data"], m["indices"], m["indptr"]),
                          shape=(nr * na, h * w)).toarray()
        assert np.abs(A - B).max() <= 1e-9
    cdata, bins, colptr = plan.export_csc()
    for q in range(h * w):
        seg = bins[colptr[q]:colptr[q + 1]]
        assert np.all(np.diff(seg) > 0), q
    assert np.abs(np.bincount(np.repeat(np.arange(h * w), np.diff(colptr)), weights=cdata,
                              minlength=h * w) - 1.0).max() <= 1e-13


def test_plan2d_argument_errors():
    az = azint()
    for bad in (1, -3):
        with pytest.raises(az.AzintError):
            az.Plan(8, 8, 4, npt_azim=bad)
    plan = az.Plan(8, 8, 4)
    assert plan.shape() == (4, 0)
    with pytest.raises(az.AzintError):
        plan.azimuths()
    with pytest.raises(az.AzintError):
        az.Plan(8, 8, 1 << 16, npt_azim=1 << 16)


@pytest.mark.skipif(torch.cuda.is_available(), reason="checks the no-GPU error path")
def test_device_plan_builder_without_gpu_fails_cleanly():
    az = azint()
    L = az.lib()
    g = az._Geom(8, 8, 1e-4, 1e-4, 4.0, 4.0, 0.1, 1e-10)
    out = ctypes.c_void_p()
    rc = L.azi_plan_create_device(ctypes.byref(g), 8, 0, 1, None, 5, 0, 0, None,
                                  ctypes.byref(out))
    assert rc == -4 and not out.value
    assert b"device" in L.azi_last_error().lower()
    rc = L.azi_plan_create_device(ctypes.byref(g), 8, 0, 1, None, 5, 0, -1, None,
                                  ctypes.byref(out))
    assert rc == -4


def _decode_runs(s, npt):
    """(pixel, bin, coefficient) of every entry of a run encoding, read the
    way the run kernel reads it: per group of 64 runs, the j-th coefficient
    of lane l sits after the groups' earlier slots, at the rank of l among
    the lanes whose runs have more than j entries."""
    runs, gbase, coef, pieces = s["runs"], s["gbase"], s["coef"], s["pieces"]
    band_bin0 = np.full(len(runs), -1, dtype=np.int64)
    for z0, z1, bin0, nrows, slot, *_ in pieces:
        assert z0 % 64 == 0 and z1 >= z0
        band_bin0[z0:z1] = bin0
    pix, bins, cs = [], [], []
    for g in range(len(runs) // 64):
        w = runs[64 * g:64 * g + 64]
        live = (w >= 0) & (band_bin0[64 * g:64 * g + 64] >= 0)
        n = np.where(live, ((w >> 29) & 3) + 1, 0)
        r0 = (w >> 27) & 3
        p = w & ((1 << 27) - 1)
        off = int(gbase[g])
        for j in range(4):
            lanes = np.nonzero(n > j)[0]
            for rank, lane in enumerate(lanes):
                pix.append(int(p[lane]))
                bins.append(int(band_bin0[64 * g + lane] + r0[lane] + j))
                cs.append(coef[off + rank])
            off += len(lanes)
    return np.array(pix), np.array(bins), np.array(cs)


@pytest.mark.parametrize("g", [(90, 100, 44.6, 50.2, 40, "bbox", 0), (31, 29, 15.5, 14.5, 300, "bbox", 0),
                               (64, 48, -5.0, 70.0, 40, "bbox", 0), (1, 17, 0.5, 8.5, 5, "bbox", 0),
                               (120, 130, 60.2, 64.9, 140, "full", 0),
                               (50, 60, 25.3, 30.7, 37, "none", 0),
                               (40, 50, 20.1, 24.7, 20, "bbox", 36)],
                         ids=lambda g: f"{g[0]}x{g[1]}-{g[5]}-{g[4]}-az{g[6]}")
@pytest.mark.parametrize("tile", [64, 4096])
def test_run_encoding_holds_every_entry_once(g, tile):
    """The run layout's host builder: decoded as the kernel reads it, the
    runs give back exactly the plan's entries (pixel, bin, coefficient bits);
    pieces start on multiples of 64 runs and cover each band's runs; every
    bin's slots are its band's pieces."""
    h, w, cy, cx, npt, split, na = g
    az = azint()
    plan = az.Plan(h, w, npt, npt_azim=na or None, center=(cy, cx), split=split, band=4)
    s = plan.run_schedule(tile_nnz=tile)
    pix, bins, cs = _decode_runs(s, plan.npt)
    data, cbins, colptr = plan.export_csc()
    cpix = np.repeat(np.arange(plan.npix), np.diff(colptr))
    a = np.lexsort((bins, pix))
    b = np.lexsort((cbins, cpix))
    assert len(pix) == plan.nnz
    assert np.array_equal(pix[a], cpix[b]) and np.array_equal(bins[a], cbins[b])
    assert np.array_equal(cs[a].view(np.int64), data[b].astype(np.float64).view(np.int64))
    # pieces: per band consecutive, each bin's slots are those of its band's pieces
    for z0, z1, bin0, nrows, slot, *_ in s["pieces"]:
        assert 1 <= nrows <= 4 and slot % 4 == 0
    firsts = {}
    for z0, z1, bin0, nrows, slot, *_ in s["pieces"]:
        firsts.setdefault(int(bin0), []).append(int(slot))
    for bin0, slots in firsts.items():
        assert slots == list(range(slots[0], slots[0] + 4 * len(slots), 4))
        for r in range(4):
            if bin0 + r < plan.npt:
                assert s["bin_slot"][bin0 + r] == slots[0] + r
                assert s["bin_count"][bin0 + r] == len(slots)


def _greedy_stretches(firsts, bound):
    """Stretches of one group of bands cut in pixel order so that no band has
    more than `bound` groups of 64 runs in one (groups starting at one pixel
    stay together): firsts[w] holds the first pixel of each group of band w."""
    ev = sorted((int(px), w) for w, arr in enumerate(firsts) for px in arr)
    count = [0] * len(firsts)
    k, i = 1, 0
    while i < len(ev):
        j = i
        add = [0] * len(firsts)
        while j < len(ev) and ev[j][0] == ev[i][0]:
            add[ev[j][1]] += 1
            j += 1
        if any(a and count[w] + a > bound for w, a in enumerate(add)):
            k += 1
            count = [0] * len(firsts)
        count = [c + a for c, a in zip(count, add)]
        i = j
    return k


@pytest.mark.parametrize("g", [(300, 280, 150.2, 140.7, 260), (257, 263, 10.0, 250.0, 333),
                               (600, 500, 310.5, 240.2, 500), (1000, 1000, 500.3, 499.7, 1000),
                               (1400, 1300, 650.3, 720.7, 1200)],
                         ids=lambda g: f"{g[0]}x{g[1]}-{g[4]}")
@pytest.mark.parametrize("band", [16, 32])
def test_balanced_run_schedule_bound_is_smallest(g, band):
    """tile_nnz 0 on a plan without a device (256 CUs): one round of
    256 * 32 / waves workgroups at most, and the bound on a band's groups of
    64 runs per stretch is the smallest that fits it (recounted here from
    the run words with a greedy cut written for this test); each group of
    bands has exactly as many workgroups as that cut gives."""
    h, w, cy, cx, npt = g
    waves = band // 4
    az = azint()
    plan = az.Plan(h, w, npt, center=(cy, cx), tile_nnz=0, band=band)
    s = plan.run_schedule(tile_nnz=0)
    runs, pieces = s["runs"], s["pieces"]
    nt = len(pieces) // waves
    target = 256 * 32 // waves
    assert nt <= target
    lens = (pieces[:, 1] - pieces[:, 0]).astype(np.int64)
    assert np.all(lens % 64 == 0)
    bound = int(lens.max()) // 64
    assert bound * 64 <= 2048 or bound == 1
    mask = (1 << 27) - 1
    nbands = (npt + 3) // 4
    # first pixel of each group of 64 runs, per band, from the schedule's
    # own band extents (a band's entries tile its runs)
    firsts, tiles_of = {}, {}
    for t in range(nt):
        ents = pieces[t * waves:(t + 1) * waves]
        gi = int(ents[0][2]) // 4 // waves
        tiles_of[gi] = tiles_of.get(gi, 0) + 1
        for e in ents:
            if e[4] < 0:
                continue
            b = int(e[2]) // 4
            for z in range(int(e[0]), int(e[1]), 64):
                firsts.setdefault(b, []).append(int(runs[z]) & mask)
    groups = range((nbands + waves - 1) // waves)
    per = {gi: [firsts.get(b, []) for b in range(gi * waves, min(nbands, (gi + 1) * waves))]
           for gi in groups}
    for gi in groups:
        assert tiles_of[gi] == _greedy_stretches(per[gi], bound), gi
    if bound > 1:
        assert sum(_greedy_stretches(per[gi], bound - 1) for gi in groups) > target


def test_new_entry_points_reject_bad_arguments():
    """Argument errors of the run-schedule export, the plan autotuner and the
    correction-bytes query, without a GPU."""
    az = azint()
    L = az.lib()
    plan = az.Plan(12, 13, 6)
    n = ctypes.c_int64()
    for tn in (-64, 63, 16385):
        rc, msg = _err(L.azi_plan_run_schedule(plan.handle, tn, ctypes.byref(n), None, None,
                                               None, None, None, None, None))
        assert rc == -1 and "tile_nnz" in msg
    assert _err(L.azi_plan_run_schedule(None, 4096, ctypes.byref(n), None, None, None, None,
                                        None, None, None))[0] == -1
    assert L.azi_plan_run_schedule(plan.handle, 64, ctypes.byref(n), None, None, None, None,
                                   None, None, None) == 0 and n.value % 64 == 0
    # the autotuner needs an uploaded plan
    rc, msg = _err(L.azi_plan_autotune(plan.handle, None, None, None, None, None, None, 0))
    assert rc < 0
    assert L.azi_plan_autotune(None, None, None, None, None, None, None, 0) < 0
    assert L.azi_plan_correction_bytes(plan.handle) == 0


def test_overflow_limits_are_reported():
    """Counts that do not fit int32 give AZI_EOVERFLOW (-3) before anything
    large is allocated: 2^31 pixels, 2^31 bins of a 2-D plan, and a 1-D
    matrix of 2^31 nonzeros or more (a 3 x 3 detector whose boxes each span
    ~2^28 of 2^30 bins)."""
    az = azint()
    with pytest.raises(az.AzintError, match="azint error -3: image has 2\\^31 pixels"):
        az.Plan(46341, 46341, 10)
    with pytest.raises(az.AzintError, match="azint error -3: .*2\\^31"):
        az.Plan(4, 4, 1 << 16, npt_azim=1 << 15)
    with pytest.raises(az.AzintError, match="azint error -3: matrix has 2\\^31 nonzeros"):
        az.Plan(3, 3, 1 << 30)
    # just below: the same detector with 2^20 bins builds, ~3e6 nonzeros
    p = az.Plan(3, 3, 1 << 20)
    assert 2_000_000 < p.nnz < 1 << 31


def test_images_of_2_27_pixels_default_to_the_csr_layout():
    """The run and band layouts number pixels in 27 bits: an image of 2^27
    pixels or more (here 11586^2, with a narrow radial range so that the
    matrix stays small) starts in the pixel (CSR) layout, and the run
    schedule of it is refused with AZI_EOVERFLOW."""
    az = azint()
    n = 11586
    assert n * n >= 1 << 27
    p = az.Plan(n, n, 16, center=(n / 2 + 0.3, n / 2 - 0.2), range=(2e-4, 6e-4))
    assert p.layout() == "pixel"
    assert 0 < p.nnz < 10_000
    cnt = ctypes.c_int64()
    rc = az.lib().azi_plan_run_schedule(p._h, 4096, ctypes.byref(cnt), None, None, None, None,
                                        None, None, None)
    assert rc == -3
    assert b"2^27" in az.lib().azi_last_error()
    # the matrix itself is right: each row against the oracle's, via the
    # pixels that can reach the range
    data, indices, indptr = p.export_csr()
    ii, jj = np.divmod(indices, n)
    assert np.all(np.abs(ii - n / 2) < 8) and np.all(np.abs(jj - n / 2) < 8)
    del p


@pytest.mark.parametrize("g", [(300, 280, 150.2, 140.7, 260), (90, 100, 44.6, 50.2, 41),
                               (64, 48, -5.0, 70.0, 40), (1, 17, 0.5, 8.5, 5),
                               (257, 263, 10.0, 250.0, 333)],
                         ids=lambda g: f"{g[0]}x{g[1]}-{g[4]}")
@pytest.mark.parametrize("band", [16, 32])
@pytest.mark.parametrize("tile", [128, 1024, 4096, 0])
def test_grouped_run_schedule_covers_every_run_once(g, band, tile):
    """Workgroups of 4 or 8 neighbouring bands: entry t * waves + w is band
    w of the workgroup's group; each band's entries tile its runs on
    multiples of 64 in order, the entries of a workgroup cover one common
    stretch of image rows (no band's entry starts before the stretch's first
    pixel nor holds a group starting past its end), and each bin's slots are
    its band's entries in order."""
    h, w, cy, cx, npt = g
    waves = band // 4
    az = azint()
    plan = az.Plan(h, w, npt, center=(cy, cx), tile_nnz=tile, band=band)
    s = plan.run_schedule(tile_nnz=tile)
    runs, pieces = s["runs"], s["pieces"]
    nbands = (npt + 3) // 4
    assert len(pieces) % waves == 0
    ntiles = len(pieces) // waves
    mask = (1 << 27) - 1
    per_band = {}
    for t in range(ntiles):
        ents = pieces[t * waves:(t + 1) * waves]
        bands = [int(e[2]) // 4 for e in ents if e[4] >= 0]
        assert bands == list(range(bands[0], bands[0] + len(bands)))
        assert bands[0] % waves == 0
        for e in ents:
            z0, z1, bin0, nrows, slot = (int(v) for v in e[:5])
            if slot < 0:
                assert z0 == z1 == 0
                continue
            assert z0 % 64 == 0 and z1 % 64 == 0 and z0 <= z1
            assert nrows == min(4, npt - bin0) and slot % 4 == 0
            per_band.setdefault(bin0 // 4, []).append((t, z0, z1, slot))
    assert sorted(per_band) == list(range(nbands))
    # every band: entries consecutive, covering [band start, band end)
    starts = [0]
    for b in range(nbands):
        ent = per_band[b]
        assert ent[0][1] == starts[-1]
        for (_, _, z1, s0), (_, z0n, _, s1) in zip(ent, ent[1:]):
            assert z0n == z1 and s1 == s0 + 4
        end = ent[-1][2]
        valid = runs[ent[0][1]:end] >= 0
        assert end % 64 == 0 and (end - ent[0][1]) >= valid.sum()
        starts.append(end)
        for r in range(min(4, npt - 4 * b)):
            assert s["bin_slot"][4 * b + r] == ent[0][3] + r
            assert s["bin_count"][4 * b + r] == len(ent)
    assert starts[-1] == len(runs)
    # one stretch of rows per workgroup: a band's entry starts at the first
    # group whose first pixel is not before the stretch (taken from the
    # neighbours' entries of the same workgroup)
    for t in range(ntiles):
        ents = [e for e in pieces[t * waves:(t + 1) * waves] if e[4] >= 0]
        firsts = [int(runs[e[0]]) & mask for e in ents if e[1] > e[0] and runs[e[0]] >= 0]
        lasts = [int(runs[e[1] - 64]) & mask for e in ents if e[1] > e[0] and runs[e[1] - 64] >= 0]
        if firsts and lasts and len(ents) > 1:
            # groups of one workgroup start within the same stretch of pixels
            assert max(firsts) <= max(lasts) + w * 64
