"""Checks that pin the oracle to facts other than itself.

Each ``pin_*`` function takes an oracle-like namespace (the real ``oracle``
package, or a copy with a planted mistake) and raises AssertionError when the
fact it checks does not hold.  The facts come from the paper and from plain
mathematics: exact rational brute force, numpy's histogram, the plain masked
mean, conservation laws, symmetry, scipy's sparse product and the adjoint
identity.
"""
from __future__ import annotations

import math
from fractions import Fraction as F

import numpy as np

TINY_CASES = [
    # (h, w, center_y, center_x, npt, pixel_y, pixel_x)
    (3, 3, 1.5, 1.5, 4, 1e-4, 1e-4),
    (4, 5, 2.0, 2.5, 5, 1e-4, 1e-4),
    (7, 6, 3.5, 3.0, 9, 1e-4, 1e-4),
    (5, 4, 0.3, 3.7, 6, 1e-4, 1e-4),      # off-centre beam
    (6, 7, -1.25, 2.2, 7, 1e-4, 1e-4),    # beam outside the detector
    (4, 6, 1.1, 2.9, 13, 1.5e-4, 1e-4),   # rectangular pixels, fine bins
]
DIST, WL = 0.1, 1e-10


def _geom_args(case):
    h, w, cy, cx, npt, py, px = case
    return dict(h=h, w=w, pixel_y=py, pixel_x=px, center_y=cy, center_x=cx,
                dist=DIST, wavelength=WL)


def exact_extent_sq(h, w, py, px, cy, cx):
    """Exact squared radial extent of every pixel square, as Fractions.

    hi^2 is the largest squared corner distance (the distance is convex);
    lo^2 is the squared distance to the point of the square nearest to the
    centre, found by clamping the centre into the square.
    """
    py, px, cy, cx = F(py), F(px), F(cy), F(cx)
    lo2, hi2 = [], []
    for i in range(h):
        for j in range(w):
            corners = [(((j + a) - cx) * px) ** 2 + (((i + b) - cy) * py) ** 2
                       for a in (0, 1) for b in (0, 1)]
            hi2.append(max(corners))
            nx = min(max(cx, F(j)), F(j + 1))
            ny = min(max(cy, F(i)), F(i + 1))
            lo2.append(((nx - cx) * px) ** 2 + ((ny - cy) * py) ** 2)
    return lo2, hi2


def exact_bbox_matrix(lo, hi, npt, pmin, pmax):
    """Exact overlap / width of every box with every bin (dense, Fractions)."""
    pmin, pmax = F(pmin), F(pmax)
    d = (pmax - pmin) / npt
    A = {}
    for p, (l, u) in enumerate(zip(lo, hi)):
        l, u = F(float(l)), F(float(u))
        if u == l:
            continue
        for b in range(npt):
            a0, a1 = pmin + b * d, pmin + (b + 1) * d
            ov = min(u, a1) - max(l, a0)
            if ov > 0:
                A[(b, p)] = ov / (u - l)
    return A


def exact_rect_area(poly, a, b, c=None, d=None):
    """Signed area of polygon `poly` (list of (x, y) Fractions, any order of
    traversal, simple or not) inside the rectangle [a, b] x [c, d]; c / d
    None leave y unbounded (a vertical slab).

    Green's theorem edge by edge, with no polygon clipping: the area is
    -(closed integral of y dx) over the boundary of the clipped region; the
    parts of that boundary on x = a or x = b have dx = 0, and those on y = c
    or y = d are accounted for by clamping y into [c, d].  So every edge
    contributes -integral of clamp(y(x), c, d) dx over its x-span within
    [a, b], integrated exactly: the span is cut where y(x) meets c or d, and
    on each piece the integrand is a constant or y(x) itself (trapezoid).
    Counter-clockwise traversal gives a positive area."""
    def clamp(v):
        if c is not None and v < c:
            return c
        if d is not None and v > d:
            return d
        return v

    total = F(0)
    n = len(poly)
    for k in range(n):
        (x0, y0), (x1, y1) = poly[k], poly[(k + 1) % n]
        if x0 == x1:
            continue
        lo_, hi_ = max(min(x0, x1), a), min(max(x0, x1), b)
        if hi_ <= lo_:
            continue
        slope = (y1 - y0) / (x1 - x0)
        yat = lambda x: y0 + slope * (x - x0)
        cuts = {lo_, hi_}
        for level in (c, d):
            if level is not None and slope != 0:
                xc = x0 + (level - y0) / slope
                if lo_ < xc < hi_:
                    cuts.add(xc)
        cuts = sorted(cuts)
        part = F(0)
        for u, v in zip(cuts[:-1], cuts[1:]):
            part += (v - u) * (clamp(yat(u)) + clamp(yat(v))) / 2
        total += -part if x1 > x0 else part
    return total


def pin_extents_exact(O):
    """P1a: lo and hi are the correctly rounded true radial extent (R2)."""
    for case in TINY_CASES:
        h, w, cy, cx, npt, py, px = case
        lo, hi, _ = O.pixel_extents(**_geom_args(case))
        lo2, hi2 = exact_extent_sq(h, w, py, px, cy, cx)
        for p in range(h * w):
            for got, ex in ((lo[p], lo2[p]), (hi[p], hi2[p])):
                ref = math.sqrt(float(ex))
                assert abs(got - ref) <= 4 * math.ulp(max(ref, 1e-300)), (case, p, got, ref)


def pin_bbox_bruteforce(O):
    """P1b: bbox coefficients equal exact overlap/width (Section 4.1)."""
    for case in TINY_CASES:
        args = _geom_args(case)
        npt = case[4]
        m = O.build_matrix(npt=npt, split="bbox", **args)
        exact = exact_bbox_matrix(m["lo"], m["hi"], npt, m["pmin"], m["pmax"])
        got = {}
        for b, p, c in zip(m["bins"].tolist(), m["pix"].tolist(), m["coef"].tolist()):
            assert (b, p) not in got, "duplicate entry"
            got[(b, p)] = c
        for key, c in got.items():
            ref = float(exact.get(key, 0))
            assert abs(c - ref) <= 1e-12, (case, key, c, ref)
        for key, ref in exact.items():
            if key not in got:
                assert float(ref) <= 1e-12, (case, key, float(ref))


def pin_results_exact(O):
    """P1c: W, U, I equal their exact rational values on integer images."""
    rng = np.random.default_rng(11)
    for case in TINY_CASES:
        h, w = case[0], case[1]
        npt = case[4]
        m = O.build_matrix(npt=npt, split="bbox", **_geom_args(case))
        x = rng.integers(0, 1 << 20, size=h * w)
        I, W, U = O.integrate(m, x.astype(np.float64))
        exact = exact_bbox_matrix(m["lo"], m["hi"], npt, m["pmin"], m["pmax"])
        for b in range(npt):
            We = sum((c * int(x[p]) for (bb, p), c in exact.items() if bb == b), F(0))
            Ue = sum((c for (bb, p), c in exact.items() if bb == b), F(0))
            assert abs(W[b] - float(We)) <= 1e-12 * max(1.0, abs(float(We))), (case, b)
            assert abs(U[b] - float(Ue)) <= 1e-12 * max(1.0, float(Ue)), (case, b)
            if Ue != 0:
                Ie = float(We / Ue)
                assert abs(I[b] - Ie) <= 1e-12 * max(1.0, abs(Ie)), (case, b, I[b], Ie)


def pin_nosplit_histogram(O):
    """P2: no splitting == ratio of numpy's weighted/unweighted histograms
    (Section 3.3), except pixels within rounding of a bin edge."""
    rng = np.random.default_rng(5)
    for (h, w, npt) in [(37, 41, 23), (64, 48, 50), (100, 100, 100)]:
        args = dict(h=h, w=w, pixel_y=1e-4, pixel_x=1e-4, center_y=h / 2 + 0.3,
                    center_x=w / 2 - 0.2, dist=DIST, wavelength=WL)
        m = O.build_matrix(npt=npt, split="none", **args)
        x = rng.integers(0, 1 << 20, size=h * w).astype(np.float64)
        I, W, U = O.integrate(m, x)
        r = m["centre"]
        hu, edges = np.histogram(r, npt, range=(m["pmin"], m["pmax"]))
        hw, _ = np.histogram(r, npt, range=(m["pmin"], m["pmax"]), weights=x)
        frac = (r - m["pmin"]) / ((m["pmax"] - m["pmin"]) / npt)
        near_edge = np.abs(frac - np.round(frac)) < 1e-9
        if not near_edge.any():
            assert np.array_equal(U, hu.astype(np.float64))
            assert np.allclose(W, hw, rtol=1e-15, atol=0)
        else:
            assert abs(U.sum() - hu.sum()) == 0
            assert np.abs(U - hu).sum() <= 2 * near_edge.sum()


def pin_naive_mean(O):
    """P3: no splitting over [0, max r] == per-bin masked mean of the pixels
    with r1 <= r < r2 (Section 3.2), the pixel at r == rmax aside."""
    rng = np.random.default_rng(6)
    h, w, npt = 30, 34, 40
    args = dict(h=h, w=w, pixel_y=1e-4, pixel_x=1e-4, center_y=11.3, center_x=20.6,
                dist=DIST, wavelength=WL)
    probe = O.build_matrix(npt=npt, split="none", **args)
    r = probe["centre"]
    rmax = float(r.max())
    m = O.build_matrix(npt=npt, split="none", range_=(0.0, rmax), **args)
    x = rng.integers(0, 1 << 16, size=h * w).astype(np.float64)
    I, W, U = O.integrate(m, x, empty=np.nan)
    frac = r / (rmax / npt)
    near = np.abs(frac - np.round(frac)) < 1e-9
    near[np.argmax(r)] = False
    assert not near.any(), "geometry chosen so that no centre sits on an edge"
    compared = 0
    for b in range(npt):
        r1, r2 = rmax * b / npt, rmax * (b + 1) / npt
        sel = x[(r >= r1) & (r < r2)]
        if b == npt - 1:
            sel = x[(r >= r1) & (r <= r2)]   # closed last bin (reading R3)
        if sel.size == 0:
            assert U[b] == 0 and np.isnan(I[b])
        else:
            assert U[b] == sel.size, (b, U[b], sel.size)
            assert abs(I[b] - sel.mean()) <= 1e-12 * abs(sel.mean())
            compared += 1
    assert compared >= npt - 2


def pin_conservation(O):
    """P4: sum U = number of pixels and sum W = sum of the image over the
    default range (Section 4: splitting conserves signal and pixel count)."""
    rng = np.random.default_rng(7)
    for (h, w, npt, cy, cx) in [(50, 60, 37, 25.0, 30.0), (41, 33, 80, 3.3, 29.1),
                                (64, 64, 7, 32.0, 32.0)]:
        for split in ("bbox", "none"):
            m = O.build_matrix(h=h, w=w, pixel_y=1e-4, pixel_x=1e-4, center_y=cy,
                               center_x=cx, dist=DIST, wavelength=WL, npt=npt,
                               split=split)
            x = rng.uniform(-1.0, 3.0, size=h * w)
            I, W, U = O.integrate(m, x)
            n = h * w
            assert abs(U.sum() - n) <= 1e-12 * n, (split, U.sum(), n)
            assert abs(W.sum() - x.sum()) <= 1e-12 * np.abs(x).sum(), split


def pin_unit_weights(O):
    """P5: every pixel's coefficients add up to one (box fully in range)."""
    m = O.build_matrix(h=40, w=45, pixel_y=1e-4, pixel_x=1e-4, center_y=20.0,
                       center_x=22.5, dist=DIST, wavelength=WL, npt=60, split="bbox")
    s = np.zeros(m["npix"])
    np.add.at(s, m["pix"], m["coef"])
    assert np.all(np.abs(s - 1.0) <= 1e-13), np.abs(s - 1.0).max()
    # every coefficient lies in (0, 1]
    assert np.all(m["coef"] > 0) and np.all(m["coef"] <= 1.0 + 1e-15)


def pin_constant_image(O):
    """P6: a constant image integrates to that constant in every bin."""
    for split in ("bbox", "none"):
        m = O.build_matrix(h=33, w=29, pixel_y=1e-4, pixel_x=1e-4, center_y=5.5,
                           center_x=14.0, dist=DIST, wavelength=WL, npt=45, split=split)
        I, W, U = O.integrate(m, np.full(m["npix"], 3.25))
        nz = U > 0
        assert np.all(np.abs(I[nz] - 3.25) <= 4e-15 * 3.25)


def pin_symmetry(O):
    """P7: on a centred square detector the radial profile of an image equals
    that of its transpose and of its mirror images."""
    rng = np.random.default_rng(8)
    n = 24
    m = O.build_matrix(h=n, w=n, pixel_y=1e-4, pixel_x=1e-4, center_y=n / 2,
                       center_x=n / 2, dist=DIST, wavelength=WL, npt=31, split="bbox")
    img = rng.uniform(0, 10, size=(n, n))
    I0, W0, U0 = O.integrate(m, img.reshape(-1))
    for t in (img.T, img[::-1, :], img[:, ::-1], img[::-1, ::-1]):
        I1, W1, U1 = O.integrate(m, np.ascontiguousarray(t).reshape(-1))
        assert np.allclose(I1, I0, rtol=1e-13, atol=0)
        assert np.allclose(W1, W0, rtol=1e-13, atol=0)


def pin_scipy_csr(O):
    """P8: the CSR arrays feed scipy.sparse.csr_matrix directly (Section 5.2.1):
    A @ x gives W, the row sums give U, A.T @ v gives the adjoint."""
    import scipy.sparse as sp
    rng = np.random.default_rng(9)
    m = O.build_matrix(h=45, w=52, pixel_y=1e-4, pixel_x=1e-4, center_y=10.0,
                       center_x=40.5, dist=DIST, wavelength=WL, npt=70, split="bbox")
    A = sp.csr_matrix((m["data"], m["indices"], m["indptr"]), shape=(m["npt"], m["npix"]))
    x = rng.uniform(0, 100, size=m["npix"])
    I, W, U = O.integrate(m, x)
    assert np.allclose(A @ x, W, rtol=1e-13, atol=0)
    assert np.allclose(np.asarray(A.sum(axis=1)).ravel(), U, rtol=1e-13, atol=0)
    g = rng.standard_normal(m["npt"])
    gx = O.integrate_vjp(m, U, grad_I=g)
    v = np.where(U > 0, g / np.where(U > 0, U, 1.0), 0.0)
    assert np.allclose(A.T @ v, gx, rtol=1e-12, atol=1e-300)
    # rows hold strictly ascending pixel ids
    for b in range(m["npt"]):
        row = m["indices"][m["indptr"][b]:m["indptr"][b + 1]]
        assert np.all(np.diff(row) > 0)


def pin_adjoint(O):
    """P9: <g, I(x)> is linear in x, so <g, I(x)> = <gx, x> exactly in real
    arithmetic, and central differences carry no truncation error."""
    rng = np.random.default_rng(10)
    m = O.build_matrix(h=30, w=26, pixel_y=1e-4, pixel_x=1e-4, center_y=14.2,
                       center_x=13.0, dist=DIST, wavelength=WL, npt=35, split="bbox")
    x = rng.uniform(0, 1, size=m["npix"])
    g = rng.standard_normal(m["npt"])
    gw = rng.standard_normal(m["npt"])
    I, W, U = O.integrate(m, x)
    gx = O.integrate_vjp(m, U, grad_I=g, grad_W=gw)
    lhs = float(np.dot(g, I) + np.dot(gw, W))
    rhs = float(np.dot(gx, x))
    assert abs(lhs - rhs) <= 1e-13 * (np.abs(g) @ np.abs(I) + np.abs(gw) @ np.abs(W))
    h = 1e-6
    for p in rng.choice(m["npix"], size=12, replace=False):
        xp, xm = x.copy(), x.copy()
        xp[p] += h
        xm[p] -= h
        Ip, Wp, _ = O.integrate(m, xp)
        Im, Wm, _ = O.integrate(m, xm)
        fd = (np.dot(g, Ip - Im) + np.dot(gw, Wp - Wm)) / (2 * h)
        scale = (np.abs(g) @ np.abs(I) + np.abs(gw) @ np.abs(W)) * 2.3e-16 / h
        assert abs(fd - gx[p]) <= 4 * scale + 1e-9 * abs(gx[p]), (p, fd, gx[p])


def pin_kahan(O):
    """P10: float32 Kahan summation stays within 2u * sum|x| (+O(n u^2)) of the
    exact sum (Kahan 1965; Higham, Accuracy and Stability, Section 4.3),
    where plain float32 summation does not."""
    rng = np.random.default_rng(12)
    u = 2.0 ** -24
    for n in (1000, 20000):
        vals = np.concatenate([rng.uniform(0, 1, n).astype(np.float32),
                               np.float32([1e4]), rng.uniform(0, 1, n).astype(np.float32)])
        exact = math.fsum(float(v) for v in vals)
        got = float(O.kahan_sum_f32(vals))
        bound = (2 * u + 4 * len(vals) * u * u) * float(np.abs(vals.astype(np.float64)).sum())
        assert abs(got - exact) <= bound, (n, got - exact, bound)
        naive = np.float32(0)
        for v in vals:
            naive = np.float32(naive + v)
        assert abs(float(naive) - exact) > abs(got - exact)


def pin_closed_forms(O):
    """Hand-derived closed forms.

    * 3x3 detector, beam at its middle: the middle pixel spans [0, sqrt(1/2)],
      an edge pixel [1/2, sqrt(5/2)], a corner pixel [sqrt(1/2), sqrt(9/2)]
      (pixel units; R2: an edge pixel's nearest point is an edge midpoint).
    * 2x2 detector, beam at the shared corner, 2 bins over [0, sqrt 2]: every
      pixel spans both bins with weight 1/2, so U = (2, 2), W = (S/2, S/2).
    * a radius equal to the distance is 2theta = 45 deg exactly (pi/4 rad),
      and q = 4 pi sin(pi/8) / lambda.
    """
    p = 1e-4
    lo, hi, rc = O.pixel_extents(3, 3, p, p, 1.5, 1.5, DIST, WL, "r_m")
    s = lambda v: math.sqrt(v) * p
    assert lo[4] == 0.0 and abs(hi[4] - s(0.5)) <= 2 * math.ulp(s(0.5))
    for e in (1, 3, 5, 7):
        assert abs(lo[e] - 0.5 * p) <= 2 * math.ulp(p) and abs(hi[e] - s(2.5)) <= 2 * math.ulp(s(2.5))
    for c in (0, 2, 6, 8):
        assert abs(lo[c] - s(0.5)) <= 2 * math.ulp(s(0.5)) and abs(hi[c] - s(4.5)) <= 2 * math.ulp(s(4.5))
    assert rc[4] == 0.0
    m = O.build_matrix(h=2, w=2, pixel_y=p, pixel_x=p, center_y=1.0, center_x=1.0,
                       dist=DIST, wavelength=WL, npt=2, split="bbox")
    assert np.array_equal(m["indptr"], [0, 4, 8])
    assert np.allclose(m["data"], 0.5, rtol=0, atol=2e-16)
    x = np.array([1.0, 2.0, 4.0, 8.0])
    I, W, U = O.integrate(m, x)
    assert np.allclose(U, [2.0, 2.0], rtol=1e-15) and np.allclose(W, [7.5, 7.5], rtol=1e-15)
    assert np.allclose(I, [3.75, 3.75], rtol=1e-15)
    r = np.array([DIST])
    assert abs(O.unit_of_radius(r, "2th_deg", DIST, WL)[0] - 45.0) <= 1e-13
    assert abs(O.unit_of_radius(r, "2th_rad", DIST, WL)[0] - math.pi / 4) <= 1e-15
    q = O.unit_of_radius(r, "q_nm", DIST, WL)[0]
    assert abs(q - 4 * math.pi * math.sin(math.pi / 8) / (WL * 1e9)) <= 1e-13 * q
    assert O.unit_of_radius(r, "r_mm", DIST, WL)[0] == 100.0


def pin_bbox_clipped(O):
    """P1d: with a range narrower than the data, each coefficient is the
    exact overlap with the bin over the FULL box width (reading R4)."""
    for case in TINY_CASES[:4]:
        args = _geom_args(case)
        npt = case[4]
        full = O.build_matrix(npt=npt, split="bbox", **args)
        span = full["pmax"] - full["pmin"]
        rng_ = (full["pmin"] + 0.31 * span, full["pmin"] + 0.77 * span)
        m = O.build_matrix(npt=npt, split="bbox", range_=rng_, **args)
        exact = exact_bbox_matrix(m["lo"], m["hi"], npt, rng_[0], rng_[1])
        got = {(b, p): c for b, p, c in zip(m["bins"].tolist(), m["pix"].tolist(),
                                              m["coef"].tolist())}
        assert len(got) > 0
        for key in set(got) | set(exact):
            assert abs(got.get(key, 0.0) - float(exact.get(key, 0))) <= 1e-12, (case, key)
        s = np.zeros(m["npix"])
        np.add.at(s, m["pix"], m["coef"])
        assert s.max() <= 1.0 + 1e-13 and s.min() < 1.0 - 1e-3


def pin_correction(O):
    """Correction map of Section 6.4 on hand-computed values."""
    raw = np.array([10, 7, 3, 1000], dtype=np.int32)
    dark = np.array([2.0, 7.0, 4.0, 0.0])
    flat = np.array([2.0, 1.0, 0.5, 1.0])
    solid = np.array([0.5, 1.0, 1.0, 0.25])
    polar = np.array([4.0, 1.0, 2.0, 1.0])
    x = O.correct(raw, dark, flat, solid, polar)
    assert np.array_equal(x, [2.0, 0.0, -1.0, 4000.0])
    assert np.array_equal(O.correct(raw), raw.astype(np.float64))
    assert np.array_equal(O.correct(raw, dark=dark), [8.0, 0.0, -1.0, 1000.0])
    assert np.array_equal(O.correct(raw, flat=flat), [5.0, 7.0, 6.0, 1000.0])
    assert np.array_equal(O.correct(raw, solid=solid, polar=polar), [5.0, 7.0, 1.5, 4000.0])



def pin_correction_norm(O):
    """The normalisation of Section 6.4, norm = (flat * solid) * polar, on
    hand-computed products; absent arrays drop out of the product."""
    flat = np.array([2.0, 0.5, 1.0, 4.0])
    solid = np.array([0.5, 1.0, 0.25, 0.5])
    polar = np.array([4.0, 2.0, 1.0, 0.125])
    assert np.array_equal(O.correction_norm(flat, solid, polar), [4.0, 1.0, 0.25, 0.25])
    assert np.array_equal(O.correction_norm(flat, None, polar), [8.0, 1.0, 1.0, 0.5])
    assert np.array_equal(O.correction_norm(None, solid, None), solid)
    assert O.correction_norm() is None
    raw = np.array([9, 3, 1, 2])
    assert np.array_equal(O.correct(raw, None, flat, solid, polar), [2.25, 3.0, 4.0, 8.0])


def _exact_centre_sq(h, w, py, px, cy, cx):
    py, px, cy, cx = F(py), F(px), F(cy), F(cx)
    return [((F(2 * j + 1, 2) - cx) * px) ** 2 + ((F(2 * i + 1, 2) - cy) * py) ** 2
            for i in range(h) for j in range(w)]


def _near(got, ref, ulps):
    if ref == 0.0:
        return got == 0.0
    return abs(got - ref) <= ulps * math.ulp(ref)


def pin_default_range(O):
    """Reading R3: without an explicit range the bins span [min lo, max hi]
    of the pixels' radial boxes when pixels are split (so that every box
    lies inside and pixels are conserved), and [min, max] of the pixel-centre
    values without splitting, as numpy's histogram of Section 3.3 takes it.
    Checked against the exact extents (square roots of exact rationals),
    including detectors whose beam lies outside them, where the range does
    not start at 0, and through the monotone unit maps of Section 3."""
    for case in TINY_CASES:
        h, w, cy, cx, npt, py, px = case
        args = _geom_args(case)
        lo2, hi2 = exact_extent_sq(h, w, py, px, cy, cx)
        c2 = _exact_centre_sq(h, w, py, px, cy, cx)
        rlo, rhi = math.sqrt(float(min(lo2))), math.sqrt(float(max(hi2)))
        for split in ("bbox", "full"):
            m = O.build_matrix(npt=npt, split=split, **args)
            assert _near(m["pmin"], rlo, 4) and _near(m["pmax"], rhi, 4), (case, split)
        m = O.build_matrix(npt=npt, split="none", **args)
        clo, chi = math.sqrt(float(min(c2))), math.sqrt(float(max(c2)))
        assert _near(m["pmin"], clo, 4) and _near(m["pmax"], chi, 4), (case, "none")
        edges = np.histogram(m["centre"], npt)[1]
        assert edges[0] == m["pmin"] and edges[-1] == m["pmax"]
        m2 = O.build_matrix2d(npt_rad=npt, npt_azim=4, split="bbox", **args)
        assert _near(m2["pmin"], rlo, 4) and _near(m2["pmax"], rhi, 4), (case, "2d")
        # 2theta in degrees: atan(r / d) * 180 / pi of the same extremes
        m = O.build_matrix(npt=npt, split="bbox", unit="2th_deg", **args)
        for got, r in ((m["pmin"], rlo), (m["pmax"], rhi)):
            ref = math.degrees(math.atan(r / DIST))
            assert _near(got, ref, 16), (case, got, ref)
    # the beam outside the detector: the box range starts well above 0
    h, w, cy, cx, npt, py, px = TINY_CASES[4]
    m = O.build_matrix(npt=npt, split="bbox", **_geom_args(TINY_CASES[4]))
    assert m["pmin"] > 0.2e-4


def pin_positions(O):
    """The abscissa returned with the profile (the tth of the usage example
    in Section 3) is each bin's centre pmin + (b + 1/2) (pmax - pmin) / npt:
    exact rationals, the midpoints of numpy's histogram edges (Section 3.3),
    and the positions stored with a built matrix are those of its range."""
    for npt, pmin, pmax in ((4, 0.0, 1.0), (7, 0.25, 3.5), (13, 1.0e-4, 2.7e-3),
                            (1, -1.0, 1.0), (1000, 0.0, 0.2)):
        got = O.positions(npt, pmin, pmax)
        assert len(got) == npt
        d = (F(pmax) - F(pmin)) / npt
        for b in range(npt):
            ref = float(F(pmin) + (b + F(1, 2)) * d)
            assert _near(got[b], ref, 4), (npt, pmin, pmax, b, got[b], ref)
        edges = np.linspace(pmin, pmax, npt + 1)
        assert np.allclose(got, (edges[:-1] + edges[1:]) / 2, rtol=1e-14, atol=0)
    for case in TINY_CASES[:3]:
        h, w, cy, cx, npt, py, px = case
        m = O.build_matrix(npt=npt, split="none", **_geom_args(case))
        edges = np.histogram(m["centre"], npt)[1]
        assert np.allclose(m["positions"], (edges[:-1] + edges[1:]) / 2, rtol=1e-14, atol=0)
        m2 = O.build_matrix2d(npt_rad=npt, npt_azim=6, split="bbox", **_geom_args(case))
        d = (F(m2["pmax"]) - F(m2["pmin"])) / npt
        for b in range(npt):
            assert _near(m2["positions"][b], float(F(m2["pmin"]) + (b + F(1, 2)) * d), 4)
        dc = 2 * F(math.pi) / 6
        for k in range(6):
            assert abs(m2["azimuths"][k] - float(-F(math.pi) + (k + F(1, 2)) * dc)) <= 1e-15


FULL_CASES = [
    # (h, w, center_y, center_x, npt, pixel_y, pixel_x)
    (5, 6, 2.5, 3.0, 9, 1e-4, 1e-4),
    (6, 5, 7.3, -2.1, 8, 1e-4, 1e-4),      # beam off the detector, left of it
    (4, 7, 1.7, 3.2, 15, 1.5e-4, 1e-4),
    (7, 7, 3.5, 3.5, 4, 1e-4, 1e-4),
]


def pin_full_exact(O):
    """P12: full-splitting coefficients equal the exact area fractions of the
    corner quadrilaterals (Section 4.2, reading R13), each bin's share
    integrated exactly in rational arithmetic from the float64 corner
    coordinates by Green's theorem (``exact_rect_area``: no polygon
    clipping, unlike the oracle), bbox where the pixel holds the centre."""
    for case in FULL_CASES:
        h, w, cy, cx, npt, py, px = case
        args = _geom_args(case)
        m = O.build_matrix(npt=npt, split="full", **args)
        corners = O.pixel_corners(h, w, py, px, cy, cx, DIST, WL, "r_m")
        pmin, pmax = F(m["pmin"]), F(m["pmax"])
        d = (pmax - pmin) / npt
        got = {(b, p): c for b, p, c in zip(m["bins"].tolist(), m["pix"].tolist(),
                                              m["coef"].tolist())}
        exact = {}
        for p in range(h * w):
            if m["lo"][p] == 0.0:
                continue
            quad = [(F(float(a)), F(float(b))) for a, b in corners[p]]
            area = exact_rect_area(quad, min(q[0] for q in quad), max(q[0] for q in quad))
            for b in range(npt):
                a_b = exact_rect_area(quad, pmin + b * d, pmin + (b + 1) * d)
                if a_b != 0:
                    exact[(b, p)] = a_b / area
        for key, ref in exact.items():
            assert abs(got.get(key, 0.0) - float(ref)) <= 1e-12, (case, key)
        for key, c in got.items():
            p = key[1]
            if m["lo"][p] != 0.0:
                assert abs(c - float(exact.get(key, 0))) <= 1e-12, (case, key)


def pin_full_physical_area(O):
    """P13: away from the beam the corner quadrilateral in (r, chi) is close
    to the pixel's image, so its split follows the physical area of the pixel
    square inside each annulus (Monte Carlo, 4e5 points per pixel)."""
    rng = np.random.default_rng(3)
    # second geometry: beam right of the detector, so the middle rows straddle
    # the azimuth cut at +-pi
    for (h, w, cy, cx, npt, pixels) in ((6, 6, -40.0, -35.0, 12, (0, 7, 14, 21, 35)),
                                        (6, 6, 3.0, 46.0, 10, (12, 13, 15, 17, 3))):
        args = dict(h=h, w=w, pixel_y=1e-4, pixel_x=1e-4, center_y=cy, center_x=cx,
                    dist=DIST, wavelength=WL)
        m = O.build_matrix(npt=npt, split="full", **args)
        delta = (m["pmax"] - m["pmin"]) / npt
        for p in pixels:
            i, j = divmod(p, w)
            u = rng.uniform(0, 1, size=(400000, 2))
            x = (j + u[:, 0] - cx) * 1e-4
            y = (i + u[:, 1] - cy) * 1e-4
            fb = np.floor((np.sqrt(x * x + y * y) - m["pmin"]) / delta).astype(int)
            frac = np.bincount(np.clip(fb, 0, npt - 1), minlength=npt) / len(fb)
            sel = m["pix"] == p
            got = np.zeros(npt)
            got[m["bins"][sel]] = m["coef"][sel]
            assert np.abs(got - frac).max() < 5e-3, (cy, cx, p, got, frac)


def pin_full_conservation(O):
    """P14: full splitting conserves pixels and signal like the bounding box
    (Section 4), and a pixel inside one bin goes there whole."""
    rng = np.random.default_rng(4)
    for (h, w, npt, cy, cx) in [(30, 25, 40, 14.6, 12.2), (20, 20, 3, 10.0, 10.0)]:
        m = O.build_matrix(h=h, w=w, pixel_y=1e-4, pixel_x=1e-4, center_y=cy, center_x=cx,
                           dist=DIST, wavelength=WL, npt=npt, split="full")
        x = rng.uniform(0, 5, size=h * w)
        I, W, U = O.integrate(m, x)
        assert abs(U.sum() - h * w) <= 1e-12 * h * w
        assert abs(W.sum() - x.sum()) <= 1e-12 * x.sum()
        s = np.zeros(h * w)
        np.add.at(s, m["pix"], m["coef"])
        assert np.abs(s - 1.0).max() <= 1e-13
        single = np.bincount(m["pix"], minlength=h * w) == 1
        assert np.all(m["coef"][single[m["pix"]]] == 1.0)


def pin_full_rotation(O):
    """P15: turning the detector by 180 degrees about the beam shifts every
    azimuth by pi and leaves every radius alone, so each pixel's full split
    equals that of its twin -- including pixels whose corners straddle the
    +-pi cut on one side and not on the other (reading R13's unwrapping)."""
    for (n, cy, cx, npt) in ((6, 3.0, 3.3, 11), (7, 2.0, 4.6, 13), (5, 1.0, 2.5, 9)):
        def mat(cy_, cx_):
            m = O.build_matrix(h=n, w=n, pixel_y=1e-4, pixel_x=1e-4, center_y=cy_,
                               center_x=cx_, dist=DIST, wavelength=WL, npt=npt, split="full")
            A = np.zeros((npt, n * n))
            A[m["bins"], m["pix"]] = m["coef"]
            return A, m
        A, m = mat(cy, cx)
        B, mb = mat(n - cy, n - cx)
        assert abs(m["pmin"] - mb["pmin"]) <= 1e-18 and abs(m["pmax"] - mb["pmax"]) <= 1e-18
        for p in range(n * n):
            i, j = divmod(p, n)
            q = (n - 1 - i) * n + (n - 1 - j)
            assert np.abs(A[:, p] - B[:, q]).max() <= 1e-9, (n, cy, cx, p, A[:, p], B[:, q])


# ----------------------------------------------------------------------------
# Two-dimensional integration (reading R14)
# ----------------------------------------------------------------------------

CASES_2D = [
    # (h, w, center_y, center_x, npt_rad, npt_azim)
    (5, 6, 2.5, 3.0, 6, 8),
    (6, 6, 3.5, 46.0, 5, 360),     # beam right of the detector: rows across +-pi
    (7, 5, 3.3, 2.2, 7, 12),       # beam inside a pixel, off the pixel grid
    (4, 7, -3.0, 2.5, 4, 36),      # beam above the detector
]


def _dense(m, npix):
    A = np.zeros((m["npt"], npix))
    A[m["bins"], m["pix"]] = m["coef"]
    return A


def _args2d(h, w, cy, cx):
    return dict(h=h, w=w, pixel_y=1e-4, pixel_x=1e-4, center_y=cy, center_x=cx,
                dist=DIST, wavelength=WL)


def pin_2d_marginal(O):
    """P16: summing a two-dimensional split over the azimuthal bins gives
    back the one-dimensional split of the same pixels (the azimuthal shares
    of a pixel add up to one), for the bounding box and for full splitting."""
    for (h, w, cy, cx, nr, na) in CASES_2D:
        args = _args2d(h, w, cy, cx)
        for split in ("bbox", "full"):
            m2 = O.build_matrix2d(npt_rad=nr, npt_azim=na, split=split, **args)
            m1 = O.build_matrix(npt=nr, split=split, **args)
            A2 = _dense(m2, h * w).reshape(na, nr, h * w).sum(axis=0)
            A1 = _dense(m1, h * w)
            assert np.abs(A2 - A1).max() <= 1e-12, (h, w, cy, cx, split)


def pin_2d_azimuth_extent(O):
    """P17: a pixel's azimuthal extent is the range of atan2 over its
    outline (dense sampling of the four edges, unwrapped around the pixel
    centre's azimuth), and the whole circle exactly when the beam lies in
    the closed pixel square."""
    for (h, w, cy, cx, nr, na) in CASES_2D:
        lo, hi, rc = O.pixel_extents(h, w, 1e-4, 1e-4, cy, cx, DIST, WL, "r_m")
        chi_lo, chi_hi, whole = O.azimuth_extents(h, w, 1e-4, 1e-4, cy, cx, lo)
        t = np.linspace(0.0, 1.0, 401)
        for p in range(h * w):
            i, j = divmod(p, w)
            inside = (i <= cy <= i + 1) and (j <= cx <= j + 1)
            assert bool(whole[p]) == inside, (cy, cx, p)
            if inside:
                continue
            xs = np.concatenate([j + t, np.full_like(t, j + 1), j + 1 - t, np.full_like(t, j)])
            ys = np.concatenate([np.full_like(t, i), i + t, np.full_like(t, i + 1), i + 1 - t])
            chi = np.arctan2((ys - cy) * 1e-4, (xs - cx) * 1e-4)
            mid = math.atan2((i + 0.5 - cy) * 1e-4, (j + 0.5 - cx) * 1e-4)
            chi = mid + np.remainder(chi - mid + math.pi, 2 * math.pi) - math.pi
            lo_s, hi_s = chi.min(), chi.max()
            shift = round((chi_lo[p] - lo_s) / (2 * math.pi)) * 2 * math.pi
            assert abs(chi_lo[p] - shift - lo_s) <= 1e-12, (cy, cx, p)
            assert abs(chi_hi[p] - shift - hi_s) <= 1e-12, (cy, cx, p)


def pin_2d_bbox_bruteforce(O):
    """P18: two-dimensional bounding-box coefficients equal the exact
    (rational) area of the box [lo, hi] x [chi_lo, chi_hi] inside each
    (radial bin x azimuthal wedge, repeated every 2 pi) over the box area,
    in row c * npt_rad + a; 1 / npt_azim per wedge for a pixel holding the
    beam."""
    pi = F(math.pi)
    for (h, w, cy, cx, nr, na) in CASES_2D:
        args = _args2d(h, w, cy, cx)
        m = O.build_matrix2d(npt_rad=nr, npt_azim=na, split="bbox", **args)
        lo, hi = m["lo"], m["hi"]
        chi_lo, chi_hi, whole = O.azimuth_extents(h, w, 1e-4, 1e-4, cy, cx, lo)
        pmin, pmax = F(m["pmin"]), F(m["pmax"])
        dr = (pmax - pmin) / nr
        dc = 2 * pi / na
        A = _dense(m, h * w)
        for p in range(h * w):
            l, u = F(float(lo[p])), F(float(hi[p]))
            rad = [max(F(0), min(u, pmin + (a + 1) * dr) - max(l, pmin + a * dr)) / (u - l)
                   for a in range(nr)]
            if whole[p]:
                azi = [F(1, na)] * na
            else:
                cl, ch = F(float(chi_lo[p])), F(float(chi_hi[p]))
                azi = []
                for c in range(na):
                    ov = F(0)
                    for turn in (-1, 0, 1):
                        e0 = -pi + c * dc + 2 * pi * turn
                        ov += max(F(0), min(ch, e0 + dc) - max(cl, e0))
                    azi.append(ov / (ch - cl))
            for c in range(na):
                for a in range(nr):
                    ref = float(rad[a] * azi[c])
                    assert abs(A[c * nr + a, p] - ref) <= 1e-12, (h, w, cy, cx, p, a, c)


def pin_2d_physical_area(O):
    """P19: away from the beam, full two-dimensional splitting follows the
    area in (r, chi) of the pixel's image: Monte Carlo over the pixel square
    with weight 1/r (the Jacobian of (x, y) -> (r, chi)), each point binned by
    its own radius and azimuth."""
    rng = np.random.default_rng(5)
    for (h, w, cy, cx, nr, na, pixels) in ((6, 6, 3.5, 46.0, 8, 360, (18, 19, 21, 12, 5)),
                                           (6, 6, -40.0, -35.0, 9, 720, (0, 7, 14, 35))):
        args = _args2d(h, w, cy, cx)
        m = O.build_matrix2d(npt_rad=nr, npt_azim=na, split="full", **args)
        dr = (m["pmax"] - m["pmin"]) / nr
        dc = 2 * math.pi / na
        for p in pixels:
            i, j = divmod(p, w)
            u = rng.uniform(0, 1, size=(400000, 2))
            x = (j + u[:, 0] - cx) * 1e-4
            y = (i + u[:, 1] - cy) * 1e-4
            r = np.sqrt(x * x + y * y)
            a = np.clip(np.floor((r - m["pmin"]) / dr).astype(int), 0, nr - 1)
            c = np.floor((np.arctan2(y, x) + math.pi) / dc).astype(int) % na
            frac = np.bincount(c * nr + a, weights=1.0 / r, minlength=nr * na)
            frac /= frac.sum()
            sel = m["pix"] == p
            got = np.zeros(nr * na)
            got[m["bins"][sel]] = m["coef"][sel]
            assert np.abs(got - frac).max() < 5e-3, (cy, cx, p)


def pin_2d_full_exact(O):
    """P19b: two-dimensional full splitting (readings R13, R14) equals the
    exact area of each corner quadrilateral inside every (radial bin, wedge)
    rectangle over its whole area, wedges repeated every 2 pi, integrated in
    rational arithmetic by Green's theorem (``exact_rect_area``), pi taken as
    its float64 value; bbox-shaped rows of pixels holding the beam are left
    to the other 2-D pins."""
    pi = F(math.pi)
    for (h, w, cy, cx, nr, na) in CASES_2D:
        m = O.build_matrix2d(npt_rad=nr, npt_azim=na, split="full", **_args2d(h, w, cy, cx))
        corners = O.pixel_corners(h, w, 1e-4, 1e-4, cy, cx, DIST, WL, "r_m")
        pmin, pmax = F(m["pmin"]), F(m["pmax"])
        dr = (pmax - pmin) / nr
        dc = 2 * pi / na
        got = {}
        for b, p, c in zip(m["bins"].tolist(), m["pix"].tolist(), m["coef"].tolist()):
            got[(b, p)] = got.get((b, p), 0.0) + c
        for p in range(h * w):
            if m["lo"][p] == 0.0:
                continue
            quad = [(F(float(a)), F(float(b))) for a, b in corners[p]]
            xs = [q[0] for q in quad]
            ys = [q[1] for q in quad]
            area = exact_rect_area(quad, min(xs), max(xs))
            exact = {}
            k0 = math.floor((min(ys) + pi) / dc) - 1
            k1 = math.ceil((max(ys) + pi) / dc) + 1
            for a in range(nr):
                for k in range(k0, k1 + 1):
                    s = exact_rect_area(quad, pmin + a * dr, pmin + (a + 1) * dr,
                                        -pi + k * dc, -pi + (k + 1) * dc)
                    if s != 0:
                        row = (k % na) * nr + a
                        exact[row] = exact.get(row, F(0)) + s / area
            rows = set(exact) | {b for (b, q) in got if q == p}
            for row in rows:
                ref = float(exact.get(row, 0))
                assert abs(got.get((row, p), 0.0) - ref) <= 1e-12, (h, w, cy, cx, p, row)


def pin_2d_conservation(O):
    """P20: two-dimensional splits conserve pixels and signal (Section 4),
    and a constant image integrates to that constant in every bin with
    pixels."""
    rng = np.random.default_rng(6)
    for (h, w, cy, cx, nr, na) in CASES_2D:
        args = _args2d(h, w, cy, cx)
        for split in ("bbox", "full"):
            m = O.build_matrix2d(npt_rad=nr, npt_azim=na, split=split, **args)
            s = np.zeros(h * w)
            np.add.at(s, m["pix"], m["coef"])
            assert np.abs(s - 1.0).max() <= 1e-13, (h, w, cy, cx, split)
            x = rng.uniform(0, 5, size=h * w)
            I, W, U = O.integrate(m, x)
            assert abs(U.sum() - h * w) <= 1e-12 * h * w
            assert abs(W.sum() - x.sum()) <= 1e-12 * x.sum()
            I, W, U = O.integrate(m, np.full(h * w, 2.5))
            assert np.all(np.abs(I[U > 0] - 2.5) <= 1e-13)


def pin_2d_rotation(O):
    """P21: a half turn of the detector about the beam adds pi to every
    azimuth, so with an even number of wedges each pixel's two-dimensional
    split equals its twin's shifted by half the wedges."""
    for (n, cy, cx, nr, na) in ((6, 3.0, 3.3, 5, 8), (7, 2.0, 4.6, 4, 12)):
        for split in ("bbox", "full"):
            ma = O.build_matrix2d(npt_rad=nr, npt_azim=na, split=split, **_args2d(n, n, cy, cx))
            mb = O.build_matrix2d(npt_rad=nr, npt_azim=na, split=split,
                                  **_args2d(n, n, n - cy, n - cx))
            A = _dense(ma, n * n).reshape(na, nr, n * n)
            B = _dense(mb, n * n).reshape(na, nr, n * n)
            for p in range(n * n):
                i, j = divmod(p, n)
                q = (n - 1 - i) * n + (n - 1 - j)
                diff = np.abs(A[:, :, p] - np.roll(B[:, :, q], -na // 2, axis=0)).max()
                assert diff <= 1e-9, (n, cy, cx, split, p)


def pin_2d_histogram(O):
    """P22: two-dimensional integration without splitting equals numpy's
    weighted and unweighted 2-D histograms of (midpoint radius, midpoint
    azimuth) over [pmin, pmax] x [-pi, pi] (Section 3.3), except pixels
    within rounding of a bin edge."""
    rng = np.random.default_rng(7)
    for (h, w, cy, cx, nr, na) in ((37, 41, 18.8, 20.3, 23, 36), (30, 20, -4.2, 9.7, 17, 72)):
        args = _args2d(h, w, cy, cx)
        m = O.build_matrix2d(npt_rad=nr, npt_azim=na, split="none", **args)
        x = rng.integers(0, 1 << 20, size=h * w).astype(np.float64)
        I, W, U = O.integrate(m, x)
        i, j = np.divmod(np.arange(h * w), w)
        xc, yc = (j + 0.5 - cx) * 1e-4, (i + 0.5 - cy) * 1e-4
        chi = np.arctan2(yc, xc)
        r = m["centre"]
        rngs = [[m["pmin"], m["pmax"]], [-math.pi, math.pi]]
        hu = np.histogram2d(r, chi, bins=[nr, na], range=rngs)[0]
        hw = np.histogram2d(r, chi, bins=[nr, na], range=rngs, weights=x)[0]
        fr = (r - m["pmin"]) / ((m["pmax"] - m["pmin"]) / nr)
        fc = (chi + math.pi) / (2 * math.pi / na)
        # the range ends are no bin edges: the extreme pixels sit on them
        inner = (np.round(fr) > 0) & (np.round(fr) < nr)
        near = ((np.abs(fr - np.round(fr)) < 1e-9) & inner) | (np.abs(fc - np.round(fc)) < 1e-9)
        assert not near.any()
        assert np.array_equal(U.reshape(na, nr), hu.T)
        assert np.allclose(W.reshape(na, nr), hw.T, rtol=1e-15, atol=0)


ALL_PINS = [pin_extents_exact, pin_bbox_bruteforce, pin_results_exact,
            pin_nosplit_histogram, pin_naive_mean, pin_conservation, pin_unit_weights,
            pin_constant_image, pin_symmetry, pin_scipy_csr, pin_adjoint, pin_kahan,
            pin_closed_forms, pin_bbox_clipped, pin_correction, pin_correction_norm,
            pin_default_range, pin_positions,
            pin_full_exact, pin_full_physical_area, pin_full_conservation,
            pin_full_rotation, pin_2d_marginal, pin_2d_azimuth_extent,
            pin_2d_bbox_bruteforce, pin_2d_physical_area, pin_2d_full_exact, pin_2d_conservation,
            pin_2d_rotation, pin_2d_histogram]
