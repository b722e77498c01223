"""FP64 CPU oracle: azimuthal integration with pixel splitting, 1-D and 2-D.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It is written from
the paper (Kieffer & Ashiotis, "PyFAI: a Python library for high performance
azimuthal integration on GPU", EuroSciPy 2014) and shares no code, table or
helper with the HIP library.

What is computed (each function cites the passage it follows):

* per-pixel radial coordinate and its extent over the pixel area
  (Section 3, coordinate list; Section 3.1 test case; Section 4.1),
* the pixel-to-bin coefficients of bounding-box splitting (Section 4.1), of
  full pixel splitting (Section 4.2), or of plain histogramming (Section
  3.3), and their two-dimensional (radius x azimuth) forms (Section 4),
* the per-pixel correction map (Section 6.4, "Kernel timings"),
* the weighted histogram W, the unweighted histogram U and their ratio
  I = W / U (Section 3.3; Section 5.2 states the same sums as a sparse
  matrix-vector product),
* the adjoint of I (and W) with respect to the corrected image,
* Kahan-compensated float32 summation (Section 5.2.2).

The integration itself reaches exactly, up to the order of the additions,
the plain definition W_b = sum_p A_bp x_p, U_b = sum_p A_bp: the
scatter-to-gather rewrite and the CSR storage of Section 5.2 only reorder
these sums.  So the oracle is that definition: a forward scatter over pixels
with the sums carried in extended precision (numpy.longdouble, a 64-bit
mantissa on x86-64), rounded once to float64.

Readings of passages the paper leaves open (numbered as in the design notes):

R1  pixel (i, j) covers [j, j+1] x [i, i+1] in pixel units; the beam centre
    is given in the same units.
R2  the bounding box of Section 4.1 spans the pixel's true radial extent:
    ``hi`` is the largest corner distance, ``lo`` the distance to the nearest
    point of the closed pixel square (0 when the centre lies inside it).
R3  bins are uniform over an explicit [pmin, pmax]; by default
    [min lo, max hi] (split) or [min centre, max centre] (no split); the
    last bin is closed.
R4  boxes partly outside the range are clipped; the weights stay normalised
    by the full box width, so the part outside is dropped.
R5  a box [fl, fh] in fractional-bin units covers bins floor(fl) ..
    ceil(fh) - 1, so no zero coefficient is ever produced.
R6  every inner bin receives 1 / (fh - fl): the overlap of a whole bin over
    the box width, which equals an even split of what the two outer bins
    leave, for uniform bins.
R7  an empty bin (U = 0) yields the caller's ``empty`` value (default 0.0).
R8  the azimuth chi = tan^-1(y/x) of the coordinate list is atan2(y, x) in
    (-pi, pi], x along pixel columns, y along pixel rows, both measured
    from the beam in metres.
R9  units: r in m or mm, 2theta in rad or deg, q in 1/nm.
R13 full pixel splitting (Section 4.2): the four pixel corners are mapped
    to (pos0, pos1) = (output unit, azimuth chi = atan2(y, x)), the edges
    between them taken as straight lines; bin b receives the area of that
    quadrilateral lying in the bin's pos0 slab over the quadrilateral's
    whole area.  The corner azimuths are unwrapped to within pi of corner 0;
    a pixel whose square holds the beam centre (lo == 0), where the
    quadrilateral is undefined, falls back to the bounding box.
R14 two-dimensional integration: npt_azim equal wedges of the periodic
    circle [-pi, pi) times the radial bins; bin (radial a, azimuthal c) is
    row c * npt_rad + a.  The bounding box becomes [lo, hi] x [chi_lo,
    chi_hi], the azimuthal extent being the range of the corner azimuths
    unwrapped to corner 0 (the whole circle for a pixel holding the beam);
    its share of a bin is the product of the radial and azimuthal shares.
    Full splitting clips the corner quadrilateral to the bin's rectangle,
    the wedge repeated every 2 pi.
"""
from __future__ import annotations

import math

import numpy as np

UNITS = ("r_m", "r_mm", "2th_rad", "2th_deg", "q_nm")
SPLITS = ("none", "bbox", "full")

__all__ = [
    "UNITS", "SPLITS", "unit_of_radius", "pixel_extents", "pixel_extents_loop",
    "default_range", "bbox_entries", "bbox_entries_loop", "nosplit_entries",
    "pixel_corners", "full_entries", "polygon_area", "clip_slab",
    "entries_to_csr", "build_matrix", "correct", "corner_azimuth", "azimuth_extents",
    "azimuth_entries_loop", "bbox2d_entries", "full2d_entries", "nosplit2d_entries", "build_matrix2d", "integrate", "integrate_loop",
    "integrate_vjp", "kahan_sum_f32", "positions", "correction_norm",
]


# ----------------------------------------------------------------------------
# Geometry (Section 3 coordinate list; Section 3.1; Section 4.1)
# ----------------------------------------------------------------------------

def unit_of_radius(r, unit: str, dist: float, wavelength: float):
    """Map a radius in metres to the output coordinate (Section 3 list).

    2theta = atan(r / d); q = 4 pi sin(2theta / 2) / lambda, with lambda in
    nm so that q is in 1/nm (reading R9).  Every map is monotone
    non-decreasing in r, so a radial interval maps to an interval.
    """
    if unit == "r_m":
        return r
    if unit == "r_mm":
        return r * 1e3
    tth = np.arctan(r / dist)
    if unit == "2th_rad":
        return tth
    if unit == "2th_deg":
        return tth * (180.0 / math.pi)
    if unit == "q_nm":
        return (4.0 * math.pi) * np.sin(tth / 2.0) / (wavelength * 1e9)
    raise ValueError(f"unknown unit {unit!r}")


def pixel_extents(h, w, pixel_y, pixel_x, center_y, center_x, dist, wavelength,
                  unit="r_m"):
    """Per-pixel (lo, hi, centre) of the output coordinate, row-major (h*w,).

    The radius of a point is r = sqrt(x^2 + y^2) measured from the beam
    centre (Section 3.1).  ``hi`` is the largest of the four corner radii and
    ``lo`` the radius of the nearest point of the pixel square (reading R2);
    the centre value is the radius of the pixel midpoint.
    """
    i = np.arange(h, dtype=np.int64)[:, None]
    j = np.arange(w, dtype=np.int64)[None, :]
    x0 = (j - center_x) * pixel_x
    x1 = ((j + 1) - center_x) * pixel_x
    y0 = (i - center_y) * pixel_y
    y1 = ((i + 1) - center_y) * pixel_y
    s00 = x0 * x0 + y0 * y0
    s01 = x1 * x1 + y0 * y0
    s10 = x0 * x0 + y1 * y1
    s11 = x1 * x1 + y1 * y1
    hi = np.sqrt(np.maximum(np.maximum(s00, s01), np.maximum(s10, s11)))
    # nearest point of [j, j+1] x [i, i+1] to the centre, per axis
    ex = np.maximum(np.maximum(j - center_x, center_x - (j + 1)), 0.0) * pixel_x
    ey = np.maximum(np.maximum(i - center_y, center_y - (i + 1)), 0.0) * pixel_y
    lo = np.sqrt(ex * ex + ey * ey)
    xc = ((j + 0.5) - center_x) * pixel_x
    yc = ((i + 0.5) - center_y) * pixel_y
    rc = np.sqrt(xc * xc + yc * yc)
    lo, hi, rc = (np.broadcast_to(a, (h, w)).reshape(-1) for a in (lo, hi, rc))
    f = lambda r: np.asarray(unit_of_radius(r, unit, dist, wavelength), dtype=np.float64)
    return f(lo), f(hi), f(rc)


def pixel_extents_loop(h, w, pixel_y, pixel_x, center_y, center_x, dist,
                       wavelength, unit="r_m"):
    """Pure-Python form of :func:`pixel_extents` for small images."""
    n = h * w
    lo, hi, rc = [0.0] * n, [0.0] * n, [0.0] * n
    for i in range(h):
        for j in range(w):
            p = i * w + j
            best = 0.0
            for a in (0, 1):
                for b in (0, 1):
                    x = ((j + a) - center_x) * pixel_x
                    y = ((i + b) - center_y) * pixel_y
                    best = max(best, x * x + y * y)
            hi[p] = math.sqrt(best)
            ex = max(j - center_x, center_x - (j + 1), 0.0) * pixel_x
            ey = max(i - center_y, center_y - (i + 1), 0.0) * pixel_y
            lo[p] = math.sqrt(ex * ex + ey * ey)
            xc = ((j + 0.5) - center_x) * pixel_x
            yc = ((i + 0.5) - center_y) * pixel_y
            rc[p] = math.sqrt(xc * xc + yc * yc)
    f = lambda v: np.asarray(unit_of_radius(np.asarray(v, dtype=np.float64), unit,
                                            dist, wavelength), dtype=np.float64)
    return f(lo), f(hi), f(rc)


def default_range(lo, hi, centre, split):
    """Reading R3: [min lo, max hi] with splitting, [min c, max c] without."""
    if split in ("bbox", "full"):
        return float(np.min(lo)), float(np.max(hi))
    return float(np.min(centre)), float(np.max(centre))


def positions(npt, pmin, pmax):
    """Bin centres pmin + (b + 0.5) * delta, delta = (pmax - pmin) / npt."""
    delta = (pmax - pmin) / npt
    return pmin + (np.arange(npt) + 0.5) * delta


# ----------------------------------------------------------------------------
# Pixel-to-bin coefficients (Section 4.1 bounding box; Section 3.3 histogram)
# ----------------------------------------------------------------------------

def bbox_entries_loop(lo, hi, npt, pmin, pmax):
    """Bounding-box splitting, one pixel at a time (Section 4.1).

    The box [lo, hi] is mapped to fractional-bin units [fl, fh]; a box inside
    one bin gives that bin its whole weight; otherwise the two outermost bins
    get the part of the box they hold, and every inner bin an equal share
    (readings R4-R6).  Returns (pixel, bin, coefficient) in scatter order.
    """
    delta = (pmax - pmin) / npt
    pix, bins, coef = [], [], []
    for p in range(len(lo)):
        fl = (float(lo[p]) - pmin) / delta
        fh = (float(hi[p]) - pmin) / delta
        if fh == fl:
            if 0.0 <= fl <= npt:
                pix.append(p); bins.append(min(math.floor(fl), npt - 1)); coef.append(1.0)
            continue
        flc = max(fl, 0.0)
        fhc = min(fh, float(npt))
        if fhc <= flc:
            continue
        width = fh - fl
        b0 = math.floor(flc)
        b1 = math.ceil(fhc) - 1
        if b0 == b1:
            pix.append(p); bins.append(b0); coef.append((fhc - flc) / width)
            continue
        pix.append(p); bins.append(b0); coef.append(((b0 + 1) - flc) / width)
        for b in range(b0 + 1, b1):
            pix.append(p); bins.append(b); coef.append(1.0 / width)
        pix.append(p); bins.append(b1); coef.append((fhc - b1) / width)
    return (np.asarray(pix, dtype=np.int64), np.asarray(bins, dtype=np.int64),
            np.asarray(coef, dtype=np.float64))


def bbox_entries(lo, hi, npt, pmin, pmax):
    """Vectorised form of :func:`bbox_entries_loop` (same arithmetic)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    delta = (pmax - pmin) / npt
    fl = (lo - pmin) / delta
    fh = (hi - pmin) / delta
    degen = fh == fl
    flc = np.maximum(fl, 0.0)
    fhc = np.minimum(fh, float(npt))
    keep = (~degen) & (fhc > flc)
    width = fh - fl
    with np.errstate(invalid="ignore", divide="ignore"):
        b0 = np.floor(flc)
        b1 = np.ceil(fhc) - 1.0
    pid = np.arange(lo.size, dtype=np.int64)
    out_p, out_b, out_c = [], [], []
    # degenerate boxes: a single full-weight entry
    dmask = degen & (fl >= 0.0) & (fl <= npt)
    if dmask.any():
        out_p.append(pid[dmask])
        out_b.append(np.minimum(np.floor(fl[dmask]), npt - 1).astype(np.int64))
        out_c.append(np.ones(int(dmask.sum())))
    if keep.any():
        kp = pid[keep]
        kfl, kfh, kw = flc[keep], fhc[keep], width[keep]
        kb0 = b0[keep].astype(np.int64)
        kb1 = b1[keep].astype(np.int64)
        span = int((kb1 - kb0).max()) + 1
        single = kb0 == kb1
        for k in range(span):
            b = kb0 + k
            m = b <= kb1
            if not m.any():
                break
            c = np.where(single, (kfh - kfl) / kw,
                         np.where(k == 0, ((kb0 + 1) - kfl) / kw,
                                  np.where(b == kb1, (kfh - kb1) / kw, 1.0 / kw)))
            out_p.append(kp[m]); out_b.append(b[m]); out_c.append(c[m])
    if not out_p:
        z = np.zeros(0, dtype=np.int64)
        return z, z.copy(), np.zeros(0)
    return np.concatenate(out_p), np.concatenate(out_b), np.concatenate(out_c)


_atan2 = np.frompyfunc(math.atan2, 2, 1)


def corner_azimuth(y, x):
    """Azimuth chi = atan2(y, x) in (-pi, pi] (Section 3 coordinate list;
    reading R8), evaluated by the C library's atan2 so that the bin a corner
    falls in is decided by the same rounding wherever the plan is built."""
    return np.asarray(_atan2(y, x), dtype=np.float64)


def pixel_corners(h, w, pixel_y, pixel_x, center_y, center_x, dist, wavelength, unit="r_m"):
    """Corner coordinates (pos0, pos1) of every pixel, shape (h*w, 4, 2), in
    the order (j, i), (j+1, i), (j+1, i+1), (j, i+1): pos0 is the output unit
    of the corner radius, pos1 its azimuth atan2(y, x) unwrapped to within pi
    of the first corner (reading R13)."""
    gi = np.arange(h + 1, dtype=np.int64)[:, None]
    gj = np.arange(w + 1, dtype=np.int64)[None, :]
    x = np.broadcast_to((gj - center_x) * pixel_x, (h + 1, w + 1))
    y = np.broadcast_to((gi - center_y) * pixel_y, (h + 1, w + 1))
    r = np.sqrt(x * x + y * y)
    pos0 = unit_of_radius(r, unit, dist, wavelength)
    chi = corner_azimuth(y, x)
    out = np.empty((h, w, 4, 2))
    for k, (a, b) in enumerate(((0, 0), (1, 0), (1, 1), (0, 1))):
        out[:, :, k, 0] = pos0[b:b + h, a:a + w]
        out[:, :, k, 1] = chi[b:b + h, a:a + w]
    chi0 = out[:, :, :1, 1]
    turns = np.round((chi0 - out[:, :, :, 1]) / (2.0 * math.pi))
    out[:, :, :, 1] = out[:, :, :, 1] + turns * (2.0 * math.pi)
    return out.reshape(h * w, 4, 2)


def clip_slab(poly, x0, x1):
    """The part of polygon `poly` (list of (x, y)) with x0 <= x <= x1, by
    clipping against the two vertical lines in turn (Sutherland-Hodgman).
    Works on floats or Fractions alike."""
    def clip(pts, inside, cross):
        out = []
        n = len(pts)
        for k in range(n):
            p, q = pts[k], pts[(k + 1) % n]
            pin, qin = inside(p), inside(q)
            if pin:
                out.append(p)
            if pin != qin:
                out.append(cross(p, q))
        return out

    def at(xc):
        def cross(p, q):
            t = (xc - p[0]) / (q[0] - p[0])
            return (xc, p[1] + t * (q[1] - p[1]))
        return cross

    pts = clip(list(poly), lambda p: p[0] >= x0, at(x0))
    if not pts:
        return []
    return clip(pts, lambda p: p[0] <= x1, at(x1))


def polygon_area(poly):
    """Absolute shoelace area."""
    s = 0
    n = len(poly)
    for k in range(n):
        (x0, y0), (x1, y1) = poly[k], poly[(k + 1) % n]
        s += x0 * y1 - x1 * y0
    return abs(s) / 2


def full_entries(corners, lo, hi, npt, pmin, pmax):
    """Full pixel splitting (Section 4.2, reading R13), one pixel at a time:
    bin b gets area(quadrilateral within bin b's slab) / area(quadrilateral).
    Pixels holding the beam centre use the bounding box of Section 4.1."""
    delta = (pmax - pmin) / npt
    pix, bins, coef = [], [], []
    for p in range(len(corners)):
        if float(lo[p]) == 0.0:
            bp, bb, bc = bbox_entries_loop(lo[p:p + 1], hi[p:p + 1], npt, pmin, pmax)
            pix += [p] * len(bb)
            bins += bb.tolist()
            coef += bc.tolist()
            continue
        xs = [float(c[0]) for c in corners[p]]
        fl = (min(xs) - pmin) / delta
        fh = (max(xs) - pmin) / delta
        # areas are taken relative to the first corner (translation leaves
        # them unchanged and keeps the products small)
        x0, y0 = float(corners[p][0][0]), float(corners[p][0][1])
        quad = [(float(c[0]) - x0, float(c[1]) - y0) for c in corners[p]]
        area = polygon_area(quad)
        if area == 0.0 or fh == fl:
            continue
        b0 = max(math.floor(fl), 0)
        b1 = min(math.ceil(fh) - 1, npt - 1)
        for b in range(b0, b1 + 1):
            e0 = (pmin + b * delta) - x0
            e1 = (pmin + (b + 1) * delta) - x0
            c = polygon_area(clip_slab(quad, e0, e1)) / area
            if c > 0.0:
                pix.append(p); bins.append(b); coef.append(c)
    return (np.asarray(pix, dtype=np.int64), np.asarray(bins, dtype=np.int64),
            np.asarray(coef, dtype=np.float64))


def nosplit_entries(centre, npt, pmin, pmax):
    """No splitting (Section 3.3): each pixel goes whole to the bin holding
    its centre; the last bin is closed (reading R3)."""
    c = np.asarray(centre, dtype=np.float64)
    delta = (pmax - pmin) / npt
    fc = (c - pmin) / delta
    m = (fc >= 0.0) & (fc <= npt)
    pid = np.arange(c.size, dtype=np.int64)[m]
    b = np.minimum(np.floor(fc[m]), npt - 1).astype(np.int64)
    return pid, b, np.ones(pid.size)


# ----------------------------------------------------------------------------
# Two-dimensional integration (Section 4; reading R14)
# ----------------------------------------------------------------------------

def azimuth_extents(h, w, pixel_y, pixel_x, center_y, center_x, lo):
    """Azimuthal extent [chi_lo, chi_hi] of every pixel square (reading R14).

    Along a straight edge that misses the beam the azimuth is monotone, so
    the extremes over the square sit at its corners: min and max of the four
    corner azimuths, unwrapped to within pi of the first corner.  A pixel
    whose square holds the beam (lo == 0) covers the whole circle: flagged
    in ``whole`` (its chi_lo, chi_hi are then meaningless)."""
    c = pixel_corners(h, w, pixel_y, pixel_x, center_y, center_x, 1.0, 1.0, "r_m")
    chi = c[:, :, 1]
    whole = np.asarray(lo, dtype=np.float64).reshape(-1) == 0.0
    return chi.min(axis=1), chi.max(axis=1), whole


def azimuth_entries_loop(chi_lo, chi_hi, whole, npt_azim):
    """Azimuthal shares of every pixel (reading R14), one pixel at a time.

    The circle [-pi, pi) is cut into npt_azim equal bins and is periodic: an
    extent in bin units [gl, gh] covers unwrapped bins floor(gl) ..
    ceil(gh) - 1, bin k meaning bin k mod npt_azim; the outer two get their
    overlap over (gh - gl), the inner ones 1 / (gh - gl), as along the
    radius (readings R5, R6).  A pixel holding the beam gives 1 / npt_azim
    to every bin."""
    delta = (2.0 * math.pi) / npt_azim
    pix, bins, coef = [], [], []
    for p in range(len(chi_lo)):
        if whole[p]:
            for k in range(npt_azim):
                pix.append(p); bins.append(k); coef.append(1.0 / npt_azim)
            continue
        gl = (float(chi_lo[p]) + math.pi) / delta
        gh = (float(chi_hi[p]) + math.pi) / delta
        width = gh - gl
        k0 = math.floor(gl)
        k1 = math.ceil(gh) - 1
        if width == 0.0:
            k1 = k0
        for k in range(k0, max(k1, k0) + 1):
            if k0 == k1:
                c = 1.0
            elif k == k0:
                c = ((k0 + 1) - gl) / width
            elif k == k1:
                c = (gh - k1) / width
            else:
                c = 1.0 / width
            if c > 0.0:
                pix.append(p); bins.append(k % npt_azim); coef.append(c)
    return (np.asarray(pix, dtype=np.int64), np.asarray(bins, dtype=np.int64),
            np.asarray(coef, dtype=np.float64))


def bbox2d_entries(rad, azi, npt_rad):
    """Two-dimensional bounding box (Section 4.1 in two dimensions, reading
    R14): the share of the box in (radial bin a, azimuthal bin c) is the
    product of its radial and azimuthal shares, stored in row
    c * npt_rad + a.  ``rad`` and ``azi`` are (pix, bin, coef) triples."""
    rp, rb, rc = rad
    ap, ab, ac = azi
    order_r = np.argsort(rp, kind="stable")
    order_a = np.argsort(ap, kind="stable")
    rp, rb, rc = rp[order_r], rb[order_r], rc[order_r]
    ap, ab, ac = ap[order_a], ab[order_a], ac[order_a]
    npix = int(max(rp.max(initial=-1), ap.max(initial=-1))) + 1
    ncount = np.bincount(ap, minlength=npix)
    astart = np.concatenate(([0], np.cumsum(ncount)))
    reps = ncount[rp]
    pix = np.repeat(rp, reps)
    rbin = np.repeat(rb, reps)
    rcoef = np.repeat(rc, reps)
    # index of the azimuthal entry paired with each repeated radial entry
    first = np.repeat(astart[rp], reps)
    offs = np.arange(pix.size) - np.repeat(np.cumsum(reps) - reps, reps)
    k = first + offs
    return pix, ab[k] * npt_rad + rbin, rcoef * ac[k]


def nosplit2d_entries(h, w, pixel_y, pixel_x, center_y, center_x, centre, npt_rad, npt_azim,
                      pmin, pmax):
    """Two-dimensional histogram without splitting (Section 3.3 in two
    dimensions, readings R3, R8, R14): each pixel goes whole to the bin of
    its midpoint's radius and azimuth; the azimuth wedge is periodic."""
    rp, rb, _ = nosplit_entries(centre, npt_rad, pmin, pmax)
    i = np.arange(h, dtype=np.int64)[:, None]
    j = np.arange(w, dtype=np.int64)[None, :]
    xc = np.broadcast_to(((j + 0.5) - center_x) * pixel_x, (h, w)).reshape(-1)
    yc = np.broadcast_to(((i + 0.5) - center_y) * pixel_y, (h, w)).reshape(-1)
    chi = corner_azimuth(yc[rp], xc[rp])
    dchi = (2.0 * math.pi) / npt_azim
    c = np.floor((chi + math.pi) / dchi).astype(np.int64) % npt_azim
    return rp, c * npt_rad + rb, np.ones(rp.size)


def full2d_entries(corners, lo, hi, npt_rad, npt_azim, pmin, pmax):
    """Full pixel splitting in two dimensions (Section 4.2, readings R13,
    R14): bin (a, c) gets area(quadrilateral within radial slab a and
    azimuthal slab c, the latter repeated every 2 pi) / area(quadrilateral).
    Pixels holding the beam use the two-dimensional bounding box."""
    delta = (pmax - pmin) / npt_rad
    dchi = (2.0 * math.pi) / npt_azim
    pix, bins, coef = [], [], []

    def swap(poly):
        return [(q[1], q[0]) for q in poly]

    for p in range(len(corners)):
        if float(lo[p]) == 0.0:
            rad = bbox_entries_loop(lo[p:p + 1], hi[p:p + 1], npt_rad, pmin, pmax)
            azi = azimuth_entries_loop([0.0], [0.0], [True], npt_azim)
            bp, bb, bc = bbox2d_entries(rad, azi, npt_rad)
            pix += [p] * len(bb)
            bins += bb.tolist()
            coef += bc.tolist()
            continue
        xs = [float(c[0]) for c in corners[p]]
        ys = [float(c[1]) for c in corners[p]]
        fl = (min(xs) - pmin) / delta
        fh = (max(xs) - pmin) / delta
        gl = (min(ys) + math.pi) / dchi
        gh = (max(ys) + math.pi) / dchi
        x0, y0 = xs[0], ys[0]
        quad = [(xs[k] - x0, ys[k] - y0) for k in range(4)]
        area = polygon_area(quad)
        if area == 0.0 or fh == fl:
            continue
        b0 = max(math.floor(fl), 0)
        b1 = min(math.ceil(fh) - 1, npt_rad - 1)
        k0 = math.floor(gl)
        k1 = max(math.ceil(gh) - 1, k0)
        for b in range(b0, b1 + 1):
            e0 = (pmin + b * delta) - x0
            e1 = (pmin + (b + 1) * delta) - x0
            slab = clip_slab(quad, e0, e1)
            if not slab:
                continue
            for k in range(k0, k1 + 1):
                t0 = (-math.pi + k * dchi) - y0
                t1 = (-math.pi + (k + 1) * dchi) - y0
                c = polygon_area(clip_slab(swap(slab), t0, t1)) / area
                if c > 0.0:
                    pix.append(p); bins.append((k % npt_azim) * npt_rad + b); coef.append(c)
    return (np.asarray(pix, dtype=np.int64), np.asarray(bins, dtype=np.int64),
            np.asarray(coef, dtype=np.float64))


def build_matrix2d(h, w, pixel_y, pixel_x, center_y, center_x, dist, wavelength,
                   npt_rad, npt_azim, unit="r_m", split="bbox", range_=None):
    """Geometry -> coefficients -> CSR for two-dimensional integration: rows
    c * npt_rad + a for azimuthal bin c of [-pi, pi) and radial bin a of the
    radial range (readings R3, R14).  Splits "none", "bbox" and "full"."""
    lo, hi, rc = pixel_extents(h, w, pixel_y, pixel_x, center_y, center_x, dist,
                               wavelength, unit)
    pmin, pmax = default_range(lo, hi, rc, split) if range_ is None else map(float, range_)
    if not pmax > pmin:
        raise ValueError("empty integration range")
    npt = npt_rad * npt_azim
    if split == "none":
        ent = nosplit2d_entries(h, w, pixel_y, pixel_x, center_y, center_x, rc, npt_rad,
                                npt_azim, pmin, pmax)
    elif split == "bbox":
        rad = bbox_entries(lo, hi, npt_rad, pmin, pmax)
        chi_lo, chi_hi, whole = azimuth_extents(h, w, pixel_y, pixel_x, center_y, center_x, lo)
        azi = azimuth_entries_loop(chi_lo, chi_hi, whole, npt_azim)
        ent = bbox2d_entries(rad, azi, npt_rad)
    elif split == "full":
        corners = pixel_corners(h, w, pixel_y, pixel_x, center_y, center_x, dist, wavelength,
                                unit)
        ent = full2d_entries(corners, lo, hi, npt_rad, npt_azim, pmin, pmax)
    else:
        raise ValueError(f"unknown two-dimensional split {split!r}")
    indptr, indices, data = entries_to_csr(*ent, npt)
    dchi = (2.0 * math.pi) / npt_azim
    return dict(npt=npt, npt_rad=npt_rad, npt_azim=npt_azim, npix=h * w, pmin=pmin,
                pmax=pmax, lo=lo, hi=hi, centre=rc, pix=ent[0], bins=ent[1], coef=ent[2],
                indptr=indptr, indices=indices, data=data,
                positions=positions(npt_rad, pmin, pmax),
                azimuths=-math.pi + (np.arange(npt_azim) + 0.5) * dchi)


def entries_to_csr(pix, bins, coef, npt):
    """CSR of A (rows = bins, columns = pixels) with ascending pixel ids in a
    row, the layout scipy.sparse.csr_matrix accepts (Section 5.2.1)."""
    order = np.lexsort((pix, bins))
    indptr = np.zeros(npt + 1, dtype=np.int64)
    np.add.at(indptr, bins + 1, 1)
    return np.cumsum(indptr), pix[order].astype(np.int64), coef[order]


def build_matrix(h, w, pixel_y, pixel_x, center_y, center_x, dist, wavelength,
                 npt, unit="r_m", split="bbox", range_=None, loop=False):
    """Geometry -> coefficients -> CSR; returns a dict of plain arrays."""
    ext = pixel_extents_loop if loop else pixel_extents
    lo, hi, rc = ext(h, w, pixel_y, pixel_x, center_y, center_x, dist, wavelength, unit)
    pmin, pmax = default_range(lo, hi, rc, split) if range_ is None else map(float, range_)
    if not pmax > pmin:
        raise ValueError("empty integration range")
    if split == "bbox":
        ent = (bbox_entries_loop if loop else bbox_entries)(lo, hi, npt, pmin, pmax)
    elif split == "full":
        corners = pixel_corners(h, w, pixel_y, pixel_x, center_y, center_x, dist, wavelength,
                                unit)
        ent = full_entries(corners, lo, hi, npt, pmin, pmax)
    elif split == "none":
        ent = nosplit_entries(rc, npt, pmin, pmax)
    else:
        raise ValueError(f"unknown split {split!r}")
    indptr, indices, data = entries_to_csr(*ent, npt)
    return dict(npt=npt, npix=h * w, pmin=pmin, pmax=pmax, lo=lo, hi=hi, centre=rc,
                pix=ent[0], bins=ent[1], coef=ent[2],
                indptr=indptr, indices=indices, data=data,
                positions=positions(npt, pmin, pmax))


# ----------------------------------------------------------------------------
# Per-frame computation
# ----------------------------------------------------------------------------

def correction_norm(flat=None, solid=None, polar=None):
    """The divisor of the correction map of Section 6.4, (flat * solid) *
    polar, formed left to right; absent arrays drop out, and None is
    returned when all three are absent."""
    norm = None
    for arr in (flat, solid, polar):
        if arr is None:
            continue
        a = np.asarray(arr, dtype=np.float64).reshape(-1)
        norm = a if norm is None else norm * a
    return norm


def correct(raw, dark=None, flat=None, solid=None, polar=None):
    """Correction map of Section 6.4: x = (raw - dark) / ((flat*solid)*polar).

    Missing arrays act as identity; the products are formed left to right.
    """
    x = np.asarray(raw).astype(np.float64).reshape(-1)
    if dark is not None:
        x = x - np.asarray(dark, dtype=np.float64).reshape(-1)
    norm = correction_norm(flat, solid, polar)
    if norm is not None:
        x = x / norm
    return x


def integrate(m, x, empty=0.0):
    """W_b = sum_p A_bp x_p, U_b = sum_p A_bp, I_b = W_b / U_b (Section 3.3).

    ``m`` is a dict holding the coefficient triplets ``pix``, ``bins``,
    ``coef`` and ``npt``.  Products are float64; their sums are carried in
    numpy.longdouble and rounded once.  An empty bin gives ``empty`` (R7).
    """
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    npt = int(m["npt"])
    pix, bins, coef = m["pix"], m["bins"], np.asarray(m["coef"], dtype=np.float64)
    prod = (coef * x[pix]).astype(np.longdouble)
    W = np.zeros(npt, dtype=np.longdouble)
    U = np.zeros(npt, dtype=np.longdouble)
    np.add.at(W, bins, prod)
    np.add.at(U, bins, coef.astype(np.longdouble))
    W = W.astype(np.float64)
    U = U.astype(np.float64)
    I = np.full(npt, float(empty))
    nz = U != 0.0
    I[nz] = W[nz] / U[nz]
    return I, W, U


def integrate_loop(m, x, empty=0.0):
    """Pure-Python form of :func:`integrate`, exact sums via math.fsum."""
    npt = int(m["npt"])
    wterms = [[] for _ in range(npt)]
    uterms = [[] for _ in range(npt)]
    for p, b, c in zip(m["pix"].tolist(), m["bins"].tolist(), m["coef"].tolist()):
        wterms[b].append(c * float(x[p]))
        uterms[b].append(c)
    W = np.array([math.fsum(t) for t in wterms])
    U = np.array([math.fsum(t) for t in uterms])
    I = np.array([W[b] / U[b] if U[b] != 0.0 else float(empty) for b in range(npt)])
    return I, W, U


def integrate_vjp(m, U, grad_I=None, grad_W=None, norm=None):
    """Adjoint of the forward map with respect to the corrected image.

    dI_b/dx_p = A_bp / U_b and dW_b/dx_p = A_bp, so with upstream gradients
    g_I and g_W:  gx_p = sum_b A_bp (g_I,b / U_b + g_W,b).  Empty bins give a
    constant and contribute nothing.  With a correction map, the gradient
    with respect to the raw counts is gx / norm (Section 6.4 map is affine in
    raw).
    """
    npt, npix = int(m["npt"]), int(m["npix"])
    U = np.asarray(U, dtype=np.float64)
    v = np.zeros(npt, dtype=np.float64)
    if grad_I is not None:
        gI = np.asarray(grad_I, dtype=np.float64)
        nz = U != 0.0
        v[nz] = gI[nz] / U[nz]
    if grad_W is not None:
        v = v + np.asarray(grad_W, dtype=np.float64)
    pix, bins, coef = m["pix"], m["bins"], np.asarray(m["coef"], dtype=np.float64)
    gx = np.zeros(npix, dtype=np.longdouble)
    np.add.at(gx, pix, (coef * v[bins]).astype(np.longdouble))
    gx = gx.astype(np.float64)
    if norm is not None:
        gx = gx / np.asarray(norm, dtype=np.float64).reshape(-1)
    return gx


def kahan_sum_f32(values):
    """Kahan compensated summation carried entirely in float32 (Section 5.2.2)."""
    s = np.float32(0.0)
    c = np.float32(0.0)
    for v in np.asarray(values, dtype=np.float32):
        y = np.float32(v - c)
        t = np.float32(s + y)
        c = np.float32(np.float32(t - s) - y)
        s = t
    return s
