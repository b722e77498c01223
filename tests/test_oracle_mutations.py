"""Planted mistakes in the oracle (CPU only): each must fail at least one pin.

Every mutant below is a plausible slip in writing the oracle -- a dropped
term, a wrong sign, an off-by-one bin, a transposed operand, a wrong
normalisation.  The test patches one oracle function at a time and checks
that the pins in ``tests/pins.py`` notice.
"""
import math

import numpy as np
import pytest

from oracle import azint_oracle as O
from tests import pins

_orig = {name: getattr(O, name) for name in
         ("pixel_extents", "bbox_entries", "nosplit_entries", "integrate",
          "integrate_vjp", "kahan_sum_f32", "unit_of_radius", "correct",
          "pixel_corners", "full_entries", "polygon_area", "corner_azimuth",
          "azimuth_entries_loop", "bbox2d_entries", "full2d_entries", "azimuth_extents",
          "nosplit2d_entries", "default_range", "positions", "correction_norm",
          "clip_slab")}


def _corners_no_unwrap(h, w, pixel_y, pixel_x, center_y, center_x, dist, wavelength,
                       unit="r_m"):
    # azimuths left in (-pi, pi]: a pixel across the cut becomes a bow tie
    i = np.arange(h)[:, None]
    j = np.arange(w)[None, :]
    out = np.empty((h, w, 4, 2))
    for k, (a, b) in enumerate(((0, 0), (1, 0), (1, 1), (0, 1))):
        x = ((j + a) - center_x) * pixel_x
        y = ((i + b) - center_y) * pixel_y
        out[:, :, k, 0] = O.unit_of_radius(np.sqrt(x * x + y * y), unit, dist, wavelength)
        out[:, :, k, 1] = np.arctan2(y, x)
    return out.reshape(h * w, 4, 2)


def _corners_wrong_order(*a, **k):
    # corners visited (0, 0), (1, 1), (1, 0), (0, 1): a self-crossing outline
    c = _orig["pixel_corners"](*a, **k)
    return c[:, [0, 2, 1, 3], :]


def _area_halved(poly):
    return _orig["polygon_area"](poly) / (2 if len(poly) == 4 else 1)


def _bbox_drop_inner(lo, hi, npt, pmin, pmax):
    p, b, c = _orig["bbox_entries"](lo, hi, npt, pmin, pmax)
    keep = np.ones(p.size, dtype=bool)
    order = np.lexsort((b, p))
    ps, bs = p[order], b[order]
    is_first = np.r_[True, ps[1:] != ps[:-1]]
    is_last = np.r_[ps[1:] != ps[:-1], True]
    keep[order] = is_first | is_last
    return p[keep], b[keep], c[keep]


def _bbox_b1_plus_one(lo, hi, npt, pmin, pmax):
    # right edge put one bin too far (where it still fits)
    p, b, c = _orig["bbox_entries"](lo, hi, npt, pmin, pmax)
    order = np.lexsort((b, p))
    ps = p[order]
    is_last = np.r_[ps[1:] != ps[:-1], True]
    shift = np.zeros(p.size, dtype=np.int64)
    shift[order] = is_last.astype(np.int64)
    nb = np.minimum(b + shift, npt - 1)
    return p, nb, c


def _bbox_clipped_width(lo, hi, npt, pmin, pmax):
    # normalises by the clipped width instead of the full box width
    p, b, c = _orig["bbox_entries"](lo, hi, npt, pmin, pmax)
    s = np.zeros(len(lo))
    np.add.at(s, p, c)
    return p, b, c / s[p]


def _bbox_delta_npt_minus_one(lo, hi, npt, pmin, pmax):
    return _orig["bbox_entries"](lo, hi, npt, pmin, pmin + (pmax - pmin) * npt / (npt - 1) if npt > 1 else pmax)


def _extents_corner_min(*a, **k):
    # lo taken as the nearest CORNER instead of the nearest point
    lo, hi, rc = _orig["pixel_extents"](*a, **k)
    args = dict(zip(("h", "w", "pixel_y", "pixel_x", "center_y", "center_x", "dist",
                     "wavelength", "unit"), a))
    args.update(k)
    h, w = args["h"], args["w"]
    i = np.arange(h)[:, None]
    j = np.arange(w)[None, :]
    best = None
    for da in (0, 1):
        for db in (0, 1):
            x = ((j + da) - args["center_x"]) * args["pixel_x"]
            y = ((i + db) - args["center_y"]) * args["pixel_y"]
            d = np.sqrt(x * x + y * y)
            best = d if best is None else np.minimum(best, d)
    lo2 = O.unit_of_radius(np.broadcast_to(best, (h, w)).reshape(-1), args.get("unit", "r_m"),
                           args["dist"], args["wavelength"])
    return np.asarray(lo2, dtype=np.float64), hi, rc


def _extents_swapped(*a, **k):
    lo, hi, rc = _orig["pixel_extents"](*a, **k)
    return hi, lo, rc


def _nosplit_ceil(centre, npt, pmin, pmax):
    p, b, c = _orig["nosplit_entries"](centre, npt, pmin, pmax)
    return p, np.minimum(b + 1, npt - 1), c


def _integrate_transposed(m, x, empty=0.0):
    # x indexed by the bin instead of the pixel
    mm = dict(m)
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    mm["pix"] = np.minimum(m["bins"], x.size - 1)
    I, W, U = _orig["integrate"](mm, x, empty)
    return I, W, U


def _integrate_inverted_ratio(m, x, empty=0.0):
    I, W, U = _orig["integrate"](m, x, empty)
    with np.errstate(divide="ignore", invalid="ignore"):
        I2 = np.where(W != 0, U / np.where(W != 0, W, 1.0), empty)
    return I2, W, U


def _integrate_dropped_u_coef(m, x, empty=0.0):
    # U counts entries instead of summing coefficients
    I, W, U = _orig["integrate"](m, x, empty)
    U2 = np.bincount(m["bins"], minlength=m["npt"]).astype(np.float64)
    I2 = np.where(U2 > 0, W / np.where(U2 > 0, U2, 1.0), empty)
    return I2, W, U2


def _vjp_no_divide(m, U, grad_I=None, grad_W=None, norm=None):
    return _orig["integrate_vjp"](m, np.ones_like(np.asarray(U)), grad_I, grad_W, norm)


def _vjp_wrong_sign_w(m, U, grad_I=None, grad_W=None, norm=None):
    gw = None if grad_W is None else -np.asarray(grad_W)
    return _orig["integrate_vjp"](m, U, grad_I, gw, norm)


def _kahan_no_comp(values):
    s = np.float32(0.0)
    for v in np.asarray(values, dtype=np.float32):
        s = np.float32(s + v)
    return s


def _unit_deg_wrong(r, unit, dist, wavelength):
    v = _orig["unit_of_radius"](r, unit, dist, wavelength)
    if unit == "2th_deg":
        return np.arctan(r / dist) * (math.pi / 180.0)
    if unit == "q_nm":
        return (4.0 * math.pi) * np.sin(np.arctan(r / dist)) / (wavelength * 1e9)
    return v


def _correct_dark_sign(raw, dark=None, flat=None, solid=None, polar=None):
    d = None if dark is None else -np.asarray(dark, dtype=np.float64)
    return _orig["correct"](raw, d, flat, solid, polar)


def _correct_norm_order(raw, dark=None, flat=None, solid=None, polar=None):
    # multiplies by the norm instead of dividing
    x = _orig["correct"](raw, dark)
    for a in (flat, solid, polar):
        if a is not None:
            x = x * np.asarray(a, dtype=np.float64).reshape(-1)
    return x


def _azimuth_mirrored(y, x):
    # atan2 with its arguments in the wrong order's sign: chi -> -chi
    return _orig["corner_azimuth"](-y, x)


def _azimuth_no_wrap(chi_lo, chi_hi, whole, npt_azim):
    # shares falling past -pi or pi are dropped instead of wrapped round
    p, b, c = _orig["azimuth_entries_loop"](chi_lo, chi_hi, whole, npt_azim)
    delta = 2 * math.pi / npt_azim
    keep = np.ones(p.size, dtype=bool)
    for e in range(p.size):
        if whole[p[e]]:
            continue
        gl = (float(chi_lo[p[e]]) + math.pi) / delta
        gh = (float(chi_hi[p[e]]) + math.pi) / delta
        if (gl < 0 and b[e] >= math.floor(gl) % npt_azim) or \
           (gh > npt_azim and b[e] <= (math.ceil(gh) - 1) % npt_azim):
            keep[e] = False
    return p[keep], b[keep], c[keep]


def _bbox2d_rows_transposed(rad, azi, npt_rad):
    # row a * npt_azim + c instead of c * npt_rad + a
    p, rows, c = _orig["bbox2d_entries"](rad, azi, npt_rad)
    npt_azim = int(azi[1].max()) + 1 if azi[1].size else 1
    a, cc = rows % npt_rad, rows // npt_rad
    return p, a * npt_azim + cc, c


def _bbox2d_sum(rad, azi, npt_rad):
    # shares averaged instead of multiplied
    p, rows, c = _orig["bbox2d_entries"](rad, (azi[0], azi[1], np.ones_like(azi[2])), npt_rad)
    p2, rows2, c2 = _orig["bbox2d_entries"]((rad[0], rad[1], np.ones_like(rad[2])), azi, npt_rad)
    return p, rows, 0.5 * (c + c2)


def _full2d_wedge_offset(corners, lo, hi, npt_rad, npt_azim, pmin, pmax):
    # wedges counted from 0 instead of from -pi: every share half a turn off
    p, b, c = _orig["full2d_entries"](corners, lo, hi, npt_rad, npt_azim, pmin, pmax)
    a, k = b % npt_rad, b // npt_rad
    return p, ((k + npt_azim // 2) % npt_azim) * npt_rad + a, c


def _nosplit2d_rows_swapped(h, w, pixel_y, pixel_x, center_y, center_x, centre, npt_rad,
                            npt_azim, pmin, pmax):
    # radial and azimuthal bins swapped in the row number where they fit
    p, rows, c = _orig["nosplit2d_entries"](h, w, pixel_y, pixel_x, center_y, center_x, centre,
                                             npt_rad, npt_azim, pmin, pmax)
    a, k = rows % npt_rad, rows // npt_rad
    ok = (k < npt_rad) & (a < npt_azim)
    return p, np.where(ok, a * npt_rad + k, rows), c


def _extents_never_whole(h, w, pixel_y, pixel_x, center_y, center_x, lo):
    chi_lo, chi_hi, whole = _orig["azimuth_extents"](h, w, pixel_y, pixel_x, center_y,
                                                     center_x, lo)
    return chi_lo, chi_hi, np.zeros_like(whole)



def _range_from_zero(lo, hi, centre, split):
    # the naive loop's [0, max] taken as the default range
    pmin, pmax = _orig["default_range"](lo, hi, centre, split)
    return 0.0, pmax


def _positions_left_edges(npt, pmin, pmax):
    return pmin + np.arange(npt) * ((pmax - pmin) / npt)


def _norm_without_polar(flat=None, solid=None, polar=None):
    return _orig["correction_norm"](flat, solid, None)


def _clip_slab_too_wide(poly, x0, x1):
    # the right edge of the slab put one slab width too far
    return _orig["clip_slab"](poly, x0, x1 + (x1 - x0))


MUTANTS = {
    "bbox_drop_inner": ("bbox_entries", _bbox_drop_inner),
    "bbox_b1_plus_one": ("bbox_entries", _bbox_b1_plus_one),
    "bbox_clipped_width": ("bbox_entries", _bbox_clipped_width),
    "bbox_delta_npt_minus_one": ("bbox_entries", _bbox_delta_npt_minus_one),
    "extents_corner_min": ("pixel_extents", _extents_corner_min),
    "extents_swapped": ("pixel_extents", _extents_swapped),
    "nosplit_ceil": ("nosplit_entries", _nosplit_ceil),
    "integrate_transposed": ("integrate", _integrate_transposed),
    "integrate_inverted_ratio": ("integrate", _integrate_inverted_ratio),
    "integrate_counts_not_coefs": ("integrate", _integrate_dropped_u_coef),
    "vjp_no_divide": ("integrate_vjp", _vjp_no_divide),
    "vjp_wrong_sign_w": ("integrate_vjp", _vjp_wrong_sign_w),
    "kahan_no_compensation": ("kahan_sum_f32", _kahan_no_comp),
    "unit_wrong_conversion": ("unit_of_radius", _unit_deg_wrong),
    "correct_dark_sign": ("correct", _correct_dark_sign),
    "correct_multiplies": ("correct", _correct_norm_order),
    "full_no_unwrap": ("pixel_corners", _corners_no_unwrap),
    "full_corner_order": ("pixel_corners", _corners_wrong_order),
    "full_area_of_pixel_wrong": ("polygon_area", _area_halved),
    "2d_azimuth_mirrored": ("corner_azimuth", _azimuth_mirrored),
    "2d_azimuth_no_wrap": ("azimuth_entries_loop", _azimuth_no_wrap),
    "2d_rows_transposed": ("bbox2d_entries", _bbox2d_rows_transposed),
    "2d_shares_averaged": ("bbox2d_entries", _bbox2d_sum),
    "2d_full_wedge_offset": ("full2d_entries", _full2d_wedge_offset),
    "2d_beam_pixel_not_whole": ("azimuth_extents", _extents_never_whole),
    "2d_nosplit_rows_swapped": ("nosplit2d_entries", _nosplit2d_rows_swapped),
    "range_from_zero": ("default_range", _range_from_zero),
    "positions_left_edges": ("positions", _positions_left_edges),
    "norm_without_polar": ("correction_norm", _norm_without_polar),
    "clip_slab_too_wide": ("clip_slab", _clip_slab_too_wide),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    attr, fn = MUTANTS[name]
    monkeypatch.setattr(O, attr, fn)
    caught = []
    for pin in pins.ALL_PINS:
        try:
            with np.errstate(all="ignore"):
                pin(O)
        except (AssertionError, ValueError, IndexError, ZeroDivisionError):
            caught.append(pin.__name__)
    assert caught, f"no pin noticed the planted mistake {name}"
