"""Shared test helpers: locating (or building) the library, oracle shortcuts."""
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_built = False


def azint():
    """The binding package; builds the library first if it is missing."""
    global _built
    import paper_1412_6367_amd as az
    if not os.path.exists(az.LIB_PATH) and not _built:
        from paper_1412_6367_amd import build
        build.build()
        _built = True
    return az


def oracle_matrix(h, w, cy, cx, npt, py=1e-4, px=1e-4, unit="r_m", split="bbox", rng=None,
                  dist=0.1, wavelength=1e-10):
    import oracle
    return oracle.build_matrix(h=h, w=w, pixel_y=py, pixel_x=px, center_y=cy, center_x=cx,
                               dist=dist, wavelength=wavelength, npt=npt, unit=unit,
                               split=split, range_=rng)


def norm_err(got, ref, scale):
    """max |got - ref| / scale over entries with scale > 0 (0 elsewhere must match)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.asarray(scale, dtype=np.float64)
    nz = scale > 0
    e = np.zeros_like(ref)
    e[nz] = np.abs(got[nz] - ref[nz]) / scale[nz]
    bad_zero = (~nz) & (got != ref)
    if bad_zero.any():
        return float("inf")
    return float(e.max()) if e.size else 0.0
