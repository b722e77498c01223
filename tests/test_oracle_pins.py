"""The oracle against facts the paper and mathematics fix (CPU only)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import azint_oracle as O
from tests import pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin(O)


@pytest.mark.parametrize("case", pins.TINY_CASES + [(17, 23, 8.5, 11.5, 29, 1e-4, 1e-4),
                                                    (12, 9, 30.0, -4.0, 11, 1e-4, 1e-4)])
@pytest.mark.parametrize("unit", oracle.UNITS)
def test_loop_equals_vectorised(case, unit):
    """The pure-Python and numpy forms perform the same IEEE operations, so
    extents and coefficients agree bit for bit, results to rounding."""
    h, w, cy, cx, npt, py, px = case
    args = dict(h=h, w=w, pixel_y=py, pixel_x=px, center_y=cy, center_x=cx,
                dist=0.1, wavelength=1e-10, npt=npt, unit=unit)
    for split in ("bbox", "none"):
        a = O.build_matrix(split=split, **args)
        b = O.build_matrix(split=split, loop=True, **args)
        for k in ("lo", "hi", "centre", "indptr", "indices", "data"):
            assert np.array_equal(a[k], b[k]), (k, split)
        x = np.random.default_rng(1).uniform(0, 5, size=h * w)
        Ia, Wa, Ua = O.integrate(a, x)
        Ib, Wb, Ub = O.integrate_loop(b, x)
        assert np.allclose(Ia, Ib, rtol=1e-15, atol=0)
        assert np.allclose(Wa, Wb, rtol=1e-15, atol=0)
        assert np.allclose(Ua, Ub, rtol=1e-15, atol=0)


def test_paper_test_case_geometry():
    """The generator uses the paper's test-case geometry, and on it the
    outermost pixel corner sits at sqrt(2) * 1024 pixels, i.e.
    2theta = atan(0.1448.../0.1)."""
    import synth
    g = json.load(open(os.path.join(GOLDEN, "paper_test_case.json")))
    assert synth.PIXEL_M == g["pixel_m"] and synth.DIST_M == g["dist_m"]
    assert synth.WAVELENGTH_M == g["wavelength_m"]
    assert (1 << synth.RAW_BITS) == 2 ** g["raw_bits_max"]
    n = g["shape"][0]
    lo, hi, rc = O.pixel_extents(n, n, g["pixel_m"], g["pixel_m"], n / 2, n / 2,
                                 g["dist_m"], g["wavelength_m"], "2th_deg")
    rmax = math.sqrt(2.0) * (n / 2) * g["pixel_m"]
    assert abs(hi.max() - math.degrees(math.atan(rmax / g["dist_m"]))) < 1e-12
    assert lo.min() == 0.0 and np.count_nonzero(lo == 0.0) == 4


@pytest.mark.slow
def test_paper_test_case_conservation():
    """Pixel and signal conservation (Section 4) on the full 2048x2048 test
    geometry with 1000 bins."""
    g = json.load(open(os.path.join(GOLDEN, "paper_test_case.json")))
    n = g["shape"][0]
    m = O.build_matrix(h=n, w=n, pixel_y=g["pixel_m"], pixel_x=g["pixel_m"],
                       center_y=n / 2, center_x=n / 2, dist=g["dist_m"],
                       wavelength=g["wavelength_m"], npt=1000, unit="2th_deg")
    x = np.random.default_rng(0).integers(0, 1 << 20, size=n * n).astype(np.float64)
    I, W, U = O.integrate(m, x)
    assert abs(U.sum() - n * n) <= 1e-12 * n * n
    assert abs(W.sum() - x.sum()) <= 1e-12 * x.sum()
    per_pixel = np.bincount(m["pix"], minlength=n * n)
    delta = (m["pmax"] - m["pmin"]) / 1000
    bound = np.ceil((m["hi"] - m["lo"]) / delta) + 1
    assert per_pixel.min() >= 1 and np.all(per_pixel <= bound)
