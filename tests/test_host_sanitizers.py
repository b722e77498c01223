"""The host plan builder under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): plan_builder.cpp and a host-only driver (tests/sanitize/) are
compiled with g++ -fsanitize=address,undefined and run over geometries that
reach the builder's edge cases -- a one-pixel and a one-row detector, a beam
off the detector, a clipped range, bins finer than pixels, full splitting,
two-dimensional plans -- and every host-side layout is built from each
matrix.  Any sanitizer report fails the run; the matrix sizes must equal the
oracle's."""
import os
import shutil
import subprocess

import pytest

import oracle
from tests.helpers import ROOT

CSRC = os.path.join(ROOT, "paper_1412_6367_amd", "csrc")
HARNESS = os.path.join(ROOT, "tests", "sanitize", "host_harness.cpp")

UNITS = {"r_m": 0, "r_mm": 1, "2th_rad": 2, "2th_deg": 3, "q_nm": 4}
SPLITS = {"none": 0, "bbox": 1, "full": 2}

CASES = [
    # h, w, center_y, center_x, npt, npt_azim, unit, split, range
    (1, 1, 0.5, 0.5, 4, 0, "r_m", "bbox", None),
    (1, 17, 0.5, 8.5, 5, 0, "r_m", "bbox", None),
    (37, 53, 10.25, 40.5, 61, 0, "r_m", "bbox", None),
    (64, 48, -5.0, 70.0, 40, 0, "r_m", "bbox", None),
    (31, 29, 15.5, 14.5, 300, 0, "r_m", "bbox", None),
    (50, 60, 25.0, 30.0, 37, 0, "r_m", "bbox", (5e-4, 2.5e-3)),
    (50, 60, 25.3, 30.7, 37, 0, "r_m", "none", None),
    (40, 33, 20.1, 16.7, 45, 0, "q_nm", "bbox", None),
    (41, 38, 20.6, 18.2, 50, 0, "r_m", "full", None),
    (30, 30, -7.0, 40.0, 25, 0, "2th_deg", "full", None),
    (24, 20, 12.0, 10.0, 15, 12, "r_m", "bbox", None),
    (18, 22, 9.3, 30.0, 10, 36, "r_m", "full", None),
    (20, 20, 10.5, 9.5, 12, 8, "r_m", "none", None),
    (300, 280, 150.2, 139.7, 250, 0, "r_m", "bbox", None),
]


def _oracle_nnz(c):
    h, w, cy, cx, npt, na, unit, split, rng = c
    args = dict(h=h, w=w, pixel_y=1e-4, pixel_x=1e-4, center_y=cy, center_x=cx, dist=0.1,
                wavelength=1e-10, unit=unit, split=split, range_=rng)
    if na:
        return len(oracle.build_matrix2d(npt_rad=npt, npt_azim=na, **args)["coef"])
    return len(oracle.build_matrix(npt=npt, **args)["coef"])


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("san") / "host_harness")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(CSRC, "plan_builder.cpp"), HARNESS, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


def test_host_builder_clean_under_sanitizers(harness):
    lines = []
    for c in CASES:
        h, w, cy, cx, npt, na, unit, split, rng = c
        lo, hi = rng if rng else (1.0, 0.0)
        lines.append(f"{h} {w} {cy!r} {cx!r} {npt} {na} {UNITS[unit]} {SPLITS[split]} "
                     f"{lo!r} {hi!r}")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([harness], input="\n".join(lines) + "\n", capture_output=True,
                       text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    out = r.stdout.split("\n")
    for c, row in zip(CASES, out):
        kind, nnz, runs = row.split()
        assert kind == "ok", (c, row)
        assert int(nnz) == _oracle_nnz(c), (c, row)
        assert int(runs) > 0
