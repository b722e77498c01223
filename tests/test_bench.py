"""Host logic of bench.py (no GPU): the one-GPU guard, the algorithmic byte
counts, the run encoding's own byte count and the measured-traffic record."""
import json
import os
import subprocess
import sys

import numpy as np

from tests.helpers import azint

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_byte_counts_of_the_c2_frame():
    """The step, integration and adjoint byte counts at the ~1e7-pixel frame
    (nnz 28 323 554, 3162 bins) in float64."""
    nnz, npix, npt = 28323554, 10001406, 3162
    # CSR yardstick of the integration of a corrected image
    assert bench.spmv_bytes(nnz, npix, npt, 8) == nnz * 12 + npix * 8 + (npt + 1) * 4 + 3 * npt * 8
    assert abs(bench.spmv_bytes(nnz, npix, npt, 8) / 1e6 - 420.0) < 0.1
    # the raw-frame step: 12-byte correction records, or (dark, 1/norm) pairs
    assert abs(bench.raw_bytes(nnz, npix, npt, 8, 12) / 1e6 - 500.0) < 0.1
    assert abs(bench.raw_bytes(nnz, npix, npt, 8, 16) / 1e6 - 540.0) < 0.1
    assert bench.raw_bytes(nnz, npix, npt, 8, 16) - bench.raw_bytes(nnz, npix, npt, 8, 12) \
        == 4 * npix
    # folded: a float dark per pixel (420 MB); integer dark counts kept in 2
    # bytes do not shrink the yardstick
    assert abs(bench.raw_bytes(nnz, npix, npt, 8, 4) / 1e6 - 420.0) < 0.1
    assert bench.raw_bytes(nnz, npix, npt, 8, 2) == bench.raw_bytes(nnz, npix, npt, 8, 4)
    assert bench.raw_bytes(nnz, npix, npt, 8, 0) == bench.raw_bytes(nnz, npix, npt, 8, 4)
    # adjoint of a 1-D plan: coefficients, column pointers and one first-bin
    # word per pixel instead of per-entry bin ids
    assert bench.bwd_bytes(nnz, npix, npt, 8) == nnz * 8 + (npix + 1) * 4 + npix * 4 + \
        npix * 8 + 2 * npt * 8


def test_encoding_bytes_count_the_runs():
    """The run encoding's bytes use one word per pixel run within a band of
    4 bins: the count from the CSC equals the runs of the exported schedule."""
    az = azint()
    plan = az.Plan(150, 140, 90, center=(70.3, 75.8), stage="fuse")
    s = plan.run_schedule()
    runs = int((s["runs"] >= 0).sum())
    got = bench.encoding_bytes(plan, np, plan.npix, plan.npt, 8, 12)
    assert got == runs * 4 + plan.nnz * 8 + plan.npix * (4 + 12) + 3 * plan.npt * 8
    # folded normalisation: the dark value (4 bytes) is stored per run
    plan.set_tiling(stage="fold")
    got = bench.encoding_bytes(plan, np, plan.npix, plan.npt, 8, 4)
    assert got == runs * (4 + 4) + plan.nnz * 8 + plan.npix * 4 + 3 * plan.npt * 8
    # the dark term summed once per correction set: nothing stored per run
    plan.set_tiling(stage="fold_sum")
    got = bench.encoding_bytes(plan, np, plan.npix, plan.npt, 8, 0)
    assert got == runs * 4 + plan.nnz * 8 + plan.npix * 4 + 3 * plan.npt * 8
    plan.set_layout("band")
    assert bench.encoding_bytes(plan, np, plan.npix, plan.npt, 8, 12) == \
        bench.raw_bytes(plan.nnz, plan.npix, plan.npt, 8, 12)


def test_measured_traffic_follows_the_kernel_sources(tmp_path, monkeypatch):
    """The committed counter record is used only for the kernel sources it
    was taken on."""
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["c2_f64"]
    assert rec["sources"] == list(bench.TRAFFIC_SOURCES)
    if rec["kernels_sha256"] == bench.kernel_source_hash():
        assert bench.measured_traffic("c2_f64") == rec["fetch_bytes"] + rec["write_bytes"]
    fake = tmp_path / "profiles"
    fake.mkdir()
    (fake / "traffic.json").write_text(json.dumps({"c2_f64": dict(rec, kernels_sha256="0" * 64)}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "1" * 64)
    assert bench.measured_traffic("c2_f64") is None
    assert bench.measured_traffic("no_such_workload") is None
