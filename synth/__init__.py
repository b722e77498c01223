"""Seeded synthetic workloads for azimuthal integration.

This module only draws random numbers and fixes sizes and detector geometry.
It holds none of the integration arithmetic, so that both the CPU oracle and
the GPU path can consume the same inputs without sharing any of the method.

Geometry follows the paper's test case (Section 3.1, "Test case"): pixels of
1e-4 m, a planar detector 0.1 m from the sample and orthogonal to the beam,
wavelength 1e-10 m, beam centre at the middle of the detector.  Raw pixel
values are integers drawn uniformly in [0, 2**20): the paper states that
detectors deliver 12 to 20 bits per pixel (Section 5.2.2, "About numerical
precision"), and such integers are exact in both float32 and float64.

Workload recipes (the five standard cases):

* ``c1``: one 100x100 image, float64, seed 0, npt 100.
* ``c2``: one 3162x3163 image (~1e7 pixels), seed 1, npt 3162, float64 and
  float32 copies of the same draw.
* ``c3``: 4096 images whose pixel counts are log-uniform in [1e2, 1e5],
  float64, seed 2.
* ``c4``: one 1000x1000 image, float64, seed 3, raw scaled by 2**-20 (exact)
  and an upstream gradient drawn N(0, 1) per bin; 64 random pixels for
  finite differences.
* ``c5``: 1024 images whose pixel counts are log-uniform in [1e3, 1e6],
  float32 storage, seed 4, with an upstream gradient per bin.

Every image of side lengths ``h = round(sqrt(N))``, ``w = round(N / h)`` uses
``npt = round(sqrt(h * w))`` bins.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PIXEL_M = 1e-4       # Section 3.1: pixel size
DIST_M = 0.1         # Section 3.1: sample-detector distance
WAVELENGTH_M = 1e-10 # Section 3.1: X-ray wavelength
RAW_BITS = 20        # Section 5.2.2: detectors give 12..20 bits per pixel


@dataclass
class Geometry:
    """Planar detector orthogonal to the beam (Section 3).

    Pixel (i, j) covers [j, j+1] x [i, i+1] in pixel coordinates; the beam
    centre is given in the same pixel coordinates (column ``center_x``, row
    ``center_y``).
    """
    h: int
    w: int
    pixel_y: float = PIXEL_M
    pixel_x: float = PIXEL_M
    center_y: float = 0.0
    center_x: float = 0.0
    dist: float = DIST_M
    wavelength: float = WAVELENGTH_M

    @property
    def npix(self) -> int:
        return self.h * self.w


def centred_geometry(h: int, w: int) -> Geometry:
    """Beam at the middle of the detector: centre (w/2, h/2) in pixels."""
    return Geometry(h=h, w=w, center_y=h / 2.0, center_x=w / 2.0)


def shape_for(n_target: int) -> tuple[int, int]:
    """Image shape with about ``n_target`` pixels: h = round(sqrt N), w = round(N/h)."""
    h = max(1, int(round(math.sqrt(n_target))))
    w = max(1, int(round(n_target / h)))
    return h, w


def npt_for(h: int, w: int) -> int:
    return max(1, int(round(math.sqrt(h * w))))


@dataclass
class Instance:
    geom: Geometry
    npt: int
    raw: np.ndarray                      # (h, w) int32 detector counts
    dark: np.ndarray | None = None       # (h, w) float64
    flat: np.ndarray | None = None
    solid: np.ndarray | None = None
    polar: np.ndarray | None = None
    grad: np.ndarray | None = None       # (npt,) float64 upstream gradient
    extra: dict = field(default_factory=dict)


def _draw(rng: np.random.Generator, h: int, w: int, npt: int, corrections: bool,
          grad: bool) -> Instance:
    geom = centred_geometry(h, w)
    raw = rng.integers(0, 1 << RAW_BITS, size=(h, w), dtype=np.int32)
    inst = Instance(geom=geom, npt=npt, raw=raw)
    if corrections:
        # Opaque per-pixel correction arrays, drawn in plausible ranges.
        inst.dark = rng.integers(0, 64, size=(h, w)).astype(np.float64)
        inst.flat = rng.uniform(0.95, 1.05, size=(h, w))
        inst.solid = rng.uniform(0.90, 1.00, size=(h, w))
        inst.polar = rng.uniform(0.95, 1.00, size=(h, w))
    if grad:
        inst.grad = rng.standard_normal(npt)
    return inst


def instance(n_target: int, seed, *, npt: int | None = None,
             corrections: bool = False, grad: bool = False) -> Instance:
    """One seeded image of about ``n_target`` pixels."""
    h, w = shape_for(n_target)
    rng = np.random.default_rng(seed)
    return _draw(rng, h, w, npt if npt is not None else npt_for(h, w),
                 corrections, grad)


def instance_hw(h: int, w: int, seed, *, npt: int, corrections: bool = False,
                grad: bool = False) -> Instance:
    rng = np.random.default_rng(seed)
    return _draw(rng, h, w, npt, corrections, grad)


def batch_sizes(n: int, lo: float, hi: float, seed: int) -> list[int]:
    """Pixel counts log-uniform in [lo, hi]: N_k = round(exp(U(ln lo, ln hi)))."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    u = rng.uniform(math.log(lo), math.log(hi), size=n)
    return [int(round(math.exp(v))) for v in u]


def batch(n: int, lo: float, hi: float, seed: int, *, grad: bool = False,
          corrections: bool = False) -> list[Instance]:
    """``n`` uneven instances; instance k draws from SeedSequence(seed).spawn(n)[k]."""
    sizes = batch_sizes(n, lo, hi, seed)
    children = np.random.SeedSequence(seed).spawn(n)
    out = []
    for k, nk in enumerate(sizes):
        h, w = shape_for(nk)
        rng = np.random.default_rng(children[k])
        out.append(_draw(rng, h, w, npt_for(h, w), corrections, grad))
    return out


def fd_coords(npix: int, count: int, seed: int) -> np.ndarray:
    """Distinct random pixel indices for finite-difference checks."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(2)[1])
    return np.sort(rng.choice(npix, size=min(count, npix), replace=False))


# Named workloads.
C1 = dict(name="c1", n=10_000, seed=0, dtype="f64")
C2 = dict(name="c2", n=10_000_000, seed=1, dtype=("f64", "f32"))
C3 = dict(name="c3", count=4096, lo=1e2, hi=1e5, seed=2, dtype="f64")
C4 = dict(name="c4", n=1_000_000, seed=3, dtype="f64", fd_coords=64, fd_h=1e-6)
C5 = dict(name="c5", count=1024, lo=1e3, hi=1e6, seed=4, dtype="f32")


def c4_instance() -> Instance:
    """The adjoint workload: raw scaled by 2**-20 (exact) into [0, 1)."""
    inst = instance(C4["n"], C4["seed"], grad=True)
    inst.extra["x"] = inst.raw.reshape(-1).astype(np.float64) * (2.0 ** -RAW_BITS)
    inst.extra["fd_coords"] = fd_coords(inst.geom.npix, C4["fd_coords"], C4["seed"])
    return inst
