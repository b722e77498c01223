"""azint: azimuthal integration on MI355X (gfx950) through a C-ABI HIP library.

Python binding of ``include/azint.h``: argument marshalling only.  Every step
of the per-frame path runs in the library's HIP kernels; PyTorch provides
device memory and streams.  Importing the package does not need a GPU; the
library itself must have been built (``python paper_1412_6367_amd/build.py``),
otherwise the first call raises.

Method: Kieffer & Ashiotis, "PyFAI: a Python library for high performance
azimuthal integration on GPU" (EuroSciPy 2014) -- bounding-box pixel
splitting (Section 4.1) applied as a CSR gather product (Section 5.2).
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np
import torch

__all__ = ["lib", "AzintError", "Plan", "Batch", "Graph", "Integrate1d", "integrate1d", "integrate2d",
           "autotune", "UNITS", "SPLITS"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libazint.so")

UNITS = {"r_m": 0, "r_mm": 1, "2th_rad": 2, "2th_deg": 3, "q_nm": 4}
LAYOUTS = {"pixel": 0, "ring": 1, "tile": 2, "band": 3, "fused": 4, "run": 5}
SPLITS = {"none": 0, "bbox": 1, "full": 2}
_DT = {torch.int16: 0, torch.int32: 2, torch.float32: 4, torch.float64: 5}
for _name, _code in (("uint16", 1), ("uint32", 3)):
    if hasattr(torch, _name):
        _DT[getattr(torch, _name)] = _code
_DT_NP = {np.dtype(np.int16): 0, np.dtype(np.uint16): 1, np.dtype(np.int32): 2,
          np.dtype(np.uint32): 3, np.dtype(np.float32): 4, np.dtype(np.float64): 5}
_STORAGE = {torch.float32: 4, torch.float64: 5}
_ACCUM = {"f64": 0, "kahan32": 1}
NUM_VARIANTS = 7


class AzintError(RuntimeError):
    pass


class Tiling(ctypes.Structure):
    """Launch and tile schedule of the forward kernel (see include/azint.h)."""
    _fields_ = [("tile_nnz", ctypes.c_int32), ("block", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("band", ctypes.c_int32), ("stage", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


STAGES = {"gather": 0, "scatter": 1, "tile": 2, "fuse": 3, "fold": 4, "fold_sum": 5}
DEFAULT_TILING = dict(tile_nnz=0, block=256, variant=5, grid=0, band=16, stage=5)


def _tiling(cur=None, **kw):
    if isinstance(kw.get("stage"), str):
        kw["stage"] = STAGES[kw["stage"]]
    d = dict(DEFAULT_TILING if cur is None else cur)
    d.update({k: v for k, v in kw.items() if v is not None})
    return Tiling(**{k: int(v) for k, v in d.items()})


class _Geom(ctypes.Structure):
    _fields_ = [("h", ctypes.c_int32), ("w", ctypes.c_int32),
                ("pixel_y_m", ctypes.c_double), ("pixel_x_m", ctypes.c_double),
                ("center_y_px", ctypes.c_double), ("center_x_px", ctypes.c_double),
                ("dist_m", ctypes.c_double), ("wavelength_m", ctypes.c_double)]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double
_SIGS = {
    "azi_version": (_I32, []),
    "azi_last_error": (ctypes.c_char_p, []),
    "azi_plan_create": (ctypes.c_int, [ctypes.POINTER(_Geom), _I32, _I32, _I32, _P, _I32, _I32,
                                       ctypes.POINTER(_P)]),
    "azi_plan_create2d": (ctypes.c_int, [ctypes.POINTER(_Geom), _I32, _I32, _I32, _I32, _P, _I32,
                                         _I32, ctypes.POINTER(_P)]),
    "azi_plan_create_device": (ctypes.c_int, [ctypes.POINTER(_Geom), _I32, _I32, _I32, _P, _I32,
                                              _I32, _I32, _P, ctypes.POINTER(_P)]),
    "azi_plan_create2d_device": (ctypes.c_int, [ctypes.POINTER(_Geom), _I32, _I32, _I32, _I32, _P,
                                                _I32, _I32, _I32, _P, ctypes.POINTER(_P)]),
    "azi_plan_shape": (ctypes.c_int, [_P, _P, _P]),
    "azi_plan_azimuths": (ctypes.c_int, [_P, _P]),
    "azi_plan_destroy": (ctypes.c_int, [_P]),
    "azi_plan_info": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "azi_plan_positions": (ctypes.c_int, [_P, _P]),
    "azi_plan_export_csr": (ctypes.c_int, [_P, _P, _P, _P]),
    "azi_plan_export_csc": (ctypes.c_int, [_P, _P, _P, _P]),
    "azi_plan_set_tiling": (ctypes.c_int, [_P, _P]),
    "azi_plan_get_tiling": (ctypes.c_int, [_P, _P, _P]),
    "azi_plan_tile_schedule": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "azi_plan_run_schedule": (ctypes.c_int, [_P, _I32, _P, _P, _P, _P, _P, _P, _P, _P]),
    "azi_plan_autotune": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _I32]),
    "azi_plan_set_layout": (ctypes.c_int, [_P, _I32]),
    "azi_plan_get_layout": (ctypes.c_int, [_P, _P]),
    "azi_plan_upload": (ctypes.c_int, [_P, _I32]),
    "azi_plan_device_bytes": (_I64, [_P]),
    "azi_plan_correction_bytes": (_I32, [_P]),
    "azi_plan_set_corrections": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "azi_correct": (ctypes.c_int, [_P, _P, _I32, _P, _P]),
    "azi_integrate1d": (ctypes.c_int, [_P, _P, _P, _P, _P, _D, _P]),
    "azi_integrate1d_raw": (ctypes.c_int, [_P, _P, _I32, _P, _P, _P, _D, _P]),
    "azi_integrate1d_raw_noalloc": (ctypes.c_int, [_P, _P, _I32, _P, _P, _P, _D, _P]),
    "azi_noalloc_scratch_bytes": (_I64, []),
    "azi_integrate1d_backward": (ctypes.c_int, [_P, _P, _P, _P, _P, _I32, _P]),
    "azi_plan_stage": (ctypes.c_int, [_P, _P, _I32, _P]),
    "azi_integrate1d_staged": (ctypes.c_int, [_P, _P, _P, _P, _D, _P]),
    "azi_batch_create": (ctypes.c_int, [_P, _I32, _I32, ctypes.POINTER(_P)]),
    "azi_batch_destroy": (ctypes.c_int, [_P]),
    "azi_batch_info": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "azi_batch_set_tiling": (ctypes.c_int, [_P, _P]),
    "azi_batch_get_tiling": (ctypes.c_int, [_P, _P, _P]),
    "azi_batch_forward": (ctypes.c_int, [_P, _P, _P, _P, _P, _D, _P]),
    "azi_batch_forward_loop": (ctypes.c_int, [_P, _P, _P, _P, _P, _D, _P]),
    "azi_batch_forward_raw": (ctypes.c_int, [_P, _P, _I32, _P, _P, _P, _D, _P]),
    "azi_batch_backward": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "azi_batch_autotune": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, ctypes.c_char_p, _I32]),
    "azi_graph_create_batch": (ctypes.c_int, [_P, _P, _P, _P, _P, _D, _P, _P, _P, _P,
                                              ctypes.POINTER(_P)]),
    "azi_graph_create_plan": (ctypes.c_int, [_P, _P, _I32, _P, _P, _P, _D, _P,
                                             ctypes.POINTER(_P)]),
    "azi_graph_launch": (ctypes.c_int, [_P, _P]),
    "azi_graph_destroy": (ctypes.c_int, [_P]),
}

_lib = None


def lib():
    """The loaded C-ABI library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise AzintError(f"{LIB_PATH} is missing: build it first "
                             "(python paper_1412_6367_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        msg = lib().azi_last_error().decode(errors="replace")
        raise AzintError(f"azint error {rc}: {msg}")


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _need(t, dtype, n, device, name):
    if t is None:
        return
    if not isinstance(t, torch.Tensor) or t.device != device:
        raise AzintError(f"{name} must be a tensor on {device}")
    if dtype is not None and t.dtype != dtype:
        raise AzintError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous() or t.numel() != n:
        raise AzintError(f"{name} must be contiguous with {n} elements, got {tuple(t.shape)}")


class Plan:
    """Coefficient matrix of one detector geometry (Sections 3, 4, 5.2.1).

    ``pixel`` is a size in metres or a (y, x) pair; ``center`` the beam centre
    (row, column) in pixel units (default: the middle of the detector).
    ``npt`` radial bins; with ``npt_azim`` (>= 2) the plan integrates in two
    dimensions, bins (wedge c, radial bin a) in row c * npt + a, and
    ``self.npt`` counts all of them.
    """

    def __init__(self, h, w, npt, *, npt_azim=None, pixel=1e-4, center=None, dist=0.1,
                 wavelength=1e-10, unit="r_m", split="bbox", range=None, dtype=torch.float64,
                 accum="f64", layout=None, device=None, **tiling):
        py, px = (pixel, pixel) if np.isscalar(pixel) else pixel
        cy, cx = (h / 2.0, w / 2.0) if center is None else center
        self.npt_rad = int(npt)
        self.npt_azim = int(npt_azim) if npt_azim else 0
        self.h, self.w = int(h), int(w)
        self.npt = self.npt_rad * max(self.npt_azim, 1)
        self.dtype = dtype
        self.accum = accum
        self._h = None
        g = _Geom(int(h), int(w), float(py), float(px), float(cy), float(cx), float(dist),
                  float(wavelength))
        rng = None if range is None else (ctypes.c_double * 2)(float(range[0]), float(range[1]))
        out = ctypes.c_void_p()
        rng_p = ctypes.cast(rng, ctypes.c_void_p) if rng else None
        if self.npt_azim:
            _check(lib().azi_plan_create2d(ctypes.byref(g), self.npt_rad, self.npt_azim,
                                           UNITS[unit], SPLITS[split], rng_p, _STORAGE[dtype],
                                           _ACCUM[accum], ctypes.byref(out)))
        else:
            _check(lib().azi_plan_create(ctypes.byref(g), self.npt_rad, UNITS[unit],
                                         SPLITS[split], rng_p, _STORAGE[dtype], _ACCUM[accum],
                                         ctypes.byref(out)))
        self._h = out
        self.device = None
        if layout is not None:
            self.set_layout(layout)
        if tiling:
            self.set_tiling(**tiling)
        if device is not None:
            self.upload(device)

    @classmethod
    def on_device(cls, h, w, npt, *, device, npt_azim=None, pixel=1e-4, center=None, dist=0.1,
                  wavelength=1e-10, unit="r_m", split="bbox", range=None, dtype=torch.float64,
                  accum="f64", stream=None):
        """A plan built by the device plan builder on ``device``: one-
        dimensional (returned uploaded there, band layout; set_layout("run")
        switches to the run encoding, built from the plan's host copy), or
        with ``npt_azim`` two-dimensional (pixel layout)."""
        dev = torch.device(device) if not isinstance(device, torch.device) else device
        idx = dev.index if dev.index is not None else torch.cuda.current_device()
        py, px = (pixel, pixel) if np.isscalar(pixel) else pixel
        cy, cx = (h / 2.0, w / 2.0) if center is None else center
        self = cls.__new__(cls)
        self.npt_rad, self.npt_azim = int(npt), int(npt_azim) if npt_azim else 0
        self.h, self.w = int(h), int(w)
        self.npt = self.npt_rad * max(self.npt_azim, 1)
        self.dtype, self.accum = dtype, accum
        self._h = None
        g = _Geom(int(h), int(w), float(py), float(px), float(cy), float(cx), float(dist),
                  float(wavelength))
        rng = None if range is None else (ctypes.c_double * 2)(float(range[0]), float(range[1]))
        out = ctypes.c_void_p()
        rng_p = ctypes.cast(rng, ctypes.c_void_p) if rng else None
        with torch.cuda.device(idx):
            if self.npt_azim:
                _check(lib().azi_plan_create2d_device(
                    ctypes.byref(g), int(npt), self.npt_azim, UNITS[unit], SPLITS[split], rng_p,
                    _STORAGE[dtype], _ACCUM[accum], idx, _stream(stream), ctypes.byref(out)))
            else:
                _check(lib().azi_plan_create_device(
                    ctypes.byref(g), int(npt), UNITS[unit], SPLITS[split], rng_p,
                    _STORAGE[dtype], _ACCUM[accum], idx, _stream(stream), ctypes.byref(out)))
        self._h = out
        self.device = torch.device("cuda", idx)
        return self

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.azi_plan_destroy(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def info(self):
        npt, npix, nnz = _I32(), _I64(), _I64()
        rng = (ctypes.c_double * 2)()
        _check(lib().azi_plan_info(self._h, ctypes.byref(npt), ctypes.byref(npix),
                                   ctypes.byref(nnz), ctypes.cast(rng, ctypes.c_void_p)))
        return dict(npt=npt.value, npix=npix.value, nnz=nnz.value, range=(rng[0], rng[1]))

    @property
    def npix(self):
        return self.h * self.w

    @property
    def nnz(self):
        return self.info()["nnz"]

    def positions(self):
        """Radial bin centres (npt_rad values)."""
        out = np.empty(self.npt_rad, dtype=np.float64)
        _check(lib().azi_plan_positions(self._h, out.ctypes.data))
        return out

    def azimuths(self):
        """Wedge centres in radians (two-dimensional plans)."""
        out = np.empty(self.npt_azim, dtype=np.float64)
        _check(lib().azi_plan_azimuths(self._h, out.ctypes.data))
        return out

    def shape(self):
        """(npt_rad, npt_azim) as the library reports them (npt_azim 0 in 1-D)."""
        a, b = _I32(), _I32()
        _check(lib().azi_plan_shape(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def _np_dtype(self):
        return np.float64 if self.dtype == torch.float64 else np.float32

    def export_csr(self):
        nnz = self.nnz
        data = np.empty(nnz, dtype=self._np_dtype())
        indices = np.empty(nnz, dtype=np.int32)
        indptr = np.empty(self.npt + 1, dtype=np.int32)
        _check(lib().azi_plan_export_csr(self._h, data.ctypes.data, indices.ctypes.data,
                                         indptr.ctypes.data))
        return data, indices, indptr

    def export_csc(self):
        nnz = self.nnz
        data = np.empty(nnz, dtype=self._np_dtype())
        bins = np.empty(nnz, dtype=np.int32)
        colptr = np.empty(self.npix + 1, dtype=np.int32)
        _check(lib().azi_plan_export_csc(self._h, data.ctypes.data, bins.ctypes.data,
                                         colptr.ctypes.data))
        return data, bins, colptr

    def set_tiling(self, **kw):
        """Change any of tile_nnz, block, variant, grid, band, stage."""
        t = _tiling(self.tiling(), **kw)
        _check(lib().azi_plan_set_tiling(self._h, ctypes.byref(t)))

    def tiling(self):
        t = Tiling()
        _check(lib().azi_plan_get_tiling(self._h, ctypes.byref(t), None))
        return t.as_dict()

    def tile_schedule(self, **tiling):
        t = _tiling(self.tiling(), **tiling)
        nt, ns = _I32(), _I32()
        _check(lib().azi_plan_tile_schedule(self._h, ctypes.byref(t), ctypes.byref(nt), None,
                                            ctypes.byref(ns), None))
        tiles = np.zeros((nt.value, 8), dtype=np.int32)
        splits = np.zeros((ns.value, 4), dtype=np.int32)
        _check(lib().azi_plan_tile_schedule(self._h, ctypes.byref(t), ctypes.byref(nt),
                                            tiles.ctypes.data, ctypes.byref(ns),
                                            splits.ctypes.data))
        return tiles, splits

    def autotune(self, x, *, stream=None):
        """Time candidate layouts and tilings on the corrected image ``x``,
        keep the fastest and return the library's JSON report as a dict
        (layouts change only while the plan has no corrections)."""
        _need(x, self.dtype, self.npix, self.device, "x")
        I, W, U = self._outs(None)
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().azi_plan_autotune(self._h, _ptr(x), _ptr(I), _ptr(W), _ptr(U),
                                       _stream(stream), buf, len(buf)))
        return json.loads(buf.value.decode())

    def run_schedule(self, tile_nnz=None):
        """Host-built run encoding of the matrix (the run layout's arrays:
        runs, gbase, coef, pieces (n, 8), bin_slot, bin_count)."""
        tn = self.tiling()["tile_nnz"] if tile_nnz is None else int(tile_nnz)
        nr, npc = _I64(), _I32()
        _check(lib().azi_plan_run_schedule(self._h, tn, ctypes.byref(nr), None, None, None,
                                           ctypes.byref(npc), None, None, None))
        runs = np.empty(nr.value, dtype=np.int32)
        gbase = np.empty(nr.value // 64, dtype=np.int32)
        coef = np.empty(self.nnz, dtype=np.float64)
        pieces = np.empty((npc.value, 8), dtype=np.int32)
        slot = np.empty(self.npt, dtype=np.int32)
        count = np.empty(self.npt, dtype=np.int32)
        _check(lib().azi_plan_run_schedule(self._h, tn, None, runs.ctypes.data,
                                           gbase.ctypes.data, coef.ctypes.data, None,
                                           pieces.ctypes.data, slot.ctypes.data,
                                           count.ctypes.data))
        return dict(runs=runs, gbase=gbase, coef=coef, pieces=pieces, bin_slot=slot,
                    bin_count=count)

    def set_layout(self, layout):
        """"pixel", "ring", "tile", "band", "fused" or "run" layout of the
        device matrix."""
        _check(lib().azi_plan_set_layout(self._h, LAYOUTS[layout]))

    def layout(self):
        v = _I32()
        _check(lib().azi_plan_get_layout(self._h, ctypes.byref(v)))
        return {c: n for n, c in LAYOUTS.items()}[v.value]

    def upload(self, device=None):
        device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        if device.type != "cuda":
            raise AzintError("plans live on a GPU")
        idx = device.index if device.index is not None else torch.cuda.current_device()
        _check(lib().azi_plan_upload(self._h, idx))
        self.device = torch.device("cuda", idx)
        return self

    def device_bytes(self):
        return int(lib().azi_plan_device_bytes(self._h))

    def correction_bytes(self):
        """Bytes per pixel of the correction the raw-frame band / run gather reads
        (0 when there is none)."""
        return int(lib().azi_plan_correction_bytes(self._h))

    def set_corrections(self, dark=None, flat=None, solid=None, polar=None, stream=None):
        for name, t in (("dark", dark), ("flat", flat), ("solid", solid), ("polar", polar)):
            _need(t, self.dtype, self.npix, self.device, name)
        _check(lib().azi_plan_set_corrections(self._h, _ptr(dark), _ptr(flat), _ptr(solid),
                                              _ptr(polar), _stream(stream)))

    def _raw_code(self, raw):
        code = _DT.get(raw.dtype)
        if code is None:
            raise AzintError(f"unsupported raw dtype {raw.dtype}")
        return code

    def correct(self, raw, out=None, stream=None):
        _need(raw, None, self.npix, self.device, "raw")
        out = torch.empty(self.npix, dtype=self.dtype, device=self.device) if out is None else out
        _need(out, self.dtype, self.npix, self.device, "x")
        _check(lib().azi_correct(self._h, _ptr(raw), self._raw_code(raw), _ptr(out),
                                 _stream(stream)))
        return out

    def _outs(self, out):
        if out is None:
            return tuple(torch.empty(self.npt, dtype=self.dtype, device=self.device)
                         for _ in range(3))
        for t in out:
            _need(t, self.dtype, self.npt, self.device, "output")
        return out

    def integrate(self, x, *, empty=0.0, out=None, stream=None):
        """(I, W, U) of a corrected image x (storage dtype, npix values)."""
        _need(x, self.dtype, self.npix, self.device, "x")
        I, W, U = self._outs(out)
        _check(lib().azi_integrate1d(self._h, _ptr(x), _ptr(I), _ptr(W), _ptr(U),
                                     float(empty), _stream(stream)))
        return I, W, U

    def integrate_raw(self, raw, *, empty=0.0, out=None, stream=None):
        """Cast + correction + integration of a raw image (Section 6.4)."""
        _need(raw, None, self.npix, self.device, "raw")
        I, W, U = self._outs(out)
        _check(lib().azi_integrate1d_raw(self._h, _ptr(raw), self._raw_code(raw), _ptr(I),
                                         _ptr(W), _ptr(U), float(empty), _stream(stream)))
        return I, W, U

    def integrate_raw_noalloc(self, raw, *, empty=0.0, out=None, stream=None):
        """integrate_raw with its partial sums in the library's static device
        array: given `out`, neither this call nor the library allocates."""
        _need(raw, None, self.npix, self.device, "raw")
        I, W, U = self._outs(out)
        _check(lib().azi_integrate1d_raw_noalloc(self._h, _ptr(raw), self._raw_code(raw),
                                                 _ptr(I), _ptr(W), _ptr(U), float(empty),
                                                 _stream(stream)))
        return I, W, U

    def stage(self, raw, *, stream=None):
        """Cast + correction of a raw image into the plan's work image."""
        _need(raw, None, self.npix, self.device, "raw")
        _check(lib().azi_plan_stage(self._h, _ptr(raw), self._raw_code(raw), _stream(stream)))

    def integrate_staged(self, *, empty=0.0, out=None, stream=None):
        """Integration of the work image left by :meth:`stage`."""
        I, W, U = self._outs(out)
        _check(lib().azi_integrate1d_staged(self._h, _ptr(I), _ptr(W), _ptr(U), float(empty),
                                            _stream(stream)))
        return I, W, U

    def backward(self, U, grad_I=None, grad_W=None, *, wrt_raw=False, out=None, stream=None):
        for name, t in (("U", U), ("grad_I", grad_I), ("grad_W", grad_W)):
            _need(t, self.dtype, self.npt, self.device, name)
        gx = torch.empty(self.npix, dtype=self.dtype, device=self.device) if out is None else out
        _need(gx, self.dtype, self.npix, self.device, "grad_x")
        _check(lib().azi_integrate1d_backward(self._h, _ptr(U), _ptr(grad_I), _ptr(grad_W),
                                              _ptr(gx), int(bool(wrt_raw)), _stream(stream)))
        return gx

    def graph(self, raw, I, W=None, U=None, *, empty=0.0, stream=None):
        out = ctypes.c_void_p()
        _check(lib().azi_graph_create_plan(self._h, _ptr(raw), self._raw_code(raw), _ptr(I),
                                           _ptr(W), _ptr(U), float(empty), _stream(stream),
                                           ctypes.byref(out)))
        # the graph holds this plan's matrix and work-buffer addresses: keep
        # the plan alive for as long as the graph
        return Graph(out, keep=(self, raw, I, W, U))


class Integrate1d(torch.autograd.Function):
    """I = W / U of a corrected image, differentiable with respect to it.

    forward(x, plan, empty) -> (I, W); backward uses the library's adjoint
    kernel: gx = A^T (gI / U + gW).
    """

    @staticmethod
    def forward(ctx, x, plan, empty=0.0):
        I, W, U = plan.integrate(x.contiguous(), empty=empty)
        ctx.plan = plan
        ctx.shape = x.shape
        ctx.save_for_backward(U)
        ctx.mark_non_differentiable(U)
        return I, W, U

    @staticmethod
    def backward(ctx, gI, gW, gU):
        (U,) = ctx.saved_tensors
        gI = None if gI is None else gI.contiguous()
        gW = None if gW is None else gW.contiguous()
        gx = ctx.plan.backward(U, gI, gW)
        return gx.view(ctx.shape), None, None


def integrate1d(image, plan, *, empty=0.0):
    """(positions, I) as the paper's ``integrate1d`` returns (Section 3)."""
    x = image.reshape(-1)
    if x.dtype == plan.dtype:
        I, _, _ = plan.integrate(x.contiguous(), empty=empty)
    else:
        I, _, _ = plan.integrate_raw(x.contiguous(), empty=empty)
    return plan.positions(), I


def integrate2d(image, plan, *, empty=0.0):
    """(radial positions, wedge centres, I as an npt_azim x npt_rad map) of
    a two-dimensional plan (Section 4)."""
    if not plan.npt_azim:
        raise ValueError("integrate2d needs a plan made with npt_azim")
    _, I = integrate1d(image, plan, empty=empty)
    return plan.positions(), plan.azimuths(), I.reshape(plan.npt_azim, plan.npt_rad)


class Graph:
    """A captured HIP graph bound to fixed device buffers."""

    def __init__(self, handle, keep=()):
        self._h = handle
        self._keep = keep

    def launch(self, stream=None):
        _check(lib().azi_graph_launch(self._h, _stream(stream)))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.azi_graph_destroy(self._h)
            self._h = None


class Batch:
    """Many plans stacked into one block-diagonal matrix (one launch per pass)."""

    def __init__(self, plans, device=None):
        if not plans:
            raise AzintError("empty batch")
        self.dtype = plans[0].dtype
        device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        idx = device.index if device.index is not None else torch.cuda.current_device()
        arr = (ctypes.c_void_p * len(plans))(*[p.handle for p in plans])
        out = ctypes.c_void_p()
        self._h = None
        _check(lib().azi_batch_create(arr, len(plans), idx, ctypes.byref(out)))
        self._h = out
        self.device = torch.device("cuda", idx)
        n = len(plans)
        self.n = n
        npix, npt, nnz = _I64(), _I64(), _I64()
        self.pix_off = np.zeros(n + 1, dtype=np.int64)
        self.bin_off = np.zeros(n + 1, dtype=np.int64)
        _check(lib().azi_batch_info(self._h, None, ctypes.byref(npix), ctypes.byref(npt),
                                    ctypes.byref(nnz), self.pix_off.ctypes.data,
                                    self.bin_off.ctypes.data))
        self.npix, self.npt, self.nnz = npix.value, npt.value, nnz.value

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.azi_batch_destroy(self._h)
            self._h = None

    def set_tiling(self, **kw):
        """Change any of tile_nnz, block, variant, grid, band, stage."""
        cur = self.tiling()
        cur.pop("ntiles")
        t = _tiling(cur, **kw)
        _check(lib().azi_batch_set_tiling(self._h, ctypes.byref(t)))

    def tiling(self):
        t, n = Tiling(), _I32()
        _check(lib().azi_batch_get_tiling(self._h, ctypes.byref(t), ctypes.byref(n)))
        d = t.as_dict()
        d["ntiles"] = n.value
        return d

    def _outs(self, out):
        if out is None:
            return tuple(torch.empty(self.npt, dtype=self.dtype, device=self.device)
                         for _ in range(3))
        for t in out:
            _need(t, self.dtype, self.npt, self.device, "output")
        return out

    def forward(self, x, *, empty=0.0, out=None, stream=None, loop=False):
        _need(x, self.dtype, self.npix, self.device, "x")
        I, W, U = self._outs(out)
        f = lib().azi_batch_forward_loop if loop else lib().azi_batch_forward
        _check(f(self._h, _ptr(x), _ptr(I), _ptr(W), _ptr(U), float(empty), _stream(stream)))
        return I, W, U

    def forward_raw(self, raw, *, empty=0.0, out=None, stream=None):
        """Cast raw images (any supported dtype, concatenated) and integrate."""
        _need(raw, None, self.npix, self.device, "raw")
        code = _DT.get(raw.dtype)
        if code is None:
            raise AzintError(f"unsupported raw dtype {raw.dtype}")
        I, W, U = self._outs(out)
        _check(lib().azi_batch_forward_raw(self._h, _ptr(raw), code, _ptr(I), _ptr(W), _ptr(U),
                                           float(empty), _stream(stream)))
        return I, W, U

    def backward(self, U, grad_I=None, grad_W=None, *, out=None, stream=None):
        for name, t in (("U", U), ("grad_I", grad_I), ("grad_W", grad_W)):
            _need(t, self.dtype, self.npt, self.device, name)
        gx = torch.empty(self.npix, dtype=self.dtype, device=self.device) if out is None else out
        _need(gx, self.dtype, self.npix, self.device, "grad_x")
        _check(lib().azi_batch_backward(self._h, _ptr(U), _ptr(grad_I), _ptr(grad_W),
                                        _ptr(gx), _stream(stream)))
        return gx

    def graph(self, x, I, W=None, U=None, *, empty=0.0, grad_I=None, grad_W=None,
              grad_x=None, stream=None):
        out = ctypes.c_void_p()
        _check(lib().azi_graph_create_batch(self._h, _ptr(x), _ptr(I), _ptr(W), _ptr(U),
                                            float(empty), _ptr(grad_I), _ptr(grad_W),
                                            _ptr(grad_x), _stream(stream), ctypes.byref(out)))
        # the graph holds this batch's matrices and work buffers: keep the
        # batch alive for as long as the graph
        return Graph(out, keep=(self, x, I, W, U, grad_I, grad_W, grad_x))

    def autotune(self, x, *, stream=None):
        I, W, U = self._outs(None)
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().azi_batch_autotune(self._h, _ptr(x), _ptr(I), _ptr(W), _ptr(U),
                                        _stream(stream), buf, len(buf)))
        return json.loads(buf.value.decode())


def _signature(batch):
    """Cache key of a batch: device, storage type, sizes."""
    name = torch.cuda.get_device_properties(batch.device).gcnArchName \
        if torch.cuda.is_available() else "cpu"
    return f"{name}|{batch.dtype}|n={batch.n}|npix={batch.npix}|nnz={batch.nnz}"


def autotune(batch, x, cache_path=None):
    """Choose the batch's tiling: reuse a cached choice for the same signature,
    else sweep on the batch's own data and record the result in the cache."""
    key = _signature(batch)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if key in cache:
        best = cache[key]["best"]
        batch.set_tiling(**{k: best[k] for k in ("tile_nnz", "block", "variant", "grid",
                                                  "band", "stage") if k in best})
        return cache[key]
    report = batch.autotune(x)
    if cache_path:
        cache[key] = report
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return report
