"""The allocation-free raw-frame entry point (azi_integrate1d_raw_noalloc)
against azi_integrate1d_raw, through the C ABI.

Both run the same kernels in the same order, so the outputs must agree bit
for bit; the second call of each pair is on a smaller image, after a larger
one has left its partial sums in the shared static array.  A small case is
also checked against the FP64 oracle.
"""
import ctypes
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.helpers import azint, norm_err, oracle_matrix

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _nan_outs(plan, dev):
    return tuple(torch.full((plan.npt,), float("nan"), dtype=plan.dtype, device=dev)
                 for _ in range(3))


def _call_raw(az, plan, raw, outs, fn):
    I, W, U = outs
    rc = getattr(az.lib(), fn)(plan.handle, raw.data_ptr(), plan._raw_code(raw), I.data_ptr(),
                               W.data_ptr(), U.data_ptr(), ctypes.c_double(-2.5), None)
    return rc


def _plan_and_frame(az, dev, h, w, npt, seed, dtype=torch.float64, accum="f64", layout=None,
                    **tiling):
    inst = synth.instance_hw(h, w, seed, npt=npt, corrections=True)
    g = inst.geom
    kw = dict(center=(g.center_y, g.center_x), dtype=dtype, accum=accum, device=dev)
    if layout:
        kw["layout"] = layout
    plan = az.Plan(g.h, g.w, npt, **kw, **tiling)
    npd = np.float64 if dtype == torch.float64 else np.float32
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=npd).reshape(-1)).to(dev)
    plan.set_corrections(t(inst.dark), t(inst.flat), t(inst.solid), t(inst.polar))
    raw = torch.from_numpy(inst.raw.reshape(-1)).to(dev)
    return plan, raw, inst


def _same_as_raw(az, plan, raw, dev, what):
    ref = _nan_outs(plan, dev)
    got = _nan_outs(plan, dev)
    assert _call_raw(az, plan, raw, ref, "azi_integrate1d_raw") == 0, what
    rc = _call_raw(az, plan, raw, got, "azi_integrate1d_raw_noalloc")
    assert rc == 0, (what, az.lib().azi_last_error())
    torch.cuda.synchronize()
    for a, b, name in zip(got, ref, "IWU"):
        assert torch.equal(a, b), (what, name)
    return got


def test_scratch_size():
    az = azint()
    assert az.lib().azi_noalloc_scratch_bytes() == 8 << 20


@pytest.mark.parametrize("layout,dtype,accum", [
    ("run", torch.float64, "f64"), ("run", torch.float32, "f64"),
    ("run", torch.float32, "kahan32"), ("band", torch.float64, "f64"),
    ("tile", torch.float64, "f64"), ("fused", torch.float64, "f64"),
    ("fused", torch.float32, "f64")])
def test_two_calls_second_smaller(layout, dtype, accum, dev):
    """A large frame then a smaller one, each equal to azi_integrate1d_raw."""
    az = azint()
    say("no-alloc", layout, dtype, accum)
    big, raw_big, _ = _plan_and_frame(az, dev, 1000, 1000, 1000, 11, dtype, accum, layout)
    small, raw_small, inst = _plan_and_frame(az, dev, 131, 97, 70, 12, dtype, accum, layout)
    _same_as_raw(az, big, raw_big, dev, f"{layout} 1000x1000")
    got = _same_as_raw(az, small, raw_small, dev, f"{layout} 131x97")
    if dtype == torch.float64:
        g = inst.geom
        m = oracle_matrix(g.h, g.w, g.center_y, g.center_x, inst.npt)
        x = oracle.correct(inst.raw, inst.dark, inst.flat, inst.solid, inst.polar)
        Io, Wo, Uo = oracle.integrate(m, x, empty=-2.5)
        _, Wa, _ = oracle.integrate(m, np.abs(x))
        I, W, U = (t.cpu().numpy() for t in got)
        assert norm_err(W, Wo, Wa) <= 1e-12
        assert norm_err(U, Uo, Uo) <= 1e-12
        assert norm_err(I, Io, np.where(Uo > 0, Wa / np.where(Uo > 0, Uo, 1), 0)) <= 1e-12
        assert np.all(I[Uo == 0] == -2.5)


def test_repeat_after_other_plan_keeps_bits(dev):
    """The shared array keeps the last call's contents; a call overwrites all
    it reads, so alternating plans gives the same bits every time."""
    az = azint()
    a, raw_a, _ = _plan_and_frame(az, dev, 400, 300, 350, 21)
    b, raw_b, _ = _plan_and_frame(az, dev, 90, 120, 64, 22)
    first = [o.clone() for o in _same_as_raw(az, a, raw_a, dev, "a")]
    _same_as_raw(az, b, raw_b, dev, "b")
    again = _same_as_raw(az, a, raw_a, dev, "a again")
    for x, y in zip(first, again):
        assert torch.equal(x, y)


def test_rejects_other_layouts(dev):
    az = azint()
    plan, raw, _ = _plan_and_frame(az, dev, 64, 64, 40, 31, layout="pixel")
    outs = _nan_outs(plan, dev)
    rc = _call_raw(az, plan, raw, outs, "azi_integrate1d_raw_noalloc")
    assert rc == -1
    assert b"layout" in az.lib().azi_last_error()


def test_rejects_plan_beyond_scratch(dev):
    """Pieces of 64 runs on a 3000x3000 frame need ~13 MB of partial sums:
    refused with a message, outputs untouched."""
    az = azint()
    plan, raw, _ = _plan_and_frame(az, dev, 3000, 3000, 3000, 41, tile_nnz=128)
    need = 16 * 4 * plan.run_schedule(128)["pieces"].shape[0]
    assert need > az.lib().azi_noalloc_scratch_bytes()
    outs = _nan_outs(plan, dev)
    rc = _call_raw(az, plan, raw, outs, "azi_integrate1d_raw_noalloc")
    torch.cuda.synchronize()
    assert rc == -1
    assert b"static scratch" in az.lib().azi_last_error()
    assert all(torch.isnan(o).all() for o in outs)
    # the plan's own entry point still works on it
    _call_raw(az, plan, raw, outs, "azi_integrate1d_raw")
    torch.cuda.synchronize()
    assert not torch.isnan(outs[2]).any()
