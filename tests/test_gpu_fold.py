"""The raw-frame path with 1/norm folded into the coefficients
(AZI_STAGE_FOLD, run layout; AZI_STAGE_FOLD_SUM also sums the dark term
once) against the FP64 oracle, and against the unfolded path
(AZI_STAGE_FUSE) on the same plan: W and I within the stated tolerance, U
bit for bit (it is summed once from the unfolded coefficients in the
per-frame order)."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.helpers import azint, oracle_matrix
from tests.test_gpu_forward import TOL32_F64, TOL64, check

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


RAW_TYPES = [np.int32, np.uint16, np.float32, np.float64]
COMBOS = [(1, 1, 1, 1), (1, 0, 0, 0), (0, 1, 1, 0), (0, 0, 0, 1), (0, 0, 0, 0)]


def _setup(az, dev, inst, dtype, accum, stage, **kw):
    g = inst.geom
    return az.Plan(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), dtype=dtype,
                   accum=accum, layout="run", stage=stage, device=dev, **kw)


def _tensor(a, dev, npd=None):
    a = np.ascontiguousarray(a).reshape(-1)
    return torch.from_numpy(a if npd is None else a.astype(npd)).to(dev)


@pytest.mark.parametrize("band", [4, 16])
@pytest.mark.parametrize("raw_dtype", RAW_TYPES, ids=lambda t: np.dtype(t).name)
@pytest.mark.parametrize("combo", COMBOS, ids=lambda c: "".join(map(str, c)))
@pytest.mark.parametrize("dtype,accum", [(torch.float64, "f64"), (torch.float32, "f64"),
                                         (torch.float32, "kahan32")],
                         ids=["f64", "f32", "k32"])
def test_fold_matches_oracle(dtype, accum, combo, raw_dtype, band, dev):
    say("fold", dtype, accum, combo, raw_dtype)
    az = azint()
    inst = synth.instance_hw(173, 181, 9, npt=150, corrections=True)
    g = inst.geom
    npd = np.float64 if dtype == torch.float64 else np.float32
    arrs = [a if on else None for a, on in zip((inst.dark, inst.flat, inst.solid, inst.polar),
                                               combo)]
    raw_np = inst.raw.reshape(-1).astype(raw_dtype)
    raw = _tensor(raw_np, dev)
    outs = {}
    for stage in ("fold_sum", "fold", "fuse"):
        plan = _setup(az, dev, inst, dtype, accum, stage, band=band)
        plan.set_corrections(*(None if a is None else _tensor(a, dev, npd) for a in arrs))
        outs[stage] = plan.integrate_raw(raw, empty=-3.0)
        torch.cuda.synchronize()
    # U does not depend on the image: the folded path's U is the unfolded one's
    assert torch.equal(outs["fold"][2], outs["fuse"][2])
    assert torch.equal(outs["fold_sum"][2], outs["fuse"][2])
    m = oracle_matrix(g.h, g.w, g.center_y, g.center_x, inst.npt)
    # the oracle corrects the same storage-type corrections as the plan holds
    x = oracle.correct(raw_np, *(None if a is None else a.astype(npd).astype(np.float64)
                                 for a in arrs))
    tol = TOL64 if dtype == torch.float64 else TOL32_F64
    check(outs["fold"], m, x, tol, empty=-3.0, what=f"fold {combo}")
    check(outs["fold_sum"], m, x, tol, empty=-3.0, what=f"fold_sum {combo}")


@pytest.mark.parametrize("band", [4, 16, 32])
def test_fold_follows_tiling_changes(band, dev):
    """Pieces, workgroup size and persistent grids change the order of the
    sums: U is summed again, and the results stay within tolerance."""
    say("fold retile")
    az = azint()
    inst = synth.instance_hw(260, 240, 10, npt=200, corrections=True)
    g = inst.geom
    t = lambda a: _tensor(a, dev)
    m = oracle_matrix(g.h, g.w, g.center_y, g.center_x, inst.npt)
    x = oracle.correct(inst.raw, inst.dark, inst.flat, inst.solid, inst.polar)
    fold = _setup(az, dev, inst, torch.float64, "f64", "fold", band=band)
    fsum = _setup(az, dev, inst, torch.float64, "f64", "fold_sum", band=band)
    fuse = _setup(az, dev, inst, torch.float64, "f64", "fuse", band=band)
    for p in (fold, fsum, fuse):
        p.set_corrections(t(inst.dark), t(inst.flat), t(inst.solid), t(inst.polar))
    for kw in (dict(tile_nnz=1024), dict(block=128), dict(grid=64), dict(tile_nnz=8192, grid=0),
               dict(block=256, tile_nnz=4096), dict(tile_nnz=0)):
        for p in (fold, fsum, fuse):
            p.set_tiling(**kw)
        a = fold.integrate_raw(t(inst.raw))
        c = fsum.integrate_raw(t(inst.raw))
        b = fuse.integrate_raw(t(inst.raw))
        torch.cuda.synchronize()
        assert torch.equal(a[2], b[2]) and torch.equal(c[2], b[2]), kw
        check(a, m, x, TOL64, what=str(kw))
        check(c, m, x, TOL64, what=f"fold_sum {kw}")


def test_fold_stage_switch_and_recorrect(dev):
    """Switching the stage of a corrected plan, and setting new corrections
    on a folded plan, keep the results right."""
    say("fold switch")
    az = azint()
    inst = synth.instance_hw(150, 170, 11, npt=120, corrections=True)
    g = inst.geom
    t = lambda a: _tensor(a, dev)
    m = oracle_matrix(g.h, g.w, g.center_y, g.center_x, inst.npt)
    plan = _setup(az, dev, inst, torch.float64, "f64", "fuse")
    plan.set_corrections(t(inst.dark), t(inst.flat), t(inst.solid), t(inst.polar))
    x = oracle.correct(inst.raw, inst.dark, inst.flat, inst.solid, inst.polar)
    for stage in ("fold", "fold_sum", "fuse", "fold_sum", "fold"):
        plan.set_tiling(stage=stage)
        check(plan.integrate_raw(t(inst.raw)), m, x, TOL64, what=stage)
    assert plan.correction_bytes() == 2         # integer dark counts: 16 bits per run
    plan.set_tiling(stage="fold_sum")
    assert plan.correction_bytes() == 0         # the dark term summed once: nothing per run
    plan.set_tiling(stage="fold")
    flat2 = inst.flat[::-1].copy()
    plan.set_corrections(None, t(flat2), None, t(inst.polar))
    x2 = oracle.correct(inst.raw, None, flat2, None, inst.polar)
    check(plan.integrate_raw(t(inst.raw)), m, x2, TOL64, what="new corrections")
    # a float64 dark that is not a float keeps its double form; fractional
    # floats and integers beyond 16 bits take a float per run
    for add, nbytes in ((0.1, 8), (0.25, 4), (70000.0, 4), (0.0, 2)):
        dark = inst.dark.reshape(-1).astype(np.float64) + add
        plan.set_corrections(t(dark), t(inst.flat), t(inst.solid), t(inst.polar))
        assert plan.correction_bytes() == nbytes, add
        x3 = oracle.correct(inst.raw, dark, inst.flat, inst.solid, inst.polar)
        check(plan.integrate_raw(t(inst.raw)), m, x3, TOL64, what=f"dark + {add}")
    # new corrections on a plan in the fold-sum stage: its dark term is
    # summed again from the new dark map (and dropped with it)
    plan.set_tiling(stage="fold_sum")
    for dark in (inst.dark * 3.0 + 7.0, None):
        plan.set_corrections(None if dark is None else t(dark), t(inst.flat), None,
                             t(inst.polar))
        assert plan.correction_bytes() == 0
        x4 = oracle.correct(inst.raw, dark, inst.flat, None, inst.polar)
        check(plan.integrate_raw(t(inst.raw)), m, x4, TOL64, what=f"fold_sum, dark {dark is None}")


@pytest.mark.parametrize("stage", ["fold", "fold_sum"])
def test_fold_graph_and_noalloc(stage, dev):
    """The folded step captured in a graph and through the allocation-free
    entry point gives the eager call's bits, replay after replay."""
    say("fold graph", stage)
    az = azint()
    inst = synth.instance_hw(300, 280, 12, npt=250, corrections=True)
    g = inst.geom
    t = lambda a: _tensor(a, dev)
    plan = _setup(az, dev, inst, torch.float64, "f64", stage)
    plan.set_corrections(t(inst.dark), t(inst.flat), t(inst.solid), t(inst.polar))
    raw = t(inst.raw)
    ref = [o.clone() for o in plan.integrate_raw(raw)]
    outs = tuple(torch.full((plan.npt,), float("nan"), dtype=torch.float64, device=dev)
                 for _ in range(3))
    gr = plan.graph(raw, *outs)
    for _ in range(3):
        for o in outs:
            o.fill_(float("nan"))
        gr.launch()
        torch.cuda.synchronize()
        for a, b in zip(outs, ref):
            assert torch.equal(a, b)
        plan.integrate_raw(raw)  # eager work between replays
    na = plan.integrate_raw_noalloc(raw)
    torch.cuda.synchronize()
    for a, b in zip(na, ref):
        assert torch.equal(a, b)


def test_fold_band_layout_is_fuse(dev):
    """The band layout takes AZI_STAGE_FOLD and _FOLD_SUM as AZI_STAGE_FUSE."""
    az = azint()
    inst = synth.instance_hw(120, 110, 13, npt=90, corrections=True)
    g = inst.geom
    t = lambda a: _tensor(a, dev)
    res = []
    for stage in ("fold", "fold_sum", "fuse"):
        p = az.Plan(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), layout="band",
                    stage=stage, device=dev)
        p.set_corrections(t(inst.dark), t(inst.flat), t(inst.solid), t(inst.polar))
        res.append(p.integrate_raw(t(inst.raw)))
        torch.cuda.synchronize()
    for r in res[:2]:
        for a, b in zip(r, res[2]):
            assert torch.equal(a, b)


@pytest.mark.parametrize("dark_lo", [4000, 40000], ids=["dark100x", "dark1000x"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_fold_sum_on_a_dark_dominated_frame(dtype, dark_lo, dev):
    """Summing the dark term once subtracts two large sums when the dark
    current outweighs the signal: frames whose dark counts are on average
    ~100 and ~1000 times their signal (signal uniform in [0, 100)) stay
    within the float64 tolerance of the oracle
    (normalised, as everywhere, by sum_p A_bp |x_p| of the corrected image),
    and the dark-per-run form on the same plan agrees with it."""
    say("fold_sum dark-dominated", dtype, dark_lo)
    az = azint()
    inst = synth.instance_hw(260, 250, 15, npt=180, corrections=True)
    g = inst.geom
    rng = np.random.default_rng(15)
    dark = rng.integers(dark_lo, dark_lo * 3 // 2, size=(g.h, g.w)).astype(np.float64)
    raw = (dark + rng.integers(0, 100, size=(g.h, g.w))).astype(np.int32)
    npd = np.float64 if dtype == torch.float64 else np.float32
    t = lambda a: _tensor(a, dev, npd)
    m = oracle_matrix(g.h, g.w, g.center_y, g.center_x, inst.npt)
    plan = _setup(az, dev, inst, dtype, "f64", "fold_sum")
    plan.set_corrections(t(dark), t(inst.flat), t(inst.solid), t(inst.polar))
    assert plan.correction_bytes() == 0
    rawt = _tensor(raw, dev)
    a = [o.clone() for o in plan.integrate_raw(rawt)]
    plan.set_tiling(stage="fold")
    b = plan.integrate_raw(rawt)
    torch.cuda.synchronize()
    x = oracle.correct(raw, *(v.astype(npd).astype(np.float64)
                              for v in (dark, inst.flat, inst.solid, inst.polar)))
    tol = TOL64 if dtype == torch.float64 else TOL32_F64
    e = check(a, m, x, tol, what=f"fold_sum, dark from {dark_lo}")
    say("normalised errors", dark_lo, e)
    check(b, m, x, tol, what=f"fold, dark from {dark_lo}")
    assert torch.equal(a[2], b[2])


def test_fold_sum_with_kahan_sums_keeps_dark_per_run(dev):
    """Plans with Kahan float sums take AZI_STAGE_FOLD_SUM as AZI_STAGE_FOLD:
    the same bits, the dark value stored per run."""
    az = azint()
    inst = synth.instance_hw(140, 150, 16, npt=100, corrections=True)
    t = lambda a: _tensor(a, dev, np.float32)
    res = []
    for stage in ("fold_sum", "fold"):
        p = _setup(az, dev, inst, torch.float32, "kahan32", stage)
        p.set_corrections(t(inst.dark), t(inst.flat), t(inst.solid), t(inst.polar))
        assert p.correction_bytes() == 2
        res.append(p.integrate_raw(_tensor(inst.raw, dev)))
        torch.cuda.synchronize()
    for a, b in zip(*res):
        assert torch.equal(a, b)


@pytest.mark.parametrize("band", [16, 32])
def test_balanced_schedule_fills_one_round_on_the_device(band, dev):
    """tile_nnz 0 on an uploaded plan: the run schedule takes at most as many
    workgroups as the device keeps resident (CUs x 8 of four wavefronts,
    x 4 of eight), the bound on a band's groups of 64 runs per stretch is the
    smallest that fits (one group less overflows the round: recounted with
    the greedy cut written for the CPU test), and the folded step on it
    matches the oracle."""
    from tests.test_abi import _greedy_stretches
    say("balanced on device", band)
    az = azint()
    h, w, cy, cx, npt = 1400, 1300, 650.3, 720.7, 1200
    waves = band // 4
    plan = az.Plan(h, w, npt, center=(cy, cx), tile_nnz=0, band=band, device=dev)
    ncu = torch.cuda.get_device_properties(dev).multi_processor_count
    target = ncu * 32 // waves
    s = plan.run_schedule(tile_nnz=0)
    runs, pieces = s["runs"], s["pieces"]
    nt = len(pieces) // waves
    assert nt <= target
    lens = (pieces[:, 1] - pieces[:, 0]).astype(np.int64)
    bound = int(lens.max()) // 64
    mask = (1 << 27) - 1
    nbands = (npt + 3) // 4
    firsts = {}
    for t in range(nt):
        for e in pieces[t * waves:(t + 1) * waves]:
            if e[4] >= 0:
                b = int(e[2]) // 4
                for z in range(int(e[0]), int(e[1]), 64):
                    firsts.setdefault(b, []).append(int(runs[z]) & mask)
    groups = range((nbands + waves - 1) // waves)
    per = [[firsts.get(b, []) for b in range(gi * waves, min(nbands, (gi + 1) * waves))]
           for gi in groups]
    assert sum(_greedy_stretches(p, bound) for p in per) == nt
    if bound > 1:
        assert sum(_greedy_stretches(p, bound - 1) for p in per) > target
    # and the step on it
    inst = synth.instance_hw(h, w, 14, npt=npt, corrections=True)
    t = lambda a: _tensor(a, dev)
    plan.set_corrections(t(inst.dark), t(inst.flat), t(inst.solid), t(inst.polar))
    m = oracle_matrix(h, w, cy, cx, npt)
    x = oracle.correct(inst.raw, inst.dark, inst.flat, inst.solid, inst.polar)
    check(plan.integrate_raw(t(inst.raw)), m, x, TOL64, what=f"balanced band {band}")
