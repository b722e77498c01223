#!/usr/bin/env python3
"""Benchmark of the azimuthal-integration hot path on one MI355X.

Step = one frame through the per-frame pipeline of Section 6.4 (cast +
dark/flat/solid-angle/polarisation correction + the sparse gather
integration that yields I, W, U; the output memset of the paper is not
needed), on the ~1e7-pixel workload (3162 x 3163 int32 frame, bounding-box
splitting, 3162 bins, float64), the correction applied to each pixel the
integration kernel gathers.  Frames rotate over 4 distinct synthetic
images already resident in HBM.  Prints ONE JSON line on stdout; progress
goes to stderr.

Extra lines in the same JSON object (``lines``): the float32-storage copy,
a cold-cache timing of the integration kernel, the 4096-instance batch (one
persistent graph launch vs a per-instance loop), the 1e6-pixel adjoint, the
1024-instance float32 forward+adjoint batch with autotuned tiles, the
matrix-free (fused) kernel on the same frame, two-dimensional integration of
the frame (1000 x 360 bins), host- vs device-built plans, full pixel
splitting of the frame, and a plain 1 GiB device copy (the measured
streaming ceiling).
"""
import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E


KERNEL_OF_LAYOUT = {
    "band": "k_band (+k_band_reduce): band-ordered gather integration",
    "run": "k_band_runs (+k_band_reduce): band-ordered gather integration, one word and one "
           "gather per pixel run",
    "pixel": "k_spmv (+k_fixup): CSR gather integration",
    "ring": "k_spmv (+k_fixup): CSR gather integration, ring-ordered image",
    "tile": "k_block (+k_block_reduce): image-tile blocked integration",
}


def kernel_of(line):
    """The step's dominant kernel, from the plan's layout and tiling."""
    t = line["tiling"]
    if line["layout"] == "run" and t["band"] in (16, 32):
        k = (f"k_runs_grouped (+k_band_reduce): run-encoded gather integration, "
             f"{t['band'] // 4} neighbouring bands of 4 bins per workgroup")
    else:
        k = KERNEL_OF_LAYOUT[line["layout"]]
    if t["stage"] == 5 and line.get("accum") == "f64":
        return k + ", 1/norm folded into the coefficients and the dark term summed once per " \
                   "correction set: the raw count is the only gathered value, no dark value " \
                   "is read per frame"
    if t["stage"] in (4, 5):
        return k + ", 1/norm folded into the coefficients and dark stored per run: the raw " \
                   "count is the only gathered value"
    return k + ", reading the raw frame and correcting in the gather"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# the integration kernels and the schedule builder (the pieces a launch
# walks decide which lines are fetched twice)
TRAFFIC_SOURCES = ("kernels.hip", "accum.h", "plan_builder.cpp")


def kernel_source_hash():
    """sha256 over the sources of the integration kernels and of the
    schedule builder."""
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1412_6367_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per launch of the integration kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE record (scaled by a plain copy's
    reading), or None when the record is missing or was taken on other
    kernel source than the one built now."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[workload]
        if kernel_source_hash() != rec["kernels_sha256"]:
            return None
        return rec["fetch_bytes"] + rec["write_bytes"]
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--main-only", action="store_true", help="skip the extra lines")
    ap.add_argument("--only", default="", help="comma list of extra lines to run")
    return ap.parse_args()


def mean_event_ms(pairs):
    return sum(a.elapsed_time(b) for a, b in pairs) / len(pairs)


def spmv_bytes(nnz, npix, npt, es):
    """Algorithmic bytes of one integration: CSR coefficients and pixel ids,
    the image, row pointers, three outputs."""
    return nnz * (es + 4) + npix * es + (npt + 1) * 4 + 3 * npt * es


def bwd_bytes(nnz, npix, npt, es):
    """Adjoint of a one-dimensional plan: CSC coefficients, column pointers
    and one first-bin word per pixel (a pixel's bins are consecutive, so no
    per-entry bin ids are needed), the gradient written, U and the upstream
    gradient read."""
    return nnz * es + (npix + 1) * 4 + npix * 4 + npix * es + 2 * npt * es


def build_plans(insts, dtype, az, threads=16):
    def mk(inst):
        g = inst.geom
        return az.Plan(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), dtype=dtype)
    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(mk, insts))


def raw_bytes(nnz, npix, npt, es, cb):
    """Algorithmic bytes of one raw-frame integration with the correction
    in the gather: the matrix, the raw int32 frame, dark and 1/norm (cb
    bytes per pixel: a pair of the storage type, or 12 for float64 with
    dark values that are floats; at least 4, a float dark map, when the
    plan stores its integer dark counts in 2 bytes or sums the dark term
    once per correction set and reads none per frame: the yardstick does
    not shrink with the encoding), row pointers, three outputs."""
    return nnz * (es + 4) + npix * (4 + max(cb, 4)) + (npt + 1) * 4 + 3 * npt * es


def encoding_bytes(plan, np, npix, npt, es, cb):
    """Bytes the run encoding itself streams per raw-frame step (a word per
    pixel run within a band of 4 bins instead of an index per entry; the
    step's roofline keeps the CSR figure of raw_bytes as its yardstick).
    With 1/norm folded into the coefficients the dark value (cb bytes) is
    stored per run beside the run word instead of gathered per pixel (cb 0
    when the dark term is summed once per correction set)."""
    if plan.layout() != "run":
        return raw_bytes(plan.nnz, npix, npt, es, cb)
    _, bins, colptr = plan.export_csc()
    full = np.diff(colptr) > 0
    first = bins[colptr[:-1][full]] // 4
    last = bins[colptr[1:][full] - 1] // 4
    runs = int((last - first + 1).sum())
    if plan.tiling()["stage"] in (4, 5):
        return runs * (4 + cb) + plan.nnz * es + npix * 4 + 3 * npt * es
    return runs * 4 + plan.nnz * es + npix * (4 + cb) + 3 * npt * es


def pipeline_line(az, torch, np, synth, dev, dtype, steps, warmup, frames_n=4, accum="f64",
                  stage=None):
    """Step = one raw int32 frame -> I, W, U with the plan's corrections
    (azi_integrate1d_raw).  With the default layout and tiling the run
    kernel casts and corrects each pixel it gathers, so the step is that
    kernel plus the per-bin reduction.  The two-pass form (correction
    kernel, then the run kernel on the corrected image) and the step
    replayed from HIP graphs are timed beside it."""
    c = synth.C2
    inst = synth.instance(c["n"], c["seed"], corrections=True)
    g = inst.geom
    tdt = torch.float64 if dtype == "f64" else torch.float32
    npd = np.float64 if dtype == "f64" else np.float32
    t0 = time.perf_counter()
    plan = az.Plan(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), dtype=tdt, accum=accum,
                   device=dev, **({"stage": stage} if stage else {}))
    log(f"[{dtype}/{accum}] plan {g.h}x{g.w} npt={inst.npt} nnz={plan.nnz} built+uploaded in "
        f"{time.perf_counter() - t0:.1f}s")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a).reshape(-1).astype(npd)).to(dev)
    plan.set_corrections(t(inst.dark), t(inst.flat), t(inst.solid), t(inst.polar))
    frames = [torch.from_numpy(inst.raw.reshape(-1)).to(dev)]
    rng = np.random.default_rng(c["seed"] + 1000)
    for _ in range(frames_n - 1):
        frames.append(torch.from_numpy(
            rng.integers(0, 1 << synth.RAW_BITS, size=g.npix, dtype=np.int32)).to(dev))
    outs = tuple(torch.empty(inst.npt, dtype=tdt, device=dev) for _ in range(3))
    for k in range(warmup):
        plan.integrate_raw(frames[k % frames_n], out=outs)
    ev = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(2)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        e = ev[k]
        e[0].record()
        plan.integrate_raw(frames[k % frames_n], out=outs)
        e[1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / steps
    step_ms = mean_event_ms(ev)
    es = 8 if dtype == "f64" else 4
    nnz = plan.nnz
    cb = plan.correction_bytes()
    rb = raw_bytes(nnz, g.npix, inst.npt, es, cb)
    enc = encoding_bytes(plan, np, g.npix, inst.npt, es, cb)
    # two-pass breakdown: correction kernel, then integration of the image
    # (its kernels' first launches untimed)
    plan.stage(frames[0])
    plan.integrate_staged(out=outs)
    pairs = []
    for k in range(max(steps // 4, 10)):
        e = tuple(torch.cuda.Event(enable_timing=True) for _ in range(3))
        e[0].record()
        plan.stage(frames[k % frames_n])
        e[1].record()
        plan.integrate_staged(out=outs)
        e[2].record()
        pairs.append(e)
    torch.cuda.synchronize()
    corr_ms = mean_event_ms([(e[0], e[1]) for e in pairs])
    spmv_ms = mean_event_ms([(e[1], e[2]) for e in pairs])
    # the same step replayed from HIP graphs (one per rotating frame buffer)
    graphs = [plan.graph(f, *outs) for f in frames]
    for k in range(warmup):
        graphs[k % frames_n].launch()
    gev = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(2)) for _ in range(steps)]
    torch.cuda.synchronize()
    for k in range(steps):
        gev[k][0].record()
        graphs[k % frames_n].launch()
        gev[k][1].record()
    torch.cuda.synchronize()
    graph_ms = mean_event_ms(gev)
    del graphs
    b = spmv_bytes(nnz, g.npix, inst.npt, es)
    # raw + dark + norm read, corrected image written
    corr_b = g.npix * (4 + 3 * es)
    line = dict(npix=g.npix, npt=inst.npt, nnz=nnz, layout=plan.layout(), accum=accum,
                tiling=plan.tiling(), ms_per_step=ms_step,
                elements_per_s=g.npix / (ms_step * 1e-3),
                correction_bytes_per_pixel=cb,
                step_ms=step_ms, step_bytes=rb, step_gbs=rb / (step_ms * 1e6),
                step_encoding_bytes=enc, step_encoding_gbs=enc / (step_ms * 1e6),
                step_frac=rb / (step_ms * 1e6) / HBM_PEAK_GBS,
                graph_step_ms=graph_ms, graph_elements_per_s=g.npix / (graph_ms * 1e-3),
                two_pass_correct_ms=corr_ms, two_pass_correct_gbs=corr_b / (corr_ms * 1e6),
                integrate_ms=spmv_ms, integrate_bytes=b,
                integrate_gbs=b / (spmv_ms * 1e6),
                integrate_frac=b / (spmv_ms * 1e6) / HBM_PEAK_GBS)
    return line, plan, outs, frames[0]


class Flush:
    """Reads 1 GiB (a sum into one scalar) to push the step's data out of the
    L2 caches and the 256 MB MALL.  Reading leaves no dirty lines behind, so
    the timed launch after it writes nothing back on the flush's account."""

    def __init__(self, torch, dev):
        self.torch = torch
        self.buf = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        self.out = torch.empty((), dtype=torch.float64, device=dev)

    def __call__(self):
        self.torch.sum(self.buf, dim=0, out=self.out)


def flushed_ms(torch, fn, flush, sets=3, reps=10):
    """The timing protocol of the paper's benchmarks (Section 6: best of 3
    sets of 10), each launch preceded by a cache flush: the median of each
    set, the best of the sets.  Returns (best, the three medians)."""
    fn()
    meds = []
    for _ in range(sets):
        pairs = []
        for _ in range(reps):
            flush()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            pairs.append((a, b))
        torch.cuda.synchronize()
        ts = sorted(a.elapsed_time(b) for a, b in pairs)
        meds.append(0.5 * (ts[(reps - 1) // 2] + ts[reps // 2]))
    return min(meds), meds


def cold_line(torch, plan, outs, frame, npix, npt, nnz, es, flush):
    """The step (raw frame, corrections in the gather) with the caches
    flushed before every launch."""
    ms, meds = flushed_ms(torch, lambda: plan.integrate_raw(frame, out=outs), flush)
    by = raw_bytes(nnz, npix, npt, es, plan.correction_bytes())
    return dict(step_ms=ms, set_medians_ms=meds, step_bytes=by, step_gbs=by / (ms * 1e6),
                step_frac=by / (ms * 1e6) / HBM_PEAK_GBS,
                protocol="1 GiB read before each launch; median of 10, best of 3 sets")


def batch_line(az, torch, np, synth, dev, cfg, dtype, with_bwd, tune, reps=20):
    tdt = torch.float64 if dtype == "f64" else torch.float32
    npd = np.float64 if dtype == "f64" else np.float32
    t0 = time.perf_counter()
    insts = synth.batch(cfg["count"], cfg["lo"], cfg["hi"], cfg["seed"], grad=with_bwd)
    plans = build_plans(insts, tdt, az)
    batch = az.Batch(plans, device=dev)
    del plans
    log(f"[{cfg['name']}] {batch.n} instances, npix={batch.npix} npt={batch.npt} "
        f"nnz={batch.nnz}, built in {time.perf_counter() - t0:.1f}s")
    x = torch.from_numpy(np.concatenate([i.raw.reshape(-1) for i in insts]).astype(npd)).to(dev)
    gI = None
    if with_bwd:
        gI = torch.from_numpy(np.concatenate([i.grad for i in insts]).astype(npd)).to(dev)
    del insts
    report = None
    if tune:
        report = az.autotune(batch, x)
        log(f"[{cfg['name']}] autotuned: {report['best']}")
    tiling = batch.tiling()
    I, W, U = (torch.empty(batch.npt, dtype=tdt, device=dev) for _ in range(3))
    gx = torch.empty(batch.npix, dtype=tdt, device=dev) if with_bwd else None
    es = 8 if dtype == "f64" else 4

    def timed(fn):
        fn()
        pairs = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            pairs.append((a, b))
        torch.cuda.synchronize()
        return mean_event_ms(pairs)

    fwd_ms = timed(lambda: batch.forward(x, out=(I, W, U)))
    loop_ms = timed(lambda: batch.forward(x, out=(I, W, U), loop=True))
    graph = batch.graph(x, I, W, U, grad_I=gI, grad_x=gx)
    graph_ms = timed(graph.launch)
    persistent = None
    if report:
        # the fastest persistent grid of the sweep (a fixed number of
        # workgroups walking the static piece schedule), timed beside the
        # chosen tiling, eagerly and captured in a graph
        pc = [c for c in report["candidates"] if c["grid"] > 0]
        if pc:
            bp = min(pc, key=lambda c: c["ms"])
            batch.set_tiling(tile_nnz=bp["tile_nnz"], block=bp["block"], grid=bp["grid"])
            p_fwd = timed(lambda: batch.forward(x, out=(I, W, U)))
            pgraph = batch.graph(x, I, W, U)
            p_graph = timed(pgraph.launch)
            del pgraph
            fb0 = spmv_bytes(batch.nnz, batch.npix, batch.npt, es)
            persistent = dict(tiling=batch.tiling(), forward_ms=p_fwd,
                              forward_frac=fb0 / (p_fwd * 1e6) / HBM_PEAK_GBS,
                              graph_forward_ms=p_graph,
                              graph_forward_frac=fb0 / (p_graph * 1e6) / HBM_PEAK_GBS)
            batch.set_tiling(**{k: tiling[k] for k in ("tile_nnz", "block", "variant", "grid",
                                                       "band", "stage")})
    fb = spmv_bytes(batch.nnz, batch.npix, batch.npt, es)
    line = dict(instances=batch.n, npix=batch.npix, npt=batch.npt, nnz=batch.nnz,
                tiling=tiling, forward_ms=fwd_ms, forward_gbs=fb / (fwd_ms * 1e6),
                forward_frac=fb / (fwd_ms * 1e6) / HBM_PEAK_GBS,
                loop_forward_ms=loop_ms, loop_elements_per_s=batch.npix / (loop_ms * 1e-3),
                batched_vs_loop=loop_ms / fwd_ms)
    if with_bwd:
        _, _, _ = batch.forward(x, out=(I, W, U))
        bwd_ms = timed(lambda: batch.backward(U, gI, out=gx))
        bb = bwd_bytes(batch.nnz, batch.npix, batch.npt, es)
        line.update(backward_ms=bwd_ms, backward_gbs=bb / (bwd_ms * 1e6),
                    backward_frac=bb / (bwd_ms * 1e6) / HBM_PEAK_GBS,
                    graph_fwd_bwd_ms=graph_ms,
                    graph_elements_per_s=batch.npix / (graph_ms * 1e-3),
                    graph_fwd_bwd_frac=(fb + bb) / (graph_ms * 1e6) / HBM_PEAK_GBS)
    else:
        line.update(graph_forward_ms=graph_ms,
                    graph_elements_per_s=batch.npix / (graph_ms * 1e-3),
                    graph_frac=fb / (graph_ms * 1e6) / HBM_PEAK_GBS)
    if report:
        line["autotune_candidates"] = len(report["candidates"])
    if persistent:
        line["persistent"] = persistent
    del graph, batch
    torch.cuda.empty_cache()
    return line


def adjoint_line(az, torch, np, synth, dev, reps=50):
    inst = synth.c4_instance()
    g = inst.geom
    plan = az.Plan(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), device=dev)
    x = torch.from_numpy(inst.extra["x"]).to(dev)
    gI = torch.from_numpy(inst.grad).to(dev)
    I, W, U = plan.integrate(x)
    gx = torch.empty_like(x)
    fw, bw = [], []
    for _ in range(reps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        plan.integrate(x, out=(I, W, U))
        ev[1].record()
        plan.backward(U, gI, out=gx)
        ev[2].record()
        fw.append((ev[0], ev[1]))
        bw.append((ev[1], ev[2]))
    torch.cuda.synchronize()
    f, b = mean_event_ms(fw), mean_event_ms(bw)
    nnz = plan.nnz
    return dict(npix=g.npix, npt=inst.npt, nnz=nnz, forward_ms=f, backward_ms=b,
                forward_gbs=spmv_bytes(nnz, g.npix, inst.npt, 8) / (f * 1e6),
                backward_gbs=bwd_bytes(nnz, g.npix, inst.npt, 8) / (b * 1e6))


def _timed(torch, fn, reps=20):
    fn()
    pairs = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        pairs.append((a, b))
    torch.cuda.synchronize()
    return mean_event_ms(pairs)


def fused_line(az, torch, np, synth, dev, reps=50):
    """Matrix-free integration of the c2 frame (float64): the bounding-box
    coefficients recomputed from the geometry per frame.  Times the kernel on
    a corrected image (warm and after a 1 GiB flush) and the whole raw-frame
    pipeline (cast + correction + integration) in its one kernel.  Bytes per
    launch: the image read and the three outputs written (the per-(tile, bin)
    partial sums are the kernel's own traffic, not counted)."""
    c = synth.C2
    inst = synth.instance(c["n"], c["seed"], corrections=True)
    g = inst.geom
    plan = az.Plan(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), layout="fused",
                   device=dev)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a).reshape(-1).astype(np.float64)).to(dev)
    x = t(inst.raw)
    outs = tuple(torch.empty(inst.npt, dtype=torch.float64, device=dev) for _ in range(3))
    flush = Flush(torch, dev)
    warm = _timed(torch, lambda: plan.integrate(x, out=outs), reps)
    cold, _ = flushed_ms(torch, lambda: plan.integrate(x, out=outs), flush)
    del flush
    plan.set_corrections(t(inst.dark), t(inst.flat), t(inst.solid), t(inst.polar))
    raw = torch.from_numpy(inst.raw.reshape(-1)).to(dev)
    pipe = _timed(torch, lambda: plan.integrate_raw(raw, out=outs), reps)
    by = g.npix * 8 + 3 * inst.npt * 8
    raw_by = g.npix * (4 + 8 + 8) + 3 * inst.npt * 8
    line = dict(npix=g.npix, npt=inst.npt, integrate_ms=warm, integrate_cold_ms=cold,
                integrate_bytes=by, integrate_gbs=by / (warm * 1e6),
                integrate_frac=by / (warm * 1e6) / HBM_PEAK_GBS,
                integrate_elements_per_s=g.npix / (warm * 1e-3),
                pipeline_ms=pipe, pipeline_elements_per_s=g.npix / (pipe * 1e-3),
                pipeline_bytes=raw_by, pipeline_gbs=raw_by / (pipe * 1e6),
                plan_device_bytes=plan.device_bytes())
    del plan
    torch.cuda.empty_cache()
    return line


def fuse_stage_line(az, torch, np, synth, dev, reps=40):
    """The corrected c2 pipeline as one call (integrate_raw), two passes
    (correction kernel, then the band kernel on the corrected image) against
    the band kernel that casts and corrects what it gathers (stage fuse)."""
    c = synth.C2
    inst = synth.instance(c["n"], c["seed"], corrections=True)
    g = inst.geom
    raw = torch.from_numpy(inst.raw.reshape(-1)).to(dev)
    line = {}
    for dt in ("f64", "f32"):
        tdt = torch.float64 if dt == "f64" else torch.float32
        npd = np.float64 if dt == "f64" else np.float32
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a).reshape(-1).astype(npd)).to(dev)
        for stage in ("gather", "fuse"):
            plan = az.Plan(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), dtype=tdt,
                           device=dev, stage=stage)
            plan.set_corrections(t(inst.dark), t(inst.flat), t(inst.solid), t(inst.polar))
            outs = tuple(torch.empty(inst.npt, dtype=tdt, device=dev) for _ in range(3))
            ms = _timed(torch, lambda: plan.integrate_raw(raw, out=outs), reps)
            name = f"{dt}_{'two_pass' if stage == 'gather' else 'fused_correction'}"
            line[name + "_ms"] = ms
            line[name + "_elements_per_s"] = g.npix / (ms * 1e-3)
            del plan
    torch.cuda.empty_cache()
    return line


def two_d_line(az, torch, np, synth, dev, nr=1000, na=360, reps=30):
    """Two-dimensional integration of the c2 frame (float64): 1000 radial
    bins x 360 azimuthal wedges, bounding-box split, default layout."""
    c = synth.C2
    inst = synth.instance(c["n"], c["seed"])
    g = inst.geom
    t0 = time.perf_counter()
    plan = az.Plan(g.h, g.w, nr, npt_azim=na, center=(g.center_y, g.center_x), device=dev)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    # the same plan from the device builder (its first call untimed)
    az.Plan.on_device(g.h, g.w, nr, npt_azim=na, center=(g.center_y, g.center_x), device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dplan = az.Plan.on_device(g.h, g.w, nr, npt_azim=na, center=(g.center_y, g.center_x),
                              device=dev)
    torch.cuda.synchronize()
    device_build_s = time.perf_counter() - t0
    del dplan
    torch.cuda.empty_cache()
    x = torch.from_numpy(inst.raw.reshape(-1).astype(np.float64)).to(dev)
    outs = tuple(torch.empty(plan.npt, dtype=torch.float64, device=dev) for _ in range(3))
    flush = Flush(torch, dev)
    warm = _timed(torch, lambda: plan.integrate(x, out=outs), reps)
    cold, _ = flushed_ms(torch, lambda: plan.integrate(x, out=outs), flush)
    del flush
    nnz = plan.nnz
    by = spmv_bytes(nnz, g.npix, plan.npt, 8)
    line = dict(npix=g.npix, npt_rad=nr, npt_azim=na, nnz=nnz, layout=plan.layout(),
                build_s=build_s, device_build_s=device_build_s,
                integrate_ms=warm, integrate_cold_ms=cold,
                integrate_bytes=by, integrate_gbs=by / (warm * 1e6),
                integrate_frac=by / (warm * 1e6) / HBM_PEAK_GBS,
                integrate_cold_frac=by / (cold * 1e6) / HBM_PEAK_GBS,
                elements_per_s=g.npix / (warm * 1e-3))
    del plan
    torch.cuda.empty_cache()
    return line


def plan_build_line(az, torch, np, synth, dev):
    """Building the c2 plan (matrix + default device layout) with the host
    builder and with the device builder."""
    c = synth.C2
    inst = synth.instance(c["n"], c["seed"])
    g = inst.geom
    t0 = time.perf_counter()
    hp = az.Plan(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), device=dev)
    torch.cuda.synchronize()
    host_s = time.perf_counter() - t0
    del hp
    az.Plan.on_device(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dp = az.Plan.on_device(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), device=dev)
    torch.cuda.synchronize()
    dev_s = time.perf_counter() - t0
    line = dict(npix=g.npix, npt=inst.npt, nnz=dp.nnz, host_build_upload_s=host_s,
                device_build_s=dev_s, speedup=host_s / dev_s)
    del dp
    torch.cuda.empty_cache()
    return line


def full_split_line(az, torch, np, synth, dev, reps=50):
    """Full pixel splitting (Section 4.2) of the c2 frame: host and device
    plan builds, and the raw-frame step with the four corrections in the
    default layout (the same kernels as the bounding-box step, over the
    full-split coefficients)."""
    c = synth.C2
    inst = synth.instance(c["n"], c["seed"], corrections=True)
    g = inst.geom
    t0 = time.perf_counter()
    plan = az.Plan(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), split="full", device=dev)
    torch.cuda.synchronize()
    host_s = time.perf_counter() - t0
    az.Plan.on_device(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), split="full",
                      device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dp = az.Plan.on_device(g.h, g.w, inst.npt, center=(g.center_y, g.center_x), split="full",
                           device=dev)
    torch.cuda.synchronize()
    dev_s = time.perf_counter() - t0
    del dp
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).to(dev)
    plan.set_corrections(t(inst.dark), t(inst.flat), t(inst.solid), t(inst.polar))
    raw = t(inst.raw)
    outs = tuple(torch.empty(inst.npt, dtype=torch.float64, device=dev) for _ in range(3))
    ms = _timed(torch, lambda: plan.integrate_raw(raw, out=outs), reps)
    nnz = plan.nnz
    by = raw_bytes(nnz, g.npix, inst.npt, 8, plan.correction_bytes())
    line = dict(npix=g.npix, npt=inst.npt, nnz=nnz, layout=plan.layout(),
                host_build_upload_s=host_s, device_build_s=dev_s, step_ms=ms,
                step_bytes=by, step_gbs=by / (ms * 1e6), step_frac=by / (ms * 1e6) / HBM_PEAK_GBS,
                elements_per_s=g.npix / (ms * 1e-3))
    del plan
    torch.cuda.empty_cache()
    return line


def stream_copy_line(torch, dev, reps=20):
    """The measured streaming ceiling: a plain device-to-device copy of 1 GiB
    (read + write counted), beside the 8 TB/s HBM specification."""
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    ms = _timed(torch, lambda: dst.copy_(src), reps)
    by = 2 * src.numel() * 8
    del src, dst
    torch.cuda.empty_cache()
    return dict(bytes=by, ms=ms, gbs=by / (ms * 1e6), frac=by / (ms * 1e6) / HBM_PEAK_GBS)


def cpu_baseline(np, synth):
    """The FP64 oracle on the host: one full ~1e7-pixel frame per repetition
    (correction + integration; the matrix is built beforehand, untimed, as
    the GPU plan is)."""
    import oracle
    c = synth.C2
    inst = synth.instance(c["n"], c["seed"], corrections=True)
    g = inst.geom
    t0 = time.perf_counter()
    m = oracle.build_matrix(h=g.h, w=g.w, pixel_y=g.pixel_y, pixel_x=g.pixel_x,
                            center_y=g.center_y, center_x=g.center_x, dist=g.dist,
                            wavelength=g.wavelength, npt=inst.npt)
    log(f"[cpu] oracle matrix built in {time.perf_counter() - t0:.1f}s")
    best = None
    total = 0.0
    reps = 0
    while reps < 40 and total < 10.0:
        t0 = time.perf_counter()
        x = oracle.correct(inst.raw, inst.dark, inst.flat, inst.solid, inst.polar)
        oracle.integrate(m, x)
        dt = time.perf_counter() - t0
        total += dt
        reps += 1
        best = dt if best is None else min(best, dt)
    return dict(value=g.npix / best, unit="elements/s", cores=1, kind="oracle",
                sample=f"full 3162x3163 frame, correction + integration, best of {reps} "
                       f"({best:.2f} s each; matrix built beforehand, untimed); "
                       f"single-threaded NumPy",
                host_cpu=host_cpu_model(), host_cpu_count=os.cpu_count(),
                host_cpus_usable=len(os.sched_getaffinity(0)))


def host_cpu_model():
    """The host CPU's model name (first entry of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path "
              "shards by instance or by image band, see the design notes", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1412_6367_amd as az
    import synth

    dev = torch.device("cuda:0")
    az.lib()
    flush = Flush(torch, dev)
    line64, plan, outs, frame = pipeline_line(az, torch, np, synth, dev, "f64", args.steps,
                                              args.warmup)
    log(f"[f64] {json.dumps(line64)}")
    es64 = 8
    cold64 = cold_line(torch, plan, outs, frame, line64["npix"], line64["npt"], line64["nnz"],
                       es64, flush)
    log(f"[f64 flushed] {json.dumps(cold64)}")
    del plan, outs, frame
    torch.cuda.empty_cache()
    result = {
        "metric": "elements/s and fraction of HBM roofline, plain vs batched+adjoint",
        "value": line64["elements_per_s"],
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": line64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "c2: one 3162x3163 int32 frame (~1e7 px), raw values uniform in "
                        "[0, 2^20), dark/flat/solid/polar corrections, bounding-box split, "
                        "3162 radial bins, float64 storage and accumulation; step = cast + "
                        "correction + sparse gather integration (I, W, U), the correction "
                        "applied inside the integration (1/norm folded into the "
                        "coefficients and the dark term summed once per correction set, "
                        "per the plan's stage)",
            "npix": line64["npix"], "npt": line64["npt"], "nnz": line64["nnz"],
        },
        # headline: the step with L2 and MALL flushed before every launch (the
        # benchmark protocol); the steady-state figure of the timed region,
        # where frames follow each other and the caches keep what the
        # previous frame left, is under "warm"
        "roofline": {
            "bound": "hbm",
            "kernel": kernel_of(line64),
            "achieved": cold64["step_gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": cold64["step_frac"],
            "traffic": measured_traffic("c2_f64_flushed"),
            "bytes_per_launch": line64["step_bytes"],
            "avg_launch_ms": cold64["step_ms"],
            "cache": "flushed: " + cold64["protocol"],
            "warm": {
                "achieved": line64["step_gbs"],
                "frac": line64["step_frac"],
                "avg_launch_ms": line64["step_ms"],
                "traffic": measured_traffic("c2_f64"),
                "cache": "warm: back-to-back steps of the timed region, 4 frames rotating",
            },
        },
        "lines": {"c2_f64": line64, "c2_f64_cold": cold64},
    }
    want = set(args.only.split(",")) if args.only else None
    run = lambda name: (not args.main_only) and (want is None or name in want)
    for name, dt, accum, stage in (("c2_f32", "f32", "f64", None),
                                   ("c2_f32_kahan", "f32", "kahan32", None),
                                   ("c2_f64_fold", "f64", "f64", "fold"),
                                   ("c2_f32_fold", "f32", "f64", "fold")):
        if not run(name):
            continue
        l32, p32, o32, f32 = pipeline_line(az, torch, np, synth, dev, dt, args.steps,
                                           args.warmup, accum=accum, stage=stage)
        l32["cold"] = cold_line(torch, p32, o32, f32, l32["npix"], l32["npt"], l32["nnz"],
                                8 if dt == "f64" else 4, flush)
        result["lines"][name] = l32
        log(f"[{name}] {json.dumps(l32)}")
        del p32, o32, f32
        torch.cuda.empty_cache()
    if run("c3"):
        result["lines"]["c3"] = batch_line(az, torch, np, synth, dev, synth.C3, "f64",
                                           False, True)
        log(f"[c3] {json.dumps(result['lines']['c3'])}")
    if run("c4"):
        result["lines"]["c4"] = adjoint_line(az, torch, np, synth, dev)
        log(f"[c4] {json.dumps(result['lines']['c4'])}")
    if run("c5"):
        result["lines"]["c5"] = batch_line(az, torch, np, synth, dev, synth.C5, "f32",
                                           True, True)
        log(f"[c5] {json.dumps(result['lines']['c5'])}")
    if run("stream_copy"):
        result["lines"]["stream_copy"] = stream_copy_line(torch, dev)
        log(f"[stream_copy] {json.dumps(result['lines']['stream_copy'])}")
    for name, fn in (("c2_fuse_stage", fuse_stage_line), ("c2_fused", fused_line),
                     ("c2_2d", two_d_line), ("c2_plan_build", plan_build_line),
                     ("c2_full_split", full_split_line)):
        if run(name):
            result["lines"][name] = fn(az, torch, np, synth, dev)
            log(f"[{name}] {json.dumps(result['lines'][name])}")
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(np, synth)
        log(f"[cpu] {json.dumps(result['cpu_baseline'])}")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
