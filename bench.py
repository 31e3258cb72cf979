#!/usr/bin/env python3
"""Benchmark of the Fourier ADI hot path on one MI355X.

One step = one classical ADI reduction (recentring shift of every frame,
median PSF, subtraction, three-shear derotation, median combine) of a
SPHERE-like cube of 4096 frames of 1024 x 1024 float32 (zero-padded to
2048 x 2048), with the cube already resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Other workloads print their own JSON line:

    python bench.py --workload batch    64 uneven cubes (T log-uniform in
        [32, 2048], N in {256, 512, 1024, 2048}) reduced in place by one
        batched call, against one call per cube
    python bench.py --workload served   Poisson arrivals (20 requests/s) of
        such cubes through the request loop (HBM-budget admission, four
        streams), against one request at a time
    python bench.py --workload window   ADI with the per-frame PSF of the
        paper's frame selection, 1024 frames of 512^2
    python bench.py --workload window_night  the same over a whole night,
        16384 frames of 256^2 (the per-frame medians in row groups)
    python bench.py --workload register registration (centroid + Moffat fit)
        of 1024 frames of 512^2
    python bench.py --workload preprocess  pre-processing of Sect. 3.2 of
        1024 frames of 512^2: star-masked master skies of 8 groups of 128
        frames, nearest-sky subtraction, bad-pixel map and repair
    python bench.py --workload mfma     one 32-point DFT stage of the line
        passes as a DFT-as-GEMM on the matrix cores (v_mfma_f32_32x32x2f32)
        against the register codelet, both checked against a direct DFT
    python bench.py --workload quality  the image-quality test of Sect. 4.1:
        256 frames of 1024^2 shifted by (3.5, 2.7) px and back and rotated by
        11.3 deg and back, residual RMS in 2-px annuli; the third-order
        spline curve of the paper (scipy, CPU, first frame) is reported beside
"""

import argparse
import json
import math
import os
import sys
import time

METRIC = "frames shifted+rotated/s at 1024² FP32 (% HBM roofline); cube p50/p99 latency"
# MI355X published peaks: HBM3E bandwidth and the FP32 vector rate.
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
# Derived, not published: the FP32 vector rate without packed instructions
# (these kernels are built without them): 256 CUs x 4 SIMDs x 16 lanes x
# 2 flop per FMA x 2.4 GHz = 78.6 TFLOP/s.
FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
HERE = os.path.dirname(os.path.abspath(__file__))


def sources_sha256():
    """Hash of the library sources; a traffic record taken from other sources
    no longer describes the kernels that run."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(HERE, "paper_1510_04331_amd", "csrc", "*"))):
        if not os.path.isfile(f):
            continue
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def read_traffic(path, fam, N, P):
    """Measured HBM bytes per frame of one kernel family (rocprofv3 FETCH_SIZE +
    WRITE_SIZE, calibrated), or None when absent or taken from other sources."""
    try:
        with open(path) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    sha = [ln.split()[1] for ln in lines if ln.startswith("source_sha256 ")]
    if not sha or sha[0] != sources_sha256():
        return None
    for ln in lines:
        f = ln.split()
        if len(f) == 5 and f[0] == "traffic" and f[1] == fam and f[2] == "N=%d" % N and f[3] == "P=%d" % P:
            return float(f[4].split("=")[1])
    return None

# Algorithmic HBM bytes per frame of each kernel family (float32, N x N frames,
# working size P): one read of every stored input value and one write of every
# stored output value; zero padding is never read, cropped values never written.
def alg_bytes_per_frame(fam, N, P, T):
    n2, nP = N * N * 4, N * P * 4
    return {
        "shift_y": 2 * n2,
        "shift_x": 2 * n2,
        "shear_x1": n2 + nP,
        "shear_y": 2 * nP,
        "shear_x2": nP + n2,
        # both medians of a step, per frame: the PSF median reads the stack and
        # writes it back as residuals, the final one reads it (plus one image
        # each); bench.py averages them over the step's two launches
        "median": 3 * n2 + 2 * n2 / T,
    }.get(fam)


# Nominal flops per frame of each line pass: every job is two real lines
# packed in one complex line, transformed forward and back at length P
# (5 P log2 P flops per complex transform).
def alg_flops_per_frame(fam, N, P):
    pairs = {"shift_y": N // 2, "shift_x": N // 2, "shear_x1": N // 2, "shear_y": P // 2,
             "shear_x2": N // 2}.get(fam)
    if pairs is None:
        return None
    return pairs * 2 * 5 * P * math.log2(P)


FAMILIES = ("shift_y", "shift_x", "shear_x1", "shear_y", "shear_x2", "median", "aux")


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle, frames spread over a process pool (the
# paper's temporal scheme).  Runs before the GPU is touched.
# ---------------------------------------------------------------------------
def _oracle_frame(args):
    import numpy as np
    import oracle as O
    f, dx, dy, ang = args
    s = O.shift(f, dx, dy)
    r = O.rotate(s, -ang)
    return float(np.sum(r))


def cpu_baseline(frames_per_core=2):
    import multiprocessing as mp
    import synth
    cores = min(os.cpu_count() or 1, 16)
    p = synth.make_params(3)
    idx = list(range(frames_per_core * cores))
    frames = synth.render_host(p, frames=idx)
    work = [(frames[i].astype("float64"), p.dx[i], p.dy[i], p.parang[i]) for i in range(len(idx))]
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_frame, work, chunksize=1)
    dt = time.perf_counter() - t0
    return {"value": len(idx) / dt, "unit": "frames/s", "cores": cores, "kind": "oracle",
            "sample": "%d frames of the 4096 x 1024^2 cube (padded to 2048^2), float64 oracle shift + "
                      "three-shear rotation per frame, one process per core (median steps excluded; "
                      "they are O(T N^2) and under 1%% of the oracle's time); wall %.1f s"
                      % (len(idx), dt)}


# ---------------------------------------------------------------------------
# Batched and served workloads.  Each cube's frames are copies of a pool of
# rendered frames of its size (64 per size, generated once on the device), so
# that filling a cube costs one device copy; the per-frame shifts and angles
# are the cube's own.
# ---------------------------------------------------------------------------
POOL_FRAMES = 64


def _pools(torch, dev, sizes):
    import synth
    pools = {}
    for k, N in enumerate(sorted(set(sizes))):
        p = synth.make_params(2, seed=synth.BASE_SEED + 100 + k, T=POOL_FRAMES, N=N)
        pools[N] = synth.render_device(p, dev)
    torch.cuda.synchronize()
    return pools


def _fill(pools, N):
    src = pools[N]

    def fill(cube, stream=None):
        T = cube.shape[0]
        for s0 in range(0, T, POOL_FRAMES):
            n = min(POOL_FRAMES, T - s0)
            cube[s0:s0 + n].copy_(src[:n])
    return fill


def _tune_classes(G, shapes):
    """Autotune every (median class, size) pair of a workload (before its
    cubes are allocated: tuning takes a full-size workspace of its own)."""
    import torch
    reps = {}
    for T, N in shapes:
        key = ((T + 63) // 64 - 1).bit_length(), N
        reps[key] = max(reps.get(key, 0), T)
    for (_, N), T in sorted(reps.items()):
        G.autotune(T, N)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return G.tuning_export()


def bench_batch(args):
    import numpy as np
    import torch
    import paper_1510_04331_amd as G
    import synth
    dev = torch.device("cuda:0")
    ps = synth.make_batch_params(64, with_screen=False)
    tuning = _tune_classes(G, [(p.T, p.N) for p in ps])
    pools = _pools(torch, dev, [p.N for p in ps])
    cubes = [torch.empty((p.T, p.N, p.N), dtype=torch.float32, device=dev) for p in ps]
    fills = [_fill(pools, p.N) for p in ps]
    dx = [torch.tensor(p.dx, dtype=torch.float64, device=dev) for p in ps]
    dy = [torch.tensor(p.dy, dtype=torch.float64, device=dev) for p in ps]
    pa = [torch.tensor(p.parang, dtype=torch.float64, device=dev) for p in ps]
    ws = torch.empty(G.batch_workspace_size(cubes, inplace=True), dtype=torch.uint8, device=dev)
    frames = sum(p.T for p in ps)
    print("batch: %d cubes, %d frames, %.1f GiB" % (len(ps), frames, sum(c.numel() for c in cubes) * 4 / 2**30),
          file=sys.stderr, flush=True)

    def refill():
        for c, f in zip(cubes, fills):
            f(c)
        torch.cuda.synchronize()

    def timed(fn, steps):
        ts = []
        for _ in range(steps):
            refill()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return ts

    def batched():
        G.adi_reduce_batch(cubes, dx, dy, pa, inplace=True, workspace=ws)

    def per_cube():
        for i in range(len(cubes)):
            G.adi_reduce_batch([cubes[i]], [dx[i]], [dy[i]], [pa[i]], inplace=True, workspace=ws)

    timed(batched, args.warmup)
    tb = timed(batched, args.steps)
    print("batched done", file=sys.stderr, flush=True)
    timed(per_cube, 1)
    tp = timed(per_cube, args.steps)
    graph = G.AdiGraph(cubes, dx, dy, pa, inplace=True, workspace=ws)
    timed(graph.launch, 1)
    tg = timed(graph.launch, args.steps)
    graph.close()
    print("graph done", file=sys.stderr, flush=True)
    mb, mp, mg = min(tb), min(tp), min(tg)

    # many small cubes (64 cubes of 16 frames of 128^2): one batched call
    # against one call per cube, where launches rather than bytes set the time
    sq = [synth.make_params(1, seed=synth.BASE_SEED + 400 + k) for k in range(64)]
    scubes = [torch.from_numpy(synth.render_host(q)).to(dev) for q in sq]
    sargs = ([torch.tensor(q.dx, dtype=torch.float64, device=dev) for q in sq],
             [torch.tensor(q.dy, dtype=torch.float64, device=dev) for q in sq],
             [torch.tensor(q.parang, dtype=torch.float64, device=dev) for q in sq])
    sws = torch.empty(G.batch_workspace_size(scubes), dtype=torch.uint8, device=dev)

    def small_batched():
        G.adi_reduce_batch(scubes, *sargs, workspace=sws)

    def small_per_cube():
        for k in range(len(scubes)):
            G.adi_reduce_batch([scubes[k]], [sargs[0][k]], [sargs[1][k]], [sargs[2][k]], workspace=sws)

    def best_ms(fn, reps=20):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return 1e3 * min(ts)
    small_frames = sum(q.T for q in sq)
    sb_ms, sp_ms = best_ms(small_batched), best_ms(small_per_cube)

    # the plain per-frame path on a sample of the batch (the first cube of
    # each size): every frame shifted and rotated by its own calls
    def per_frame_rate():
        frames, t_all = 0, 0.0
        for N in sorted(set(p.N for p in ps)):
            k = next(i for i, p in enumerate(ps) if p.N == N)
            c = cubes[k]
            fills[k](c)
            n = min(c.shape[0], 32)
            one_dx = [dx[k][i:i + 1] for i in range(n)]
            one_dy = [dy[k][i:i + 1] for i in range(n)]
            one_pa = [pa[k][i:i + 1] for i in range(n)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(n):
                f = G.shift(c[i:i + 1], one_dx[i], one_dy[i])
                G.rotate(f, -one_pa[i], out=f)
            torch.cuda.synchronize()
            t_all += time.perf_counter() - t0
            frames += n
        return frames / t_all

    pf_rate = per_frame_rate()

    # small cube (16 frames of 128^2): host-side cost of one eager call vs one
    # graph replay, back to back on one stream
    q = synth.make_params(1)
    small = torch.from_numpy(synth.render_host(q)).to(dev)
    sdx, sdy, spa = (torch.tensor(a, dtype=torch.float64, device=dev) for a in (q.dx, q.dy, q.parang))
    sws = torch.empty(G.batch_workspace_size([small]), dtype=torch.uint8, device=dev)
    reps = 200

    def per_call(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e6
    eager_us = per_call(lambda: G.adi_reduce_batch([small], [sdx], [sdy], [spa], workspace=sws))
    sg = G.AdiGraph([small], [sdx], [sdy], [spa], workspace=sws)
    graph_us = per_call(sg.launch)
    sg.close()
    out = {"metric": "frames reduced/s, 64 uneven cubes in one batched call (vs one call per cube)",
           "value": round(frames / mb, 1), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(1e3 * mb, 3), "higher_is_better": True,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "64 cubes, T log-uniform in [32, 2048], N in {256,512,1024,2048}, P = 2N, "
                                  "in-place full ADI reduction", "frames": frames,
                      "bytes": int(sum(c.numel() for c in cubes) * 4)},
           "per_cube_path": {"value": round(frames / mp, 1), "ms_per_step": round(1e3 * mp, 3)},
           "graph_replay": {"value": round(frames / mg, 1), "ms_per_step": round(1e3 * mg, 3)},
           "tuning": tuning.strip().split("\n"),
           "small_cubes_64x16x128": {"batched_frames_per_s": round(small_frames / (sb_ms * 1e-3), 1),
                                     "per_cube_frames_per_s": round(small_frames / (sp_ms * 1e-3), 1),
                                     "batched_ms": round(sb_ms, 3), "per_cube_ms": round(sp_ms, 3)},
           "per_frame_path": {"frames_shifted_rotated_per_s": round(pf_rate, 1),
                              "sample": "first cube of each size, up to 32 frames each, one shift and one rotation "
                                        "call per frame"},
           "small_cube_16x128_us_per_reduction": {"eager": round(eager_us, 1), "graph": round(graph_us, 1)},
           "step_ms_all": [round(1e3 * t, 3) for t in tb]}
    print(json.dumps(out), flush=True)


def bench_window(args, night=False):
    """ADI with the per-frame PSF of the paper's frame selection on the
    NACO-like cube (1024 frames of 512^2): frames 2 s apart, angles spanning
    60 degrees, t_max = 1200 s, alpha_min = 2 arcsin(1 FWHM / (2 x 10 px)),
    so each frame's PSF comes from the frames 23 to 35 degrees away.

    night: a whole night instead, 16384 frames of 256^2 2 s apart (9.1 h),
    angles spanning 180 degrees, t_max = 1200 s, alpha_min for 1 FWHM at
    50 px (4.6 degrees); the per-frame medians then run in row groups."""
    import numpy as np
    import torch
    import paper_1510_04331_amd as G
    import synth
    dev = torch.device("cuda:0")
    if night:
        p = synth.make_params(2, T=16384, N=256)
        p.parang = np.linspace(-90.0, 90.0, p.T)
        r_min = 50.0
    else:
        p = synth.make_params(2)
        r_min = 10.0
    cube = synth.render_device(p, dev)
    times = np.arange(p.T, dtype=np.float64) * 2.0
    t_max, amin = 1200.0, G.alpha_min_deg(1.0, 4.0, r_min)
    ws = torch.empty(G.workspace_size(5, p.T, p.N), dtype=torch.uint8, device=dev)
    G.autotune(p.T, p.N)
    for _ in range(args.warmup):
        G.adi_reduce_window(cube, p.dx, p.dy, p.parang, times, t_max, amin, workspace=ws)
    torch.cuda.synchronize()
    G.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        G.adi_reduce_window(cube, p.dx, p.dy, p.parang, times, t_max, amin, workspace=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    med_ms, _ = G.timing_read("median")
    G.timing_enable(False)
    sel_n = np.zeros(p.T)
    for i0 in range(0, p.T, 1024):                        # selected frames per row, in slices of rows
        rows = slice(i0, min(p.T, i0 + 1024))
        sel_n[rows] = ((np.abs(times[None, :] - times[rows, None]) < t_max) &
                       (np.abs(p.parang[None, :] - p.parang[rows, None]) > amin)).sum(axis=1)
    out = {"metric": "frames reduced/s, ADI with the per-frame PSF of the frame selection",
           "value": round(p.T / dt, 1), "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(1e3 * dt, 3), "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "%s, %d frames of %dx%d (P = %d), frames 2 s apart, angles over %g deg, "
                                  "t_max 1200 s, alpha_min %.2f deg"
                                  % ("whole night" if night else "NACO-like cube", p.T, p.N, p.N, p.P,
                                     float(p.parang[-1] - p.parang[0]), amin),
                      "mean_selected_frames": round(float(sel_n.mean()), 1),
                      "rows_selecting_nothing": int((sel_n == 0).sum())},
           "median_ms_per_step": round(med_ms / args.steps, 3)}
    print(json.dumps(out), flush=True)


def bench_register(args):
    """Registration of the NACO-like cube (1024 frames of 512^2): brightest
    pixel over the whole frame, patch centroid, Moffat fit over 24 x 24."""
    import torch
    import paper_1510_04331_amd as G
    import synth
    dev = torch.device("cuda:0")
    p = synth.make_params(2)
    cube = synth.render_device(p, dev)
    for _ in range(args.warmup):
        G.register(cube, 500.0, 4, 5000, half=12)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = G.register(cube, 500.0, 4, 5000, half=12)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    flags = res["flags"].cpu()
    err = float(max((res["dx"].cpu().numpy() - p.dx).__abs__().max(), (res["dy"].cpu().numpy() - p.dy).__abs__().max()))
    out = {"metric": "frames registered/s (centroid + Moffat fit)", "value": round(p.T / dt, 1), "unit": "frames/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * dt, 3),
           "higher_is_better": True, "dtype": "f64 fit on f32 frames", "data": "synthetic",
           "config": {"workload": "NACO-like cube, 1024 frames of 512x512, threshold 500, fit box 24x24"},
           "centroid_found": int((flags & 1).sum()), "fit_converged": int(((flags >> 1) & 1).sum()),
           "max_shift_error_px": round(err, 4)}
    print(json.dumps(out), flush=True)


def bench_preprocess(args):
    """Pre-processing of Sect. 3.2 on the NACO-like cube (1024 frames of
    512^2) with a 100 ADU sky and 300 hot, cold or dead pixels added: one step
    masks the star (radius 20 px) in a copy, takes the NaN-aware median sky of
    each group of 128 frames, fills the masked hole of each sky by neighbour
    medians, subtracts from every frame the sky nearest in time, maps the bad
    pixels of a dark frame (5 sigma, one pass: the hot and dead pixels; the
    cold ones hide inside the sigma that the hot ones inflate) and repairs
    them in the cube by neighbour medians."""
    import numpy as np
    import torch
    import paper_1510_04331_amd as G
    import synth
    dev = torch.device("cuda:0")
    p = synth.make_params(2)
    T, N = p.T, p.N
    raw = synth.render_device(p, dev)
    raw += 100.0
    rng = np.random.default_rng(synth.BASE_SEED + 7)
    bad = rng.choice(N * N, 300, replace=False)
    vals = torch.tensor(np.where(np.arange(300) % 3 == 0, 5.0e4, np.where(np.arange(300) % 3 == 1, -500.0, np.nan)),
                        dtype=torch.float32, device=dev)
    raw.view(T, N * N)[:, torch.from_numpy(bad).to(dev)] = vals
    dark = torch.from_numpy(rng.normal(100.0, 5.0, (N, N)).astype(np.float32)).to(dev)
    dark.view(N * N)[torch.from_numpy(bad).to(dev)] = vals
    times = np.arange(T, dtype=np.float64) * 2.0
    xs, ys = N / 2.0 - p.dx, N / 2.0 - p.dy                       # star position of every frame
    groups = 8
    gs = T // groups
    sky_times = torch.tensor([times[g * gs:(g + 1) * gs].mean() for g in range(groups)], dtype=torch.float64,
                             device=dev)
    skies = torch.empty((groups, N, N), dtype=torch.float32, device=dev)
    masked = torch.empty_like(raw)
    work = torch.empty_like(raw)

    def step():
        masked.copy_(raw)
        G.mask_disk(masked, xs, ys, 20.0)
        for g in range(groups):
            G.median_nan(masked[g * gs:(g + 1) * gs], out=skies[g])
        sky_passes = G.badpix_fix(skies)
        work.copy_(raw)
        G.subtract_nearest(work, times, skies, sky_times)
        m, stats = G.badpix_map(dark, 5.0)
        return sky_passes, G.badpix_fix(work, m), m

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sky_passes, passes, m = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    left = int(torch.isnan(work).sum())
    out = {"metric": "frames pre-processed/s (star masks, group master skies, nearest-sky subtraction, bad-pixel "
                     "map and repair)", "value": round(T / dt, 1), "unit": "frames/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * dt, 3), "higher_is_better": True,
           "dtype": "f32 (f64 statistics)", "data": "synthetic",
           "config": {"workload": "NACO-like cube, 1024 frames of 512x512 + 100 ADU sky, 300 hot/cold/NaN pixels; "
                                  "8 master skies of 128 frames, star masks of 20 px, 5-sigma map of a dark frame"},
           "bad_pixels_mapped": int(m.sum()), "sky_fill_passes": int(sky_passes), "repair_passes": int(passes),
           "nan_left": left}
    print(json.dumps(out), flush=True)


def bench_quality(args):
    """Image-quality test of Sect. 4.1 on SPHERE-like frames: one step is the
    double shift and the double rotation of every frame plus the annular RMS
    of both residual stacks."""
    import numpy as np
    import torch
    import paper_1510_04331_amd as G
    import synth
    from scipy import ndimage
    dev = torch.device("cuda:0")
    T = min(args.frames, 256)
    p = synth.make_params(3, T=T, N=args.size)
    cube = synth.render_device(p, dev)
    N = p.N
    dx, dy = np.full(T, 3.5), np.full(T, 2.7)
    ang = np.full(T, 11.3)
    n_rings = int(N * 0.7072 // 2.0) + 1

    def step():
        s = G.shift(G.shift(cube, dx, dy), -dx, -dy)
        rs, _ = G.annular_rms(s, cube, 2.0, n_rings)
        del s
        r = G.rotate(G.rotate(cube, ang), -ang)
        rr, _ = G.annular_rms(r, cube, 2.0, n_rings)
        return rs, rr

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rs, rr = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    base, _ = G.annular_rms(cube[:1], None, 2.0, n_rings)
    f0 = cube[0].double().cpu().numpy()
    peak = float(f0.max())
    # the paper's comparison curve: third-order spline round trips of frame 0
    spl_s = ndimage.shift(ndimage.shift(f0, (2.7, 3.5), order=3, mode="constant"), (-2.7, -3.5), order=3,
                          mode="constant")
    spl_r = ndimage.rotate(ndimage.rotate(f0, 11.3, reshape=False, order=3, mode="constant"), -11.3, reshape=False,
                           order=3, mode="constant")
    f0t = torch.from_numpy(f0.astype(np.float32)).to(dev)
    ss, _ = G.annular_rms(torch.from_numpy(spl_s.astype(np.float32)).to(dev), f0t, 2.0, n_rings)
    sr, _ = G.annular_rms(torch.from_numpy(spl_r.astype(np.float32)).to(dev), f0t, 2.0, n_rings)
    radii = [r for r in (10, 25, 50, 100, 200, 400) if r // 2 < n_rings]
    prof = lambda v: {str(r): float("%.3g" % (float(v[r // 2]) / peak)) for r in radii}
    out = {"metric": "frames round-tripped/s (double shift + double rotation + annular RMS of both)",
           "value": round(T / dt, 1), "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(1e3 * dt, 3), "higher_is_better": True, "dtype": "f32 (f64 sums)",
           "data": "synthetic",
           "config": {"workload": "%d SPHERE-like frames of %dx%d, shift (3.5, 2.7) px and back, rotation 11.3 deg "
                                  "and back, RMS in 2-px annuli" % (T, N, N)},
           "profile_radius_px_over_peak": {
               "image": prof(base.cpu().numpy()[0]),
               "fourier_shift_residual": prof(rs.cpu().numpy()[0]),
               "spline_shift_residual": prof(ss.cpu().numpy()),
               "fourier_rotation_residual": prof(rr.cpu().numpy()[0]),
               "spline_rotation_residual": prof(sr.cpu().numpy())}}
    print(json.dumps(out), flush=True)


def bench_mfma(args):
    """Runs the measurement program built next to the library (one DFT stage
    on the matrix cores against the register codelet) and prints its result
    as one JSON line."""
    import subprocess
    exe = os.path.join(HERE, "paper_1510_04331_amd", "dft32_mfma")
    if not os.path.exists(exe):
        raise RuntimeError("dft32_mfma is not built; run __graft_entry__.build()")
    r = subprocess.run([exe, str(1 << 20), "64"], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("dft32_mfma failed (%d): %s %s" % (r.returncode, r.stdout, r.stderr))
    res = json.loads(r.stdout.strip().splitlines()[-1])
    out = {"metric": "time per 32-point complex DFT stage and vector, matrix cores vs register codelet",
           "value": res["mfma_over_valu_time"], "unit": "ratio (mfma / valu time)", "n_gpus": 1, "steps": 5,
           "warmup": 1, "ms_per_step": res["mfma_32x32x2_f32"]["ms"], "higher_is_better": False, "dtype": "f32",
           "data": "synthetic", "config": {"workload": res["what"]}, "result": res}
    print(json.dumps(out), flush=True)


def bench_served(args):
    import numpy as np
    import torch
    import synth
    from paper_1510_04331_amd import serve
    dev = torch.device("cuda:0")
    n = args.requests
    arr = synth.make_arrivals(n, rate=args.rate)
    ps = synth.make_batch_params(n, seed=synth.BASE_SEED + 5, with_screen=False)
    pools = _pools(torch, dev, [p.N for p in ps])
    import paper_1510_04331_amd as G
    _tune_classes(G, [(p.T, p.N) for p in ps])
    free_b, total_b = torch.cuda.mem_get_info(dev)
    budget = int(args.budget_gib * 2**30) if args.budget_gib else int(0.6 * free_b)

    def requests():
        return [serve.Request(rid=i, arrival=float(arr[i]), T=p.T, N=p.N, dx=p.dx, dy=p.dy, parang=p.parang,
                              fill=_fill(pools, p.N)) for i, p in enumerate(ps)]

    res = {}
    for name, slots, mb in (("served", args.slots, args.max_batch), ("one_at_a_time", 1, 1)):
        ex = serve.TorchExecutor(dev, slots)
        adm = serve.Admission(budget, slots, mb, ex.group_bytes, cost=ex.cost, big_cost=args.big_ms)
        st = serve.run(requests(), ex, adm)
        torch.cuda.synchronize()
        res[name] = st.summary()
        print("%s: %s" % (name, json.dumps(res[name])), file=sys.stderr, flush=True)
    s = res["served"]
    out = {"metric": "frames/s served at %.0f requests/s; p50/p99 request latency" % args.rate,
           "value": s["frames_per_s"], "unit": "frames/s", "n_gpus": 1, "steps": n, "warmup": 0,
           "ms_per_step": None, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "Poisson arrivals, %d requests at %.1f/s, cubes as in the 64-cube batch "
                                  "(T log-uniform in [32, 2048], N in {256..2048})" % (n, args.rate),
                      "slots": args.slots, "max_batch": args.max_batch, "hbm_budget_bytes": budget,
                      "large_request_ms": args.big_ms},
           "latency_ms": s["latency_ms"], "served": s, "one_at_a_time": res["one_at_a_time"]}
    print(json.dumps(out), flush=True)


def roofline(d, fam, traffic):
    """The dominant kernel against the HBM roofline: algorithmic bytes per
    launch (one read of every stored input, one write of every stored output)
    over the mean launch duration, against the 8 TB/s peak.  The line passes'
    FFT arithmetic is reported beside it: nominal flops (5 P log2 P per
    complex transform) against the published FP32 peak and against the
    derived non-packed rate."""
    r = {"bound": "hbm", "kernel": fam, "achieved": round(d["achieved_GBps"], 1), "peak": HBM_PEAK_GBS,
         "unit": "GB/s", "frac": round(d["achieved_GBps"] / HBM_PEAK_GBS, 4), "traffic": traffic,
         "alg_bytes_per_launch": int(d["alg_bytes_per_launch"]), "avg_launch_ms": round(d["avg_launch_ms"], 4)}
    if "achieved_TFLOPs" in d:
        r["alu"] = {"achieved_TFLOPs": round(d["achieved_TFLOPs"], 2),
                    "peak_fp32_published_TFLOPs": FP32_PEAK_TFLOPS,
                    "frac_published": round(d["achieved_TFLOPs"] / FP32_PEAK_TFLOPS, 4),
                    "peak_fp32_nonpacked_derived_TFLOPs": round(FP32_NONPACKED_TFLOPS, 1),
                    "frac_nonpacked": round(d["achieved_TFLOPs"] / FP32_NONPACKED_TFLOPS, 4)}
    return r


def _oracle_shift_rotate(args):
    import numpy as np
    import oracle as O
    f, dx, dy, ang = args
    s = O.shift(f, dx, dy)
    r = O.rotate(s, -ang)
    return r, float(np.sum(r))


def verify_frames(G, torch, cube, p, frames):
    """Per-frame error of the shift + derotation against the FP64 oracle on
    sampled frames, and flux conservation on the zero-padded frames, outside
    the timed region.  The GPU side runs the whole cube through the same
    passes as the reduction (shift, then rotation chunks of the default
    size); the oracle recomputes the sampled frames one by one."""
    import multiprocessing as mp
    import numpy as np
    T, N = p.T, p.N
    shifted = G.shift(cube, p.dx, p.dy)
    rot = G.rotate(shifted, -p.parang)
    del shifted
    torch.cuda.synchronize()
    got = {t: rot[t].double().cpu().numpy() for t in frames}
    del rot
    host = {t: cube[t].double().cpu().numpy() for t in frames}
    torch.cuda.empty_cache()
    with mp.get_context("spawn").Pool(min(len(frames), 16)) as pool:
        refs = pool.map(_oracle_shift_rotate, [(host[t], p.dx[t], p.dy[t], p.parang[t]) for t in frames])
    # padded flux: shift and rotation of the sampled frames on P x P output
    idx = torch.tensor(frames, device=cube.device)
    sub = cube.index_select(0, idx).contiguous()
    sp, fs = G.shift(sub, p.dx[frames], p.dy[frames], keep_padded=True, flux=True)
    rp, fr = G.rotate(sub, -p.parang[frames], keep_padded=True, flux=True)
    fs, fr = fs.cpu().numpy(), fr.cpu().numpy()
    per = []
    for k, t in enumerate(frames):
        ref, _ = refs[k]
        scale = float(np.abs(host[t]).sum())
        per.append({"frame": int(t),
                    "rel_l2": float("%.3g" % (np.linalg.norm(got[t] - ref) / np.linalg.norm(ref))),
                    "flux_err": float("%.3g" % (abs(got[t].sum() - ref.sum()) / scale)),
                    "padded_flux_err_shift": float("%.3g" % (abs(fs[k, 1] - fs[k, 0]) / scale)),
                    "padded_flux_err_rotate": float("%.3g" % (abs(fr[k, 1] - fr[k, 0]) / scale))})
    del sp, rp, sub
    torch.cuda.empty_cache()
    return {"what": "shift + derotation by -parang of sampled frames of the timed cube against the float64 oracle; "
                    "flux_err = |sum_gpu - sum_oracle| / sum|frame| (N x N windows); padded_flux_err = |sum out - sum "
                    "in| / sum|frame| over the whole P x P output", "bar": {"rel_l2": 1e-5, "flux_err": 1e-6},
            "max_rel_l2": max(q["rel_l2"] for q in per), "max_flux_err": max(q["flux_err"] for q in per),
            "frames": per}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=4096)
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=("adi", "batch", "served", "window", "window_night", "register",
                                           "preprocess", "quality", "mfma"),
                    default="adi")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip autotuning (default launch shapes; keeps tuning launches out of profiles)")
    ap.add_argument("--requests", type=int, default=1000)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--max-batch", type=int, default=8)
    ap.add_argument("--budget-gib", type=float, default=None)
    ap.add_argument("--big-ms", type=float, default=50.0,
                    help="estimated device time from which a served request runs alone")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain device copy of the cube (known bytes) before the timed steps, "
                         "to scale hardware byte counters")
    ap.add_argument("--traffic", default=None,
                    help="calibrated counter record (default: profiles/traffic_adi_<N>.txt)")
    ap.add_argument("--verify-frames", type=int, default=8,
                    help="sampled frames checked against the oracle after the timed steps (0: none)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (sharding over several GPUs is designed but not "
              "implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "served":
        return bench_served(args)
    if args.workload == "window":
        return bench_window(args)
    if args.workload == "window_night":
        return bench_window(args, night=True)
    if args.workload == "register":
        return bench_register(args)
    if args.workload == "quality":
        return bench_quality(args)
    if args.workload == "preprocess":
        return bench_preprocess(args)
    if args.workload == "mfma":
        return bench_mfma(args)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline()
        print("cpu baseline: %.3f frames/s on %d cores" % (cpu["value"], cpu["cores"]), file=sys.stderr,
              flush=True)

    import numpy as np
    import torch
    import paper_1510_04331_amd as G
    import synth

    dev = torch.device("cuda:0")
    p = synth.make_params(3, T=args.frames, N=args.size)
    T, N, P = p.T, p.N, p.P
    print("generating cube T=%d N=%d on the device" % (T, N), file=sys.stderr, flush=True)
    cube = synth.render_device(p, dev)
    dx = torch.tensor(p.dx, dtype=torch.float64, device=dev)
    dy = torch.tensor(p.dy, dtype=torch.float64, device=dev)
    pa = torch.tensor(p.parang, dtype=torch.float64, device=dev)
    nws = G.workspace_size(2, T, N)
    ws = torch.empty(nws, dtype=torch.uint8, device=dev)
    tuning = "" if args.no_tune else G.autotune(T, N, workspace=ws)   # launch shapes (ws is scratch here)
    print("tuning: %s" % tuning.replace("\n", "; "), file=sys.stderr, flush=True)
    torch.cuda.synchronize()

    if args.calibrate_copy:
        scratch = torch.empty_like(cube)
        scratch.copy_(cube)
        torch.cuda.synchronize()
        print("copy calibration: %d bytes read, %d bytes written" % (cube.numel() * 4, cube.numel() * 4),
              file=sys.stderr, flush=True)
        del scratch
    for _ in range(args.warmup):
        G.adi_reduce(cube, dx, dy, pa, workspace=ws)
    torch.cuda.synchronize()
    print("warmup done", file=sys.stderr, flush=True)

    G.timing_enable(True)
    step_ms = []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        final = G.adi_reduce(cube, dx, dy, pa, workspace=ws)
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - t0) * 1e3)
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t_all
    fams = {}
    for fam in FAMILIES:
        ms, n = G.timing_read(fam)
        if n:
            fams[fam] = {"ms_per_step": ms / args.steps, "launches_per_step": n / args.steps,
                         "avg_launch_ms": ms / n}
    G.timing_enable(False)
    assert torch.isfinite(final).all()
    copy_ceiling = measure_copy(torch, cube)
    verify = None
    if args.verify_frames > 0:
        rng = np.random.default_rng(synth.BASE_SEED + 11)
        fixed = [0, T - 1, min(511, T - 1), min(512, T - 1)]
        frames = sorted(set(fixed + [int(x) for x in rng.integers(0, T, max(0, args.verify_frames - 4))]))
        print("verifying frames %s against the oracle" % frames, file=sys.stderr, flush=True)
        del ws
        torch.cuda.empty_cache()
        verify = verify_frames(G, torch, cube, p, frames)

    ms_per_step = total_s * 1e3 / args.steps
    value = T / (ms_per_step / 1e3)
    # shift + rotate alone (the five line passes), from the per-kernel events
    sr_ms = sum(fams[f]["ms_per_step"] for f in ("shift_y", "shift_x", "shear_x1", "shear_y", "shear_x2")
                if f in fams)
    for fam, d in fams.items():
        b = alg_bytes_per_frame(fam, N, P, T)
        if b is None:
            continue
        frames_per_launch = T / d["launches_per_step"]
        d["alg_bytes_per_launch"] = b * frames_per_launch
        d["achieved_GBps"] = d["alg_bytes_per_launch"] / (d["avg_launch_ms"] * 1e-3) / 1e9
        fl = alg_flops_per_frame(fam, N, P)
        if fl is not None:
            d["alg_flops_per_launch"] = fl * frames_per_launch
            d["achieved_TFLOPs"] = d["alg_flops_per_launch"] / (d["avg_launch_ms"] * 1e-3) / 1e12
    dom = max((f for f in fams if "achieved_GBps" in fams[f]), key=lambda f: fams[f]["ms_per_step"])
    traffic = None
    tpath = args.traffic or os.path.join(HERE, "profiles", "traffic_adi_%d.txt" % N)
    per_frame = read_traffic(tpath, dom, N, P)
    if per_frame is not None:
        traffic = round(per_frame * T / fams[dom]["launches_per_step"])
    sl = sorted(step_ms)

    def pct(q):
        return sl[min(len(sl) - 1, int(math.ceil(q * len(sl))) - 1)]

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "SPHERE-like ADI cube: %d frames %dx%d float32, zero-padded to %dx%d; full "
                               "reduction (shift, median PSF, subtract, derotate, median combine)"
                               % (T, N, N, P, P),
                   "frames": T, "size": N, "pad": P, "parallelism": "single GPU"},
        "roofline": roofline(fams[dom], dom, traffic),
        "copy_ceiling": copy_ceiling,
        "cpu_baseline": cpu,
        "tuning": tuning.strip().split("\n") if tuning else "defaults",
        "latency_ms": {"p50": round(pct(0.5), 3), "p99": round(pct(0.99), 3)},
        "shift_rotate_frames_per_s": round(T / (sr_ms / 1e3), 1) if sr_ms else None,
        "shift_rotate_hbm_frac": round(56.0 * N * N * (T / (sr_ms / 1e3)) / (HBM_PEAK_GBS * 1e9), 4)
        if sr_ms else None,
        "kernels": {f: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}
                    for f, d in fams.items()},
        "per_frame_check": verify,
    }
    print(json.dumps(out), flush=True)


def measure_copy(torch, cube, reps=3):
    """Measured HBM ceiling beside the published peak: a plain device-to-device
    copy of the cube (torch copy_), read + write bytes over the fastest of
    `reps` copies, timed with events on the copy's stream, outside the timed
    region."""
    dst = torch.empty_like(cube)
    dst.copy_(cube)
    best = None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(cube)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    del dst
    torch.cuda.empty_cache()
    gbs = 2.0 * cube.numel() * cube.element_size() / (best * 1e-3) / 1e9
    return {"GBps": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_copy":
            2 * cube.numel() * cube.element_size(), "what": "device-to-device copy of the cube, best of %d" % reps}


if __name__ == "__main__":
    main()
