#!/usr/bin/env python3
"""Throughput of the whole hot path on one MI355X, on synthetic seeded inputs.

Headline (the batched workload the metric names): 4096 binary images of uneven
sizes (sides U{28,64,128,256}, Gaussian random fields with sigma U[2,8] px
thresholded at the median), ECT at 128 directions x 128 per-image thresholds
and Euler-Laplace at 512 xi per image (|xi| ~ U[0.01, 1]).  One step = one pass
of every stage over the batch -- per-vertex classification and ordered
compaction, sign-vector bucketing, the exact ECT and the Laplace transform --
replayed as one HIP graph (FP32 kernel values, FP64 phases and accumulation).
value = (xi, critical point) Laplace evaluations per second of step time;
ect_dirs_per_s beside it; the plain per-image FP64 loop on the same GPU gives
the batched speedup.  Inputs are resident in HBM before the timed region.

Rows for the other workloads, each timed the same way (graph replays) with its
per-stage kernel times and the roofline of its dominant kernel: grf_512 (one
512x512 field, ECT 360 x 256, Fourier/Laplace/Bessel at 4096 xi, Fourier
backward), volume_128 (128^3 volume, ECT 2048 x 256, Fourier/Laplace with a
log-scale output at 16384 xi), diff_256 (256 fields 128x128, Fourier and
Laplace at 1024 shared xi, forward and both backward passes), small_binary
(64x64, FP64), the Radon transform and exact representations, four axes.

Roofline: a kernel's average duration comes from HIP events the library
records around that kernel alone (ect_set_stage_events), on the stream it is
launched on, over K eager steps after the timed graph replays.

The cpu_baseline leg runs the FP64 oracle on a bounded sample of every
workload, times it on the host cores (all of them, then one) and compares the
GPU results with it: every row carries its error against the oracle (ECT
bit-exactness, the per-query gate ratio, normwise, strict and condition
number of the hybrid results and gradients).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ξ·crit-pt evals/s (hybrid), ECT dirs/s; batched FP32 vs plain FP64 @1e-5"
KERNELS = ("fourier", "laplace", "bessel")


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-graph", action="store_true", help="time eager steps instead of graph replays")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (timing on the host cores and every row's error against it)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-path comparisons")
    ap.add_argument("--only-headline", action="store_true", help="measure the batched workload alone")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the Radon transform and exact-representation measurements")
    ap.add_argument("--rows", default="grf,volume,diff,small",
                    help="comma-separated rows measured beside the headline (grf, volume, diff, small); "
                         "the four-axis row follows --no-4d")
    ap.add_argument("--no-4d", action="store_true", help="skip the four-axis workload")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default schedule knobs")
    ap.add_argument("--serial-ect", action="store_true",
                    help="batch step: run the ECT before the Laplace pass on one stream (no side stream)")
    ap.add_argument("--traffic-json", nargs=5,
                    metavar=("WORKLOAD", "FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="write profiles/traffic_<WORKLOAD>.json from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE "
                         "counter files of this build's bench run and of --calibrate-copy (no GPU needed)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device copy 5 times (counter calibration) and exit")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_digest(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measure_next(plan, w, dirs, thr, n, cls_counts, ord_counts, steps):
    """Radon transform at the step's thresholds (kernel time from the library's
    stage events) and the exact representations of the step's directions
    (whole-call time: every kernel of the build, sort included; then their
    binary-search evaluation at the thresholds)."""
    import numpy as np
    import torch

    from paper_2405_02256_amd import _native as N
    from paper_2405_02256_amd import hipevents, roofline

    sgn = lambda d: int(d[0] < 0) + 2 * int(d[1] < 0)
    pair = lambda e: e ^ 3 if e >= 2 else e
    c_pts = float(sum(cls_counts[0][sgn(d)] for d in w.ect_dirs))
    o_pts = float(sum(ord_counts[pair(sgn(d))] for d in w.ect_dirs))
    out = {}
    rad = plan.radon(dirs, thr)
    # the Radon call's own directions per workgroup (the plan's knobs were
    # tuned for the step's combined ECT + hybrid launch); restored afterwards
    saved = getattr(plan, "tuning", None)
    base = saved if saved is not None else (0, 2048, 0, 0)
    best = None
    from paper_2405_02256_amd import autotune as AT
    for td, ch in AT.ECT_CANDIDATES:
        plan.set_tuning(base[0], base[1], td, ch)
        ev = [(hipevents.Event(), hipevents.Event()) for _ in range(steps)]
        for a, b in ev:
            N.check(N.ect_set_stage_events(N.STAGE_ECT, a.handle, b.handle), "stage events")
            plan.radon(dirs, thr, out=rad)
        torch.cuda.synchronize()
        N.ect_set_stage_events(N.STAGE_ECT, None, None)
        t = float(np.mean([a.elapsed_ms(b) for a, b in ev]))
        if best is None or t < best[0]:
            best = (t, td, ch)
    plan.set_tuning(*base)
    ms, td_best, ch_best = best
    roof = roofline.alu_roofline("radon", n, c_pts + o_pts, ms * 1e-3)
    out["radon_thresholds"] = {"kernel_ms": ms, "dirs_per_s": len(w.ect_dirs) / (ms * 1e-3),
                               "points_streamed": c_pts + o_pts, "dirs_per_workgroup": td_best, "list_parts": ch_best or "auto", "roofline": roof}
    for kind, pts in (("ect", c_pts), ("radon", c_pts + o_pts)):
        rep = plan.exact(dirs, kind)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        plan.exact(dirs, kind, reuse=rep)
        e0.record()
        for _ in range(steps):
            plan.exact(dirs, kind, reuse=rep)
        e1.record()
        torch.cuda.synchronize()
        ms_b = e0.elapsed_time(e1) / steps
        ln = rep.length.cpu().numpy()
        entries = float(ln.sum())
        nbytes = 8.0 * pts + 12.0 * entries
        o = torch.empty((rep.rows, thr.shape[0]), dtype=torch.int32, device=thr.device)
        rep.eval(thr, out=o)
        e0.record()
        for _ in range(steps):
            rep.eval(thr, out=o)
        e1.record()
        torch.cuda.synchronize()
        ms_e = e0.elapsed_time(e1) / steps
        out[f"{kind}_exact"] = {"build_ms": ms_b, "rows": rep.rows, "points": pts, "entries": entries,
                                "rows_per_s": rep.rows / (ms_b * 1e-3),
                                "roofline": roofline.hbm_roofline(nbytes, ms_b * 1e-3),
                                "eval_ms": ms_e, "eval_values_per_s": rep.rows * thr.shape[0] / (ms_e * 1e-3)}
    return out


def measure_4d(steps):
    """The four-axis workload (24^4 quantised field, primal): every stage of the
    step on it, kernel times from the library's stage events, the hybrid
    evaluation rate and the fused kernel's ALU roofline, and the exact (T, E)
    build of its 512 directions."""
    import numpy as np
    import torch

    from paper_2405_02256_amd import _native as N
    from paper_2405_02256_amd import api, hipevents, roofline
    from paper_2405_02256_amd import workloads as W

    dev = torch.device("cuda:0")
    w = W.hypervolume_24()
    img = w.images[0]
    plan = api.Plan(torch.from_numpy(img).to(dev))
    dirs = torch.from_numpy(w.ect_dirs).to(dev)
    thr = torch.from_numpy(w.ect_thresholds).to(dev)
    xi = torch.from_numpy(w.hybrid_xi).to(dev)
    kern = ("fourier", "laplace", "bessel")
    g = torch.from_numpy(np.random.default_rng(7).standard_normal((len(w.hybrid_xi), 2))).to(dev)
    eo = torch.empty((len(w.ect_dirs), thr.shape[0]), dtype=torch.int32, device=dev)
    outs = plan.hybrid_multi(xi, kern, 1.0, "fp32")
    gx = torch.empty((len(w.hybrid_xi), 4), dtype=torch.float64, device=dev)
    gs = torch.empty((), dtype=torch.float64, device=dev)

    def step():
        plan.rerun()
        plan.ect(dirs, thr, out=eo)
        plan.hybrid_multi(xi, kern, 1.0, "fp32", outs=outs)
        plan.hybrid_backward(xi, outs["fourier"], g, "fourier", 1.0, "fp32", grad_xi=gx, grad_s=gs)

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    names = ["precompute", "ect", "hybrid_fused", "hybrid_bwd_fourier"]
    evs = {nm: [(hipevents.Event(), hipevents.Event()) for _ in range(steps)] for nm in names}
    for i in range(steps):
        for stg, nm in enumerate(names):
            N.check(N.ect_set_stage_events(stg, evs[nm][i][0].handle, evs[nm][i][1].handle), "stage events")
        step()
    torch.cuda.synchronize()
    for stg in range(4):
        N.ect_set_stage_events(stg, None, None)
    ms = {nm: float(np.mean([a.elapsed_ms(b) for a, b in evs[nm]])) for nm in names}
    if plan.check() != 0:
        raise RuntimeError("device error flags set on the four-axis workload")
    cls_counts, ord_counts = plan.counts()
    e = sum(((w.hybrid_xi[:, a] < 0) * (1 << a) for a in range(4)))
    pair = np.where(e >= 8, e ^ 15, e)
    pairs = float(ord_counts[0][pair].sum())
    ed = sum(((w.ect_dirs[:, a] < 0) * (1 << a) for a in range(4)))
    ect_pairs = float(cls_counts[0][ed].sum())
    # share of Bessel (query, point) pairs on the small-argument branch, on 256 sampled xi
    rng = np.random.default_rng(11)
    sel = rng.choice(len(w.hybrid_xi), 256, replace=False)
    lists = [plan.export(0, 1, b)[0].astype(np.float64) - (np.array(img.shape[::-1]) / 2.0) for b in range(8)]
    small = tot = 0.0
    for q in sel:
        z = np.abs(lists[pair[q]] @ w.hybrid_xi[q])
        small += float((z < 8.0).sum())
        tot += float(z.size)
    small_frac = small / max(tot, 1.0)
    roof = roofline.alu_roofline("+".join(kern), 4, pairs, ms["hybrid_fused"] * 1e-3, small_frac)
    rep = plan.exact(dirs, "ect")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    plan.exact(dirs, "ect", reuse=rep)
    e0.record()
    for _ in range(steps):
        plan.exact(dirs, "ect", reuse=rep)
    e1.record()
    torch.cuda.synchronize()
    return {"workload": "hypervolume_24: 24^4 smoothed noise quantised into 8 levels, primal; ECT 512 dirs "
                        "(uniform on S^3) x 256 thresholds; Euler-Fourier/Laplace/Bessel at 4096 xi, "
                        "|xi|~U[0.01,1]; Fourier backward",
            "stage_kernel_ms": ms, "hybrid_pairs_per_kernel": pairs,
            "hybrid_evals_per_s": pairs * (len(kern) + 1) / (sum(ms.values()) * 1e-3),
            "ect_dirs_per_s": len(w.ect_dirs) / (ms["ect"] * 1e-3), "ect_pairs": ect_pairs,
            "bessel_small_branch_fraction": small_frac, "hybrid_fused_roofline": roof,
            "ect_roofline": roofline.alu_roofline("ect", 4, ect_pairs, ms["ect"] * 1e-3),
            "exact_ect_build_ms": e0.elapsed_time(e1) / steps}


STAGES = (("precompute", 0), ("ect", 1), ("hybrid", 2), ("hybrid_bwd", 3))


def stage_kernel_ms(run_once, reps):
    """Mean duration (ms) of each library stage's main kernel over `reps` eager
    calls of run_once (HIP events the library records on the call's stream);
    stages that run_once does not launch are absent."""
    import numpy as np
    import torch

    from paper_2405_02256_amd import _native as N
    from paper_2405_02256_amd import hipevents

    evs = {nm: [(hipevents.Event(), hipevents.Event()) for _ in range(reps)] for nm, _ in STAGES}
    torch.cuda.synchronize()
    for i in range(reps):
        for nm, stg in STAGES:
            N.check(N.ect_set_stage_events(stg, evs[nm][i][0].handle, evs[nm][i][1].handle), "stage events")
        run_once()
    torch.cuda.synchronize()
    for _, stg in STAGES:
        N.ect_set_stage_events(stg, None, None)
    out = {}
    for nm, _ in STAGES:
        try:
            out[nm] = float(np.mean([a.elapsed_ms(b) for a, b in evs[nm]]))
        except RuntimeError:
            pass   # never recorded: this call sequence does not launch the stage
    return out


def capture(fn, plans):
    """Record fn() into a HIP graph (after one eager call sized every workspace);
    the evaluation workspaces it recorded are kept alive with it."""
    import torch
    fn()
    torch.cuda.synchronize()
    keep = [dict(p._eval_ws) for p in plans]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    return g, keep


def time_steps(run, steps, warmup):
    """Seconds per call of run(), K calls bracketed by device synchronisations."""
    import torch
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def sign_index(v):
    import numpy as np
    v = np.asarray(v)
    return sum((v[..., a] < 0).astype(np.int64) << a for a in range(v.shape[-1]))


def pair_index(e, n):
    import numpy as np
    full = (1 << n) - 1
    return np.where(e >= (1 << (n - 1)), e ^ full, e)


def precompute_bytes(n, pixel_bytes, entries, num_images, nl):
    """Algorithmic bytes of the precompute: every pixel read once, each list
    entry written as packed vertex coordinates (uint16 per axis) and an int16
    value, and the list offsets."""
    return float(pixel_bytes) + (2.0 * n + 2.0) * float(entries) + 8.0 * (num_images + 1) * nl


def dominant(stage_ms, models):
    """(name, roofline) of the longest of the step's kernels; models maps a
    stage name to a function of its duration in seconds."""
    name = max((k for k in models if k in stage_ms), key=stage_ms.get)
    roof = models[name](stage_ms[name] * 1e-3)
    roof["kernel"] = name
    roof["kernel_ms"] = stage_ms[name]
    return name, roof


# kernels of each bench stage (a stage's launch = one launch of each)
TRAFFIC_STAGES = {
    "batch_4096": {"precompute": r"tile_count_2p_kernel|tile_block_\w+_kernel|tile_copy_kernel",
                   "ect": r"ect_batch_kernel<2>", "hybrid": r"hybrid_kernel<2, 2, 0, false>"},
    "grf_512": {"precompute": r"classify_compact<2, 0, unsigned char, true>",
                "ect_hybrid_fused": r"ect_hybrid_kernel<2, 7, 0>", "hybrid_bwd_fourier": r"hybrid_kernel<2, 1, 0, true>",
                "ect": r"ect_direct_kernel<2, false>", "hybrid_fused": r"hybrid_kernel<2, 7, 0, false>"},
}


def counter_means(path, counter):
    """Mean value per dispatch of one counter for every kernel of a rocprofv3 counter_collection.csv."""
    import csv
    import collections
    tot, disp = collections.defaultdict(float), collections.defaultdict(set)
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            k = r["Kernel_Name"]
            tot[k] += float(r["Counter_Value"])
            disp[k].add(r["Dispatch_Id"])
    return {k: tot[k] / len(disp[k]) for k in tot}


def write_traffic_json(workload, fetch_csv, write_csv, cfetch_csv, cwrite_csv):
    """HBM bytes per launch of each bench stage: FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each scaled by
    what it reads for a plain device copy of known size."""
    import re
    nbytes = 256 << 20
    cf, cw = counter_means(cfetch_csv, "FETCH_SIZE"), counter_means(cwrite_csv, "WRITE_SIZE")
    f_scale = nbytes / (1024.0 * max(cf.values()))
    w_scale = nbytes / (1024.0 * max(cw.values()))
    fetch, write = counter_means(fetch_csv, "FETCH_SIZE"), counter_means(write_csv, "WRITE_SIZE")
    out = {}
    for stage, rx in TRAFFIC_STAGES[workload].items():
        ks = [k for k in fetch if re.search(rx, k)]
        if ks:
            out[stage] = sum(1024.0 * (fetch[k] * f_scale + write.get(k, 0.0) * w_scale) for k in ks)
    csrc = os.path.join(ROOT, "paper_2405_02256_amd", "csrc")
    doc = {"source_digest": source_digest(sorted(os.path.join(csrc, f) for f in os.listdir(csrc))),
           "bytes_per_launch": out, "fetch_scale": f_scale, "write_scale": w_scale,
           "note": "FETCH_SIZE + WRITE_SIZE per launch, scaled by a plain 256 MiB device copy's readings"}
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
    print(path)


def traffic_for(workload, kernel):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    runs (FETCH_SIZE + WRITE_SIZE, copy-calibrated), if they were taken on the
    current kernel sources; else None."""
    csrc = os.path.join(ROOT, "paper_2405_02256_amd", "csrc")
    digest = source_digest(sorted(os.path.join(csrc, f) for f in os.listdir(csrc)))
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    try:
        tr = json.load(open(path))
    except (OSError, ValueError):
        return None
    if tr.get("source_digest") != digest:
        return None
    return tr.get("bytes_per_launch", {}).get(kernel)


def bench_batch(args, dev, tuning_out):
    """The headline: 4096 ragged images in one graph, and the per-image FP64 loop."""
    import numpy as np
    import torch

    from paper_2405_02256_amd import api, pipeline, roofline
    from paper_2405_02256_amd import workloads as W

    w = W.batch_4096(4)
    imgs = [torch.from_numpy(im).to(dev) for im in w.images]
    plan = api.Plan(imgs)
    dirs = torch.from_numpy(w.ect_dirs).to(dev)
    thr = torch.from_numpy(w.ect_thresholds).to(dev)
    xi = torch.from_numpy(w.hybrid_xi).to(dev)
    nq = len(w.hybrid_xi) // len(imgs)
    offs = torch.arange(len(imgs) + 1, dtype=torch.int64, device=dev) * nq
    # the ECT runs on a side stream beside the Laplace pass (its latency-bound
    # workgroups fill the compute units the ALU-bound pass leaves idle)
    step = pipeline.Step(plan, dirs, thr, xi, kernels=("laplace",), s=1.0, precision="fp32", hybrid_offsets=offs,
                         concurrent=not args.serial_ect)
    if not args.no_autotune:
        log("batch_4096: autotuning")
        t = step.autotune()
        tuning_out.update(hybrid_target_items=t.hybrid_target_items, ect_dirs_per_group=t.ect_dirs_per_group,
                          ect_chunks=t.ect_chunks)
    log("batch_4096: capture and timing")
    if args.no_graph:
        run = step.run
    else:
        step.capture()
        run = step.replay
    sec = time_steps(run, args.steps, args.warmup)
    if plan.check() != 0:
        raise RuntimeError("device error flags set on the batch")
    c, o = plan.counts()
    ex = w.hybrid_xi.reshape(len(imgs), nq, 2)
    pairs = float(np.take_along_axis(o, pair_index(sign_index(ex), 2), axis=1).sum())
    ect_pairs = float(c[:, sign_index(w.ect_dirs)].sum())
    stage_ms = stage_kernel_ms(step.run, args.steps)
    # one launch holding both (combined), or the ECT on its side stream inside
    # the Laplace launch's window (concurrent): the window's work is both
    combined = "ect" not in stage_ms or (step.concurrent and stage_ms["ect"] <= stage_ms["hybrid"])
    nbytes = precompute_bytes(2, sum(im.size for im in w.images), c.sum() + o.sum(), len(imgs), 6)
    models = {"precompute": lambda s: roofline.hbm_roofline(nbytes, s),
              "ect": lambda s: roofline.alu_roofline("ect", 2, ect_pairs, s),
              "hybrid": (lambda s: roofline.alu_roofline_parts([("ect", 2, ect_pairs, 1.0),
                                                                 ("laplace", 2, pairs, 1.0)], s)) if combined
              else (lambda s: roofline.alu_roofline("laplace", 2, pairs, s))}
    dom, roof = dominant(stage_ms, models)
    roof["traffic"] = traffic_for("batch_4096", dom)
    if combined and dom == "hybrid" and "ect" in stage_ms:
        roof["window"] = "Laplace launch, batched ECT on a side stream inside it; work of both"
        te = traffic_for("batch_4096", "ect")
        roof["traffic"] = roof["traffic"] + te if roof["traffic"] is not None and te is not None else None
    rows_all = {k: models[k](stage_ms[k] * 1e-3) for k in models if k in stage_ms}
    log(f"batch_4096: {sec * 1e3:.4f} ms/step, stages {stage_ms}")

    sides = np.array(w.meta["sides"])
    rng = np.random.default_rng(44)
    sample = np.sort(np.concatenate([rng.choice(np.nonzero(sides == s)[0], 24, replace=False)
                                     for s in (28, 64, 128, 256)]))
    ect_all = step.ect_out.reshape(len(imgs), len(w.ect_dirs), -1)
    y_all = step.hy_out["laplace"].reshape(len(imgs), nq)
    gpu = {"sample": sample, "ect": ect_all[torch.from_numpy(sample).to(dev)].cpu().numpy(),
           "laplace": y_all[torch.from_numpy(sample).to(dev)].cpu().numpy()}

    fp64 = None
    if not args.no_fp64:
        log("batch_4096: per-image FP64 loop")
        plans = [api.Plan(im) for im in imgs]
        outs_e = [torch.empty((len(w.ect_dirs), thr.shape[1]), dtype=torch.int32, device=dev) for _ in plans]
        outs_h = [torch.empty(nq, dtype=torch.float64, device=dev) for _ in plans]
        xis = [xi[i * nq:(i + 1) * nq] for i in range(len(plans))]

        def per_image():
            for i, pl in enumerate(plans):
                pl.rerun()
                pl.ect(dirs, thr[i], out=outs_e[i])
                pl.hybrid(xis[i], "laplace", 1.0, "fp64", out=outs_h[i])

        per_image()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        per_image()
        torch.cuda.synchronize()
        t_loop = time.perf_counter() - t0
        y64 = torch.cat(outs_h).cpu().numpy()
        e64 = torch.cat(outs_e).cpu().numpy()
        y32 = step.hy_out["laplace"].cpu().numpy()
        fp64 = {"per_image_fp64_loop_ms": t_loop * 1e3, "speedup": t_loop / sec,
                "ect_identical": bool(np.array_equal(step.ect_out.cpu().numpy(), e64)),
                "fp32_vs_fp64_normwise": float(np.abs(y32 - y64).max() / np.abs(y64).max())}
        gpu["laplace_fp64"] = y64.reshape(len(imgs), nq)[sample]
        del plans, outs_e, outs_h
    row = {"workload": "batch_4096: 4096 binary GRF images, sides U{28,64,128,256}, sigma U[2,8] px, median "
                       "threshold, primal; ECT 128 dirs x 128 per-image thresholds; Euler-Laplace at 512 xi "
                       "per image, |xi|~U[0.01,1]; one HIP graph",
           "ms_per_step": sec * 1e3, "hybrid_pairs": pairs, "ect_pairs": ect_pairs,
           "hybrid_evals_per_s": pairs / sec, "ect_dirs_per_s": len(imgs) * len(w.ect_dirs) / sec,
           "stage_kernel_ms": stage_ms,
           "stage_note": ("the ECT runs on a side stream while the hybrid (Laplace) launch runs; the two stage "
                          "times overlap" if step.concurrent else
                          "the ECT workgroups run inside the hybrid launch" if combined else None),
           "rooflines": rows_all, "precompute_vertices": float(sum((im.shape[0] + 1) * (im.shape[1] + 1)
                                                                   for im in w.images)),
           "precompute_list_entries": float(c.sum() + o.sum()), "batched_vs_per_image": fp64}
    return row, roof, w, gpu


def bench_grf(args, dev, tuning_out):
    """grf_512: the single-field step (combined ECT + fused hybrid launch, Fourier backward)."""
    import numpy as np
    import torch

    from paper_2405_02256_amd import api, pipeline, roofline
    from paper_2405_02256_amd import workloads as W

    w = W.grf_512(2)
    img = w.images[0]
    gout = np.random.default_rng(12).standard_normal((len(w.hybrid_xi), 2))
    dirs = torch.from_numpy(w.ect_dirs).to(dev)
    thr = torch.from_numpy(w.ect_thresholds).to(dev)
    xi = torch.from_numpy(w.hybrid_xi).to(dev)
    plan = api.Plan(torch.from_numpy(img).to(dev))
    step = pipeline.Step(plan, dirs, thr, xi, kernels=KERNELS, s=1.0, precision="fp32",
                         backward_kernel="fourier", grad_out=torch.from_numpy(gout).to(dev))
    c, o = plan.counts()
    lists = [plan.export(0, 1, b)[0] for b in range(2)]
    pr = pair_index(sign_index(w.hybrid_xi), 2)
    pairs = float(o[0][pr].sum())
    ect_pairs = float(c[0][sign_index(w.ect_dirs)].sum())
    small = 0.0
    for b in range(2):
        z = np.abs(w.hybrid_xi[pr == b] @ (lists[b].astype(np.float64) - 256.0).T)
        small += float((z < 8.0).sum())
    small_frac = small / max(pairs, 1.0)
    if not args.no_autotune:
        log("grf_512: autotuning")
        t = step.autotune()
        tuning_out.update(hybrid_target_items=t.hybrid_target_items, ect_dirs_per_group=t.ect_dirs_per_group,
                          ect_chunks=t.ect_chunks)
    if args.no_graph:
        run = step.run
    else:
        step.capture()
        run = step.replay
    sec = time_steps(run, args.steps, args.warmup)
    if plan.check() != 0:
        raise RuntimeError("device error flags set on grf_512")
    st = stage_kernel_ms(step.run, args.steps)
    stage_ms = {"precompute": st["precompute"], "ect_hybrid_fused": st["hybrid"],
                "hybrid_bwd_fourier": st["hybrid_bwd"]}
    ref = stage_kernel_ms(lambda: (plan.ect(step.ect_q, step.ect_thr, out=step.ect_out),
                                   plan.hybrid_multi(step.hy_q, KERNELS, 1.0, "fp32", outs=step.hy_out)),
                          args.steps)
    stage_ms["ect"] = ref["ect"]
    stage_ms["hybrid_fused"] = ref["hybrid"]
    # the graph's last replay left the step's outputs; recompute them once eagerly for the oracle leg
    step.run()
    torch.cuda.synchronize()
    gpu = {"ect": step.ect_out.cpu().numpy(), "grad_xi": step.grad_xi.cpu().numpy(),
           "grad_s": float(step.grad_s.cpu()), "gout": gout}
    for k in KERNELS:
        gpu[k] = step.hy_out[k].cpu().numpy()
    nbytes = precompute_bytes(2, img.size, c.sum() + o.sum(), 1, 6) + 40.0 * len(w.hybrid_xi)
    models = {"precompute": lambda s: roofline.hbm_roofline(nbytes, s),
              "ect_hybrid_fused": lambda s: roofline.alu_roofline_parts(
                  [("ect", 2, ect_pairs, 1.0), ("+".join(KERNELS), 2, pairs, small_frac)], s),
              "hybrid_bwd_fourier": lambda s: roofline.alu_roofline("fourier_bwd", 2, pairs, s)}
    dom, roof = dominant(stage_ms, models)
    roof["traffic"] = traffic_for("grf_512", dom)
    fp64_ms = None
    if not args.no_fp64:
        step64 = pipeline.Step(plan, dirs, thr, xi, kernels=KERNELS, s=1.0, precision="fp64",
                               backward_kernel="fourier", grad_out=torch.from_numpy(gout).to(dev))
        fp64_ms = time_steps(step64.run, max(3, args.steps // 5), 1) * 1e3
    log(f"grf_512: {sec * 1e3:.4f} ms/step, stages {stage_ms}")
    row = {"workload": "grf_512: 512x512 binary Gaussian random field (sigma 8 px, median threshold), primal; "
                       "ECT 360 dirs x 256 thresholds; Euler-Fourier/Laplace/Bessel at 4096 xi, |xi|~U[0.01,1]; "
                       "Fourier backward; one HIP graph",
           "ms_per_step": sec * 1e3, "hybrid_evals_per_s": pairs * (len(KERNELS) + 1) / sec,
           "ect_dirs_per_s": len(w.ect_dirs) / sec, "stage_kernel_ms": stage_ms,
           "stage_note": "the step launches precompute (which also buckets the shared query set), "
                         "ect_hybrid_fused (the ECT inside the fused hybrid pass) and hybrid_bwd_fourier; ect and "
                         "hybrid_fused are the two passes launched separately, for reference",
           "bessel_small_branch_fraction": small_frac, "roofline": roof,
           "fp64_path_ms_per_step": fp64_ms, "fp32_vs_fp64_speedup": None if fp64_ms is None
           else fp64_ms / (sec * 1e3)}
    return row, w, gpu, plan, (dirs, thr, c, o)


def bench_volume(args, dev):
    """volume_128: ECT at 2048 directions and Fourier + Laplace (log-scale) at 16384 xi."""
    import numpy as np
    import torch

    from paper_2405_02256_amd import api, pipeline, roofline
    from paper_2405_02256_amd import workloads as W

    w = W.volume_128(3)
    vol = w.images[0]
    plan = api.Plan(torch.from_numpy(vol).to(dev), origin=np.zeros(3))
    dirs = torch.from_numpy(w.ect_dirs).to(dev)
    thr = torch.from_numpy(w.ect_thresholds).to(dev)
    xi = torch.from_numpy(w.hybrid_xi).to(dev)
    ker = ("fourier", "laplace")
    step = pipeline.Step(plan, dirs, thr, xi, kernels=ker, s=1.0, precision="fp32", log_scale_laplace=True)
    if not args.no_autotune:
        log("volume_128: autotuning")
        step.autotune()
    if args.no_graph:
        run = step.run
    else:
        step.capture()
        run = step.replay
    sec = time_steps(run, max(5, args.steps // 5), 2)
    flags = plan.check()
    if flags != 0:
        raise RuntimeError(f"device error flags {flags:#x} set on volume_128")
    c, o = plan.counts()
    pairs = float(o[0][pair_index(sign_index(w.hybrid_xi), 3)].sum())
    ect_pairs = float(c[0][sign_index(w.ect_dirs)].sum())
    stage_ms = stage_kernel_ms(step.run, max(5, args.steps // 5))
    combined = "ect" not in stage_ms
    step.run()
    torch.cuda.synchronize()
    gpu = {"ect": step.ect_out.cpu().numpy(), "fourier": step.hy_out["fourier"].cpu().numpy(),
           "laplace": step.hy_out["laplace"].cpu().numpy(), "log_scale": step.hy_ls["laplace"].cpu().numpy()}
    nbytes = precompute_bytes(3, vol.size, c.sum() + o.sum(), 1, 12)
    models = {"precompute": lambda s: roofline.hbm_roofline(nbytes, s),
              "ect": lambda s: roofline.alu_roofline("ect", 3, ect_pairs, s),
              "hybrid": (lambda s: roofline.alu_roofline_parts([("ect", 3, ect_pairs, 1.0),
                                                                 ("fourier+laplace", 3, pairs, 1.0)], s))
              if combined else (lambda s: roofline.alu_roofline("fourier+laplace", 3, pairs, s))}
    dom, roof = dominant(stage_ms, models)
    roof["traffic"] = traffic_for("volume_128", dom)
    log(f"volume_128: {sec * 1e3:.4f} ms/step, stages {stage_ms}")
    row = {"workload": "volume_128: 128^3 smoothed noise quantised into 8 levels, primal, corner origin; ECT 2048 "
                       "Fibonacci dirs x 256 thresholds; Euler-Fourier and Euler-Laplace (log-scale output) at "
                       "16384 xi, |xi|~U[0.01,4]; one HIP graph",
           "ms_per_step": sec * 1e3, "hybrid_evals_per_s": 2 * pairs / sec, "ect_dirs_per_s": len(w.ect_dirs) / sec,
           "hybrid_pairs_per_kernel": pairs, "ect_pairs": ect_pairs, "stage_kernel_ms": stage_ms,
           "stage_note": ("the ECT workgroups run inside the hybrid launch" if combined else None),
           "precompute_roofline": models["precompute"](stage_ms["precompute"] * 1e-3), "roofline": roof}
    return row, w, gpu


def bench_diff(args, dev):
    """diff_256: a training step at 1024 shared xi: fused Fourier + Laplace forward, both backward passes."""
    import numpy as np
    import torch

    from paper_2405_02256_amd import api, roofline
    from paper_2405_02256_amd import autotune as AT
    from paper_2405_02256_amd import workloads as W

    w = W.diff_256(5)
    imgs = [torch.from_numpy(im).to(dev) for im in w.images]
    plan = api.Plan(imgs)
    q = api.QuerySet(torch.from_numpy(w.hybrid_xi).to(dev))
    q.validate(plan.num_images, 2)
    ker = ("fourier", "laplace")
    wts = w.meta["loss_weights"]
    gF = torch.from_numpy(wts.reshape(-1, 2)).to(dev).contiguous()
    gL = torch.from_numpy(np.ascontiguousarray(wts[..., 0]).reshape(-1)).to(dev)
    if not args.no_autotune:
        log("diff_256: autotuning")
        AT.tune(plan, None, None, q, ker, 1.0, "fp32", backward_kernel="fourier", grad_out=gF)
    outs = plan.hybrid_multi(q, ker, 1.0, "fp32")
    nq = len(w.hybrid_xi)
    bufs = {k: (torch.empty((nq, 2), dtype=torch.float64, device=dev), torch.empty((), dtype=torch.float64,
                                                                                   device=dev)) for k in ker}
    gx = torch.empty((nq, 2), dtype=torch.float64, device=dev)
    gs = torch.empty((), dtype=torch.float64, device=dev)

    def step():
        plan.rerun()
        plan.hybrid_multi(q, ker, 1.0, "fp32", outs=outs)
        plan.hybrid_backward(q, outs["fourier"], gF, "fourier", 1.0, "fp32", grad_xi=bufs["fourier"][0],
                             grad_s=bufs["fourier"][1], reuse_prepared=True)
        plan.hybrid_backward(q, outs["laplace"], gL, "laplace", 1.0, "fp32", grad_xi=bufs["laplace"][0],
                             grad_s=bufs["laplace"][1], reuse_prepared=True)
        torch.add(bufs["fourier"][0], bufs["laplace"][0], out=gx)
        torch.add(bufs["fourier"][1], bufs["laplace"][1], out=gs)

    if args.no_graph:
        run = step
    else:
        g, keep = capture(step, [plan])
        run = g.replay
    sec = time_steps(run, args.steps, args.warmup)
    if plan.check() != 0:
        raise RuntimeError("device error flags set on diff_256")
    c, o = plan.counts()
    pairs = float(o[:, pair_index(sign_index(w.hybrid_xi), 2)].sum())
    stage_ms = stage_kernel_ms(step, args.steps)
    step()
    torch.cuda.synchronize()
    gpu = {"fourier": outs["fourier"].cpu().numpy(), "laplace": outs["laplace"].cpu().numpy(),
           "grad_xi": gx.cpu().numpy(), "grad_s": float(gs.cpu())}
    models = {"hybrid": lambda s: roofline.alu_roofline("fourier+laplace", 2, pairs, s),
              "hybrid_bwd": lambda s: roofline.alu_roofline("laplace_bwd", 2, pairs, s),
              "precompute": lambda s: roofline.hbm_roofline(
                  precompute_bytes(2, sum(im.size for im in w.images), c.sum() + o.sum(), len(imgs), 6), s)}
    dom, roof = dominant(stage_ms, models)
    log(f"diff_256: {sec * 1e3:.4f} ms/step, stages {stage_ms}")
    row = {"workload": "diff_256: 256 binary GRF images 128x128 (sigma U[2,8] px); Euler-Fourier and Euler-Laplace "
                       "at 1024 shared xi (|xi|~U[0.01,0.5], >= 0.02 rad from the axes), s = 1; forward and both "
                       "backward passes of the seeded loss sum(W * outputs); one HIP graph",
           "ms_per_step": sec * 1e3, "hybrid_evals_per_s": 4 * pairs / sec, "hybrid_pairs_per_kernel": pairs,
           "stage_kernel_ms": stage_ms, "stage_note": "hybrid_bwd is the Laplace backward (the last one launched)",
           "roofline": roof}
    return row, w, gpu


def bench_small(args, dev):
    """small_binary: the 64x64 image, FP64, ECT 64 x 64 and Fourier at 256 xi (latency)."""
    import torch

    from paper_2405_02256_amd import api, pipeline
    from paper_2405_02256_amd import workloads as W

    w = W.small_binary(1)
    plan = api.Plan(torch.from_numpy(w.images[0]).to(dev))
    step = pipeline.Step(plan, torch.from_numpy(w.ect_dirs).to(dev), torch.from_numpy(w.ect_thresholds).to(dev),
                         torch.from_numpy(w.hybrid_xi).to(dev), kernels=("fourier",), s=1.0, precision="fp64")
    if args.no_graph:
        run = step.run
    else:
        step.capture()
        run = step.replay
    sec = time_steps(run, args.steps, args.warmup)
    stage_ms = stage_kernel_ms(step.run, args.steps)
    step.run()
    torch.cuda.synchronize()
    gpu = {"ect": step.ect_out.cpu().numpy(), "fourier": step.hy_out["fourier"].cpu().numpy()}
    row = {"workload": "small_binary: 64x64 Bernoulli(0.5) image after a 3x3 majority filter, primal; ECT 64 dirs x "
                       "64 thresholds; Euler-Fourier at 256 xi; FP64; one HIP graph",
           "latency_us": sec * 1e6, "stage_kernel_ms": stage_ms}
    return row, w, gpu


def oracle_leg(rows, batch, grf, vol, diff, small):
    """cpu_baseline: the FP64 oracle on bounded samples of every workload, timed
    on the host cores; every row gets its error against it.  Returns the
    cpu_baseline object of the headline (the batch)."""
    import numpy as np

    from oracle import gates as G
    from oracle import oracle as O

    cores = O.max_threads()
    timing = {}

    def timed(key, fn):
        t0 = time.perf_counter()
        r = fn()
        timing[key] = timing.get(key, 0.0) + time.perf_counter() - t0
        return r

    # ---- headline: 24 images of each side, every direction and every xi of each ----
    w, gpu = batch
    sides = np.array(w.meta["sides"])
    nq = len(w.hybrid_xi) // len(w.images)
    ect_ok = True
    ys, refs, S2s, S1s, y64s = [], [], [], [], []
    t_side = {}
    for k, i in enumerate(gpu["sample"]):
        img = w.images[i]
        t0 = time.perf_counter()
        e = O.ect(img, w.ect_dirs, w.ect_thresholds[i])
        ref = O.hybrid(img, w.hybrid_xi[i * nq:(i + 1) * nq], "laplace", 1.0)
        t_side[int(sides[i])] = t_side.get(int(sides[i]), 0.0) + time.perf_counter() - t0
        ect_ok &= bool(np.array_equal(e, gpu["ect"][k]))
        S1, S2 = G.term_scales(img, w.hybrid_xi[i * nq:(i + 1) * nq], "laplace", 1.0)
        ys.append(gpu["laplace"][k]); refs.append(ref); S2s.append(S2); S1s.append(S1)
        if "laplace_fp64" in gpu:
            y64s.append(gpu["laplace_fp64"][k])
    counts = {s: int((sides == s).sum()) for s in t_side}
    per = {s: int((sides[gpu["sample"]] == s).sum()) for s in t_side}
    t_full = sum(t_side[s] * counts[s] / per[s] for s in t_side)
    err = {"ect_bit_exact": ect_ok, "ect_rows_checked": int(len(gpu["sample"]) * len(w.ect_dirs)),
           "laplace_fp32": G.g9_stats(np.concatenate(ys), np.concatenate(refs), np.concatenate(S2s),
                                      np.concatenate(S1s))}
    if y64s:
        err["laplace_fp64_loop"] = G.g9_stats(np.concatenate(y64s), np.concatenate(refs), np.concatenate(S2s),
                                              np.concatenate(S1s))
    err["sample"] = (f"{len(gpu['sample'])} images (24 of each side), all 128 directions and all 512 xi of each")
    rows["batch"]["error_vs_oracle"] = err
    # one core, 4 images of each side
    O.set_threads(1)
    t1_side = {}
    for s in sorted(t_side):
        ids = [i for i in gpu["sample"] if sides[i] == s][:4]
        t0 = time.perf_counter()
        for i in ids:
            O.ect(w.images[i], w.ect_dirs, w.ect_thresholds[i])
            O.hybrid(w.images[i], w.hybrid_xi[i * nq:(i + 1) * nq], "laplace", 1.0)
        t1_side[s] = (time.perf_counter() - t0) / len(ids)
    O.set_threads(cores)
    t1_full = sum(t1_side[s] * counts[s] for s in t1_side)
    pairs = rows["batch"]["hybrid_pairs"]
    cpu = {"value": pairs / t_full, "unit": "ξ·crit-pt evals/s", "cores": cores, "kind": "oracle",
           "sample": (f"FP64 oracle (ECT over every cell at 128 directions x 128 thresholds, Euler-Laplace cell "
                      f"form at 512 xi) on {len(gpu['sample'])} of the 4096 images, 24 of each side, "
                      f"{sum(t_side.values()):.1f} s on {cores} OpenMP threads, scaled by the count of each side "
                      f"to the whole batch ({t_full:.1f} s per step)"),
           "value_1core": pairs / t1_full, "sample_1core": (f"4 images of each side on 1 thread, "
                                                           f"{sum(4 * v for v in t1_side.values()):.1f} s, scaled "
                                                           f"to the whole batch ({t1_full:.1f} s per step)"),
           "step_s_all_cores": t_full, "step_s_1core": t1_full}

    # ---- grf_512: every ECT row, every Fourier/Laplace xi, 1024 Bessel xi, 1024 gradients ----
    if grf is not None:
        w, gpu = grf
        img = w.images[0]
        e = timed("grf_512", lambda: O.ect(img, w.ect_dirs, w.ect_thresholds))
        er = {"ect_bit_exact": bool(np.array_equal(e, gpu["ect"])), "ect_rows_checked": len(w.ect_dirs)}
        sel_b = np.arange(0, len(w.hybrid_xi), 4)
        for k in KERNELS:
            sel = sel_b if k == "bessel" else np.arange(len(w.hybrid_xi))
            xs = w.hybrid_xi[sel]
            y = gpu[k][sel]
            if k == "fourier":
                ref = timed("grf_512", lambda: O.hybrid(img, xs, k, 1.0))
                S1, S2 = G.term_scales(img, xs, k, 1.0)
                y = y[:, 0] + 1j * y[:, 1]
            elif k == "laplace":
                ref, m = timed("grf_512", lambda: O.hybrid(img, xs, k, 1.0, with_shift=True))
                S1, S2 = G.term_scales(img, xs, k, 1.0, shift=m)
                y = y * np.exp(-m)
            else:
                ref = timed("grf_512", lambda: O.hybrid(img, xs, k, 1.0))
                S1, S2 = G.term_scales(img, xs, k, 1.0)
            er[k] = G.g9_stats(y, ref, S2, S1)
        sel = np.arange(0, len(w.hybrid_xi), 4)
        gx, gs = timed("grf_512", lambda: O.hybrid_grad(img, w.hybrid_xi[sel], "fourier", 1.0, gpu["gout"][sel]))
        S2x, _, _, _ = G.grad_scales(img, w.hybrid_xi[sel], "fourier", 1.0, gpu["gout"][sel])
        er["grad_xi_fourier"] = G.g9_stats(gpu["grad_xi"][sel], gx, S2x)
        er["sample"] = ("all 360 ECT rows, all 4096 xi of Fourier and Laplace (Laplace in the oracle's shifted "
                        "form), 1024 xi of Bessel, grad_xi at 1024 xi (per component)")
        rows["grf_512"]["error_vs_oracle"] = er

    # ---- volume_128: 32 directions, 128 xi of each kernel ----
    if vol is not None:
        w, gpu = vol
        v = w.images[0]
        org = np.zeros(3)
        sd = np.linspace(0, len(w.ect_dirs) - 1, 32).astype(int)
        e = timed("volume_128", lambda: O.ect(v, w.ect_dirs[sd], w.ect_thresholds, origin=org))
        er = {"ect_bit_exact": bool(np.array_equal(e, gpu["ect"][sd])), "ect_rows_checked": len(sd)}
        sq = np.linspace(0, len(w.hybrid_xi) - 1, 128).astype(int)
        xs = w.hybrid_xi[sq]
        ref = timed("volume_128", lambda: O.hybrid(v, xs, "fourier", 1.0, origin=org))
        S1, S2 = G.term_scales(v, xs, "fourier", 1.0, origin=org)
        y = gpu["fourier"][sq]
        er["fourier"] = G.g9_stats(y[:, 0] + 1j * y[:, 1], ref, S2, S1)
        ref, m = timed("volume_128", lambda: O.hybrid(v, xs, "laplace", 1.0, origin=org, with_shift=True))
        S1, S2 = G.term_scales(v, xs, "laplace", 1.0, origin=org, shift=m)
        er["laplace_log_scale"] = G.g9_stats(gpu["laplace"][sq] * np.exp(gpu["log_scale"][sq] - m), ref, S2, S1)
        er["max_log_scale"] = float(gpu["log_scale"].max())
        er["sample"] = "32 of the 2048 ECT directions, 128 of the 16384 xi (Laplace in the oracle's shifted form)"
        rows["volume_128"]["error_vs_oracle"] = er

    # ---- diff_256: forward at 4 images x 64 xi, grad_xi of 8 xi summed over all 256 images ----
    if diff is not None:
        w, gpu = diff
        nq = len(w.hybrid_xi)
        wts = w.meta["loss_weights"]
        rng = np.random.default_rng(56)
        er = {}
        for k in ("fourier", "laplace"):
            ys, refs, S2s, S1s = [], [], [], []
            for i in rng.choice(len(w.images), 4, replace=False):
                qs = rng.choice(nq, 64, replace=False)
                ref = timed("diff_256", lambda: O.hybrid(w.images[i], w.hybrid_xi[qs], k, 1.0))
                S1, S2 = G.term_scales(w.images[i], w.hybrid_xi[qs], k, 1.0)
                y = gpu[k].reshape(len(w.images), nq, -1)[i, qs]
                ys.append(y[:, 0] + 1j * y[:, 1] if k == "fourier" else y[:, 0])
                refs.append(ref); S2s.append(S2); S1s.append(S1)
            er[k] = G.g9_stats(np.concatenate(ys), np.concatenate(refs), np.concatenate(S2s), np.concatenate(S1s))
        qs = rng.choice(nq, 8, replace=False)
        ref = np.zeros((8, 2))
        S2x = []
        for i, im in enumerate(w.images):
            for k, g in (("fourier", wts[i, qs]), ("laplace", wts[i, qs, 0])):
                a, _ = timed("diff_256", lambda: O.hybrid_grad(im, w.hybrid_xi[qs], k, 1.0, g))
                ref += a
                S2x.append(G.grad_scales(im, w.hybrid_xi[qs], k, 1.0, g)[0])
        er["grad_xi_fourier_plus_laplace"] = G.g9_stats(gpu["grad_xi"][qs], ref, G.combine_rss(*S2x))
        er["sample"] = ("forward at 4 images x 64 xi per kernel; grad_xi of the loss at 8 xi, summed over all 256 "
                        "images and both kernels (per component)")
        rows["diff_256"]["error_vs_oracle"] = er

    # ---- small_binary: everything ----
    if small is not None:
        w, gpu = small
        img = w.images[0]
        e = timed("small_binary", lambda: O.ect(img, w.ect_dirs, w.ect_thresholds))
        ref = timed("small_binary", lambda: O.hybrid(img, w.hybrid_xi, "fourier", 1.0))
        S1, _ = G.term_scales(img, w.hybrid_xi, "fourier", 1.0)
        y = gpu["fourier"]
        ok, ratio = G.fp64_gate(y[:, 0] + 1j * y[:, 1], ref, S1)
        rows["small_binary"]["error_vs_oracle"] = {
            "ect_bit_exact": bool(np.array_equal(e, gpu["ect"])), "ect_rows_checked": len(w.ect_dirs),
            "fourier_fp64": {"checked": len(ref), "max_ratio_to_1e-11_S1": ratio, "pass": bool(ok),
                             "normwise": float(np.abs(y[:, 0] + 1j * y[:, 1] - ref).max() / np.abs(ref).max())}}
    cpu["oracle_check_s"] = timing
    return cpu


def main():
    args = parse()
    if args.traffic_json:
        write_traffic_json(*args.traffic_json)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        nbytes = 256 << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 5}), flush=True)
        return

    rows = {}
    tuning = {}
    batch_row, roof, w4, gpu4 = bench_batch(args, dev, tuning)
    rows["batch"] = batch_row
    grf = vol = diff = small = None
    sel = set(r.strip() for r in args.rows.split(",") if r.strip())
    if not args.only_headline:
        if "grf" in sel:
            tg = {}
            rows["grf_512"], wg, gpug, plan_g, (dirs_g, thr_g, cg, og) = bench_grf(args, dev, tg)
            rows["grf_512"]["tuning"] = tg
            grf = (wg, gpug)
            if not args.no_next:
                log("Radon transform and exact representations (grf_512)")
                rows["grf_512"]["radon_and_exact"] = measure_next(plan_g, wg, dirs_g, thr_g, 2, cg, og[0],
                                                                  args.steps)
            del plan_g
        if "volume" in sel:
            log("volume_128")
            rows["volume_128"], wv, gpuv = bench_volume(args, dev)
            vol = (wv, gpuv)
        if "diff" in sel:
            log("diff_256")
            rows["diff_256"], wd, gpud = bench_diff(args, dev)
            diff = (wd, gpud)
        if "small" in sel:
            log("small_binary")
            rows["small_binary"], ws, gpus = bench_small(args, dev)
            small = (ws, gpus)
        if not args.no_4d:
            log("four-axis workload")
            rows["four_axes"] = measure_4d(args.steps)
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log("oracle leg: timing on the host cores and every row's error against the oracle")
        cpu = oracle_leg(rows, (w4, gpu4), grf, vol, diff, small)

    b = rows.pop("batch")
    res = {
        "metric": METRIC,
        "value": b["hybrid_evals_per_s"],
        "unit": "ξ·crit-pt evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": b["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": b["workload"], "graph": not args.no_graph,
                   "ect_stream": "serial" if args.serial_ect else "side stream beside the Laplace pass",
                   "precision": "FP32 kernel values, FP64 phases and accumulation", "tuning": tuning},
        "ect_dirs_per_s": b["ect_dirs_per_s"],
        "batched_vs_per_image": b["batched_vs_per_image"],
        "stage_kernel_ms": b["stage_kernel_ms"],
        "stage_note": b["stage_note"],
        "roofline": roof,
        "rooflines_per_stage": b["rooflines"],
        "precompute_vertices": b["precompute_vertices"],
        "precompute_list_entries": b["precompute_list_entries"],
        "error_vs_oracle": b.get("error_vs_oracle"),
        "rows": rows,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
