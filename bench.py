#!/usr/bin/env python3
"""Throughput of the whole hot path on one MI355X.

Workload (synthetic, seeded): one 512x512 binary image, a Gaussian random field
(sigma 8 px) thresholded at its median; ECT at 360 directions x 256 thresholds;
Euler-Fourier, Euler-Laplace and Euler-Bessel transforms at 4096 vectors xi
with |xi| ~ U[0.01, 1] and uniform angle; one Euler-Fourier backward pass.

One step = one pass of every stage on that batch: per-vertex classification
and ordered compaction, sign-vector bucketing, the exact ECT, the three
hybrid transforms (one fused pass over the (xi, point) pairs; FP32 kernel
values, FP64 phases and accumulation) and the backward pass, replayed as one
HIP graph.  value = (query, critical point)
hybrid evaluations (three forward kernels + the backward) per second of step
time.  Inputs are resident in HBM before the timed region.

Roofline: the dominant kernel's average duration comes from HIP events that
the library records around that kernel alone (ect_set_stage_events), over K
profiled eager steps that follow the timed graph replays.  The CPU baseline
times the FP64 oracle on a bounded sample of the same step on the host cores.
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
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-path comparison")
    ap.add_argument("--cpu-budget", type=float, default=10.0, help="scale of the oracle sample")
    ap.add_argument("--no-batch", action="store_true", help="skip the 4096-image batched comparison")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the Radon transform and exact-representation measurements")
    ap.add_argument("--no-4d", action="store_true", help="skip the four-axis workload")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default schedule knobs")
    ap.add_argument("--concurrent", action="store_true", help="run the ECT branch on a side stream")
    ap.add_argument("--separate-ect", action="store_true",
                    help="launch the ECT before the hybrid pass instead of inside its launch")
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
        nbytes = 32.0 * pts + 12.0 * entries
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


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2405_02256_amd import _native as N
    from paper_2405_02256_amd import api, hipevents, pipeline, roofline
    from paper_2405_02256_amd import workloads as W

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

    w = W.grf_512(2)
    img = w.images[0]
    rng = np.random.default_rng(12)
    gout = rng.standard_normal((len(w.hybrid_xi), 2))
    img_t = torch.from_numpy(img).to(dev)
    dirs = torch.from_numpy(w.ect_dirs).to(dev)
    thr = torch.from_numpy(w.ect_thresholds).to(dev)
    xi = torch.from_numpy(w.hybrid_xi).to(dev)
    g_t = torch.from_numpy(gout).to(dev)
    log("building plan")
    plan = api.Plan(img_t)
    step = pipeline.Step(plan, dirs, thr, xi, kernels=KERNELS, s=1.0, precision="fp32",
                         backward_kernel="fourier", grad_out=g_t, fused=True, concurrent=args.concurrent,
                         combined=not args.separate_ect)

    # work per step: sum over xi of the ordinary list length of its orthant pair
    n = 2
    lists = [plan.export(0, 1, b)[0] for b in range(2)]
    counts = np.array([len(L) for L in lists])
    e = ((w.hybrid_xi[:, 0] < 0) * 1 + (w.hybrid_xi[:, 1] < 0) * 2)
    pair = np.where(e >= 2, e ^ 3, e)
    per_kernel_pairs = float(counts[pair].sum())
    evals_per_step = per_kernel_pairs * (len(KERNELS) + 1)
    cls_counts, _ = plan.counts()
    ect_pairs = float(sum(cls_counts[0][((d[0] < 0) * 1 + (d[1] < 0) * 2)] for d in w.ect_dirs))
    # fraction of Bessel pairs on the small-argument branch
    x_of = [(L.astype(np.float64) - 256.0) for L in lists]
    small = 0.0
    for b in range(2):
        sel = w.hybrid_xi[pair == b]
        if len(sel):
            z = np.abs(sel @ x_of[b].T)
            small += float((z < 8.0).sum())
    small_frac = small / max(per_kernel_pairs, 1.0)

    tuning = None
    if not args.no_autotune:
        log("autotuning schedule knobs")
        t = step.autotune()
        tuning = {"hybrid_target_items": t.hybrid_target_items, "ect_dirs_per_group": t.ect_dirs_per_group,
                  "ect_chunks": t.ect_chunks}
        log(f"tuning {tuning}")
    log("warm-up and graph capture")
    step.run()
    torch.cuda.synchronize()
    use_graph = not args.no_graph
    if use_graph:
        step.capture()
        run = step.replay
    else:
        run = step.run
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    if plan.check() != 0:
        raise RuntimeError("device error flags set during warm-up")

    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = (t1 - t0) / args.steps
    value = evals_per_step / sec
    log(f"{sec * 1e3:.4f} ms/step, {value:.4e} evals/s")

    # ---- live per-stage kernel timing (library-recorded HIP events) ----
    st = int(torch.cuda.current_stream().cuda_stream)
    # the step's own launches (the ECT inside the hybrid launch unless
    # --separate-ect), and the ECT and hybrid passes launched alone for reference
    names = ["precompute", "ect_hybrid_fused", "ect", "hybrid_fused", "hybrid_bwd_fourier"]
    evs = {nm: [(hipevents.Event(), hipevents.Event()) for _ in range(args.steps)] for nm in names}

    def arm(stage, pair_):
        N.check(N.ect_set_stage_events(stage, pair_[0].handle, pair_[1].handle), "stage events")

    for i in range(args.steps):
        arm(N.STAGE_PRECOMPUTE, evs["precompute"][i])
        if step.combined:
            plan.rerun_prepare(step.hy_q)   # as the step does: the query bucketing rides in this launch
        else:
            plan.rerun()
        arm(N.STAGE_HYBRID, evs["ect_hybrid_fused"][i])
        plan.ect_hybrid_multi(step.ect_q, step.ect_thr, step.hy_q, KERNELS, 1.0, "fp32", ect_out=step.ect_out,
                              outs=step.hy_out)
        arm(N.STAGE_ECT, evs["ect"][i])
        plan.ect(step.ect_q, step.ect_thr, out=step.ect_out)
        arm(N.STAGE_HYBRID, evs["hybrid_fused"][i])
        plan.hybrid_multi(step.hy_q, KERNELS, 1.0, "fp32", outs=step.hy_out)
        arm(N.STAGE_HYBRID_BWD, evs["hybrid_bwd_fourier"][i])
        plan.hybrid_backward(step.hy_q, step.hy_out["fourier"], step.grad_out, "fourier", 1.0, "fp32",
                             grad_xi=step.grad_xi, grad_s=step.grad_s)
    torch.cuda.synchronize()
    for stg in range(4):
        N.ect_set_stage_events(stg, None, None)
    stage_ms = {nm: float(np.mean([a.elapsed_ms(b) for a, b in evs[nm]])) for nm in names}
    log("stage kernel ms: " + ", ".join(f"{k}={v:.4f}" for k, v in stage_ms.items()))
    # "ect" and "hybrid_fused" are the two passes launched one after the other
    # with the step's knobs, for reference; the step itself launches
    # "ect_hybrid_fused" when it combines them
    in_step = (["precompute", "ect_hybrid_fused", "hybrid_bwd_fourier"] if step.combined
               else ["precompute", "ect", "hybrid_fused", "hybrid_bwd_fourier"])
    dom = max(in_step, key=stage_ms.get)
    dsec = stage_ms[dom] * 1e-3
    # the step's compaction launch also buckets the shared query set (16 B read and one record written per row)
    prep_bytes = (16.0 + 24.0) * len(w.hybrid_xi) if step.combined else 0.0
    if dom == "ect_hybrid_fused":
        roof = roofline.alu_roofline_parts([("ect", n, ect_pairs, 1.0),
                                            ("+".join(KERNELS), n, per_kernel_pairs, small_frac)], dsec)
    elif dom == "precompute":
        nbytes = img.size + 32.0 * float(cls_counts.sum() + counts.sum()) + 8 * 2 * 6 + prep_bytes
        roof = roofline.hbm_roofline(nbytes, dsec)
    elif dom == "ect":
        roof = roofline.alu_roofline("ect", n, ect_pairs, dsec)
    elif dom == "hybrid_bwd_fourier":
        roof = roofline.alu_roofline("fourier_bwd", n, per_kernel_pairs, dsec)
    else:
        roof = roofline.alu_roofline("+".join(KERNELS), n, per_kernel_pairs, dsec, small_frac)
    roof["kernel"] = dom
    roof["kernel_ms"] = stage_ms[dom]
    roof["traffic"] = None
    # HBM traffic of the dominant kernel from committed rocprofv3 counter runs, if taken on this source
    src_hash = source_digest(sorted(os.path.join(ROOT, "paper_2405_02256_amd", "csrc", f)
                                    for f in os.listdir(os.path.join(ROOT, "paper_2405_02256_amd", "csrc"))))
    tpath = os.path.join(ROOT, "profiles", "traffic_grf_512.json")
    if os.path.exists(tpath):
        try:
            tr = json.load(open(tpath))
            if tr.get("source_digest") == src_hash and dom in tr.get("bytes_per_launch", {}):
                roof["traffic"] = tr["bytes_per_launch"][dom]
        except (OSError, ValueError):
            pass

    # ---- Radon transform at the thresholds and the exact representations, same field ----
    next_rows = None
    if not args.no_next:
        log("Radon transform and exact representations")
        next_rows = measure_next(plan, w, dirs, thr, n, cls_counts, counts, args.steps)
        log("next rows: " + json.dumps(next_rows))

    # ---- four-axis workload ----
    four = None
    if not args.no_4d:
        log("four-axis workload")
        four = measure_4d(args.steps)
        log("four axes: " + json.dumps(four))

    # ---- FP64 path on the same step, for the FP32-vs-FP64 comparison ----
    fp64 = None
    if not args.no_fp64:
        step64 = pipeline.Step(plan, dirs, thr, xi, kernels=KERNELS, s=1.0, precision="fp64",
                               backward_kernel="fourier", grad_out=g_t, fused=True, concurrent=args.concurrent)
        step64.run()
        torch.cuda.synchronize()
        reps = max(3, args.steps // 5)
        t0 = time.perf_counter()
        for _ in range(reps):
            step64.run()
        torch.cuda.synchronize()
        fp64 = (time.perf_counter() - t0) / reps

    # ---- CPU baseline: the FP64 oracle on a bounded sample of the same step ----
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        b = args.cpu_budget
        full = {"ect": len(w.ect_dirs), "fourier": len(w.hybrid_xi), "laplace": len(w.hybrid_xi),
                "bessel": len(w.hybrid_xi), "grad": len(w.hybrid_xi)}
        base = {"ect": 72, "fourier": 512, "laplace": 512, "bessel": 96, "grad": 384}
        samp = {k: int(min(full[k], max(4, base[k] * b))) for k in base}
        tcpu = {}
        sel_d = np.linspace(0, len(w.ect_dirs) - 1, samp["ect"]).astype(int)
        t0 = time.perf_counter()
        O.ect(img, w.ect_dirs[sel_d], w.ect_thresholds)
        tcpu["ect"] = time.perf_counter() - t0
        for k in KERNELS:
            sel = np.linspace(0, len(w.hybrid_xi) - 1, samp[k]).astype(int)
            t0 = time.perf_counter()
            O.hybrid(img, w.hybrid_xi[sel], k, 1.0)
            tcpu[k] = time.perf_counter() - t0
        sel = np.linspace(0, len(w.hybrid_xi) - 1, samp["grad"]).astype(int)
        t0 = time.perf_counter()
        O.hybrid_grad(img, w.hybrid_xi[sel], "fourier", 1.0, gout[sel])
        tcpu["grad"] = time.perf_counter() - t0
        t_step = sum(tcpu[k] * full[k] / samp[k] for k in tcpu)
        cpu = {"value": evals_per_step / t_step, "unit": "ξ·crit-pt evals/s", "cores": O.max_threads(),
               "kind": "oracle",
               "sample": (f"FP64 oracle (cell forms over all cells) on {samp['ect']} of 360 ECT directions, "
                          f"{samp['fourier']}/{samp['laplace']}/{samp['bessel']} of 4096 xi for "
                          f"Fourier/Laplace/Bessel and {samp['grad']} xi of the Fourier gradient; "
                          f"{sum(tcpu.values()):.1f} s of wall time on {O.max_threads()} OpenMP threads "
                          f"(" + ", ".join(f"{k} {v:.2f} s" for k, v in tcpu.items()) + ") scaled to one "
                          f"full step ({t_step:.1f} s)")}

    # ---- batched FP32 (one graph) vs the plain per-image FP64 path, 4096 ragged images ----
    batch = None
    if not args.no_batch:
        log("batched comparison: 4096 ragged images")
        w4 = W.batch_4096(4)
        imgs4 = [torch.from_numpy(im).to(dev) for im in w4.images]
        plan4 = api.Plan(imgs4)
        dirs4 = torch.from_numpy(w4.ect_dirs).to(dev)
        thr4 = torch.from_numpy(w4.ect_thresholds).to(dev)
        xi4 = torch.from_numpy(w4.hybrid_xi).to(dev)
        nq = len(w4.hybrid_xi) // len(imgs4)
        offs4 = torch.arange(len(imgs4) + 1, dtype=torch.int64, device=dev) * nq
        step4 = pipeline.Step(plan4, dirs4, thr4, xi4, kernels=("laplace",), s=1.0, precision="fp32",
                              hybrid_offsets=offs4)
        if not args.no_autotune:
            step4.autotune()
        step4.capture()
        for _ in range(3):
            step4.replay()
        torch.cuda.synchronize()
        reps = 10
        t0 = time.perf_counter()
        for _ in range(reps):
            step4.replay()
        torch.cuda.synchronize()
        t_batched = (time.perf_counter() - t0) / reps
        y32 = step4.hy_out["laplace"].cpu().numpy()
        e32 = step4.ect_out.cpu().numpy()
        plans = [api.Plan(im) for im in imgs4]
        outs_e = [torch.empty((len(w4.ect_dirs), thr4.shape[1]), dtype=torch.int32, device=dev) for _ in plans]
        outs_h = [torch.empty(nq, dtype=torch.float64, device=dev) for _ in plans]
        xis = [xi4[i * nq:(i + 1) * nq] for i in range(len(plans))]

        def per_image():
            for i, pl in enumerate(plans):
                pl.rerun()
                pl.ect(dirs4, thr4[i], out=outs_e[i])
                pl.hybrid(xis[i], "laplace", 1.0, "fp64", out=outs_h[i])

        per_image()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        per_image()
        torch.cuda.synchronize()
        t_loop = time.perf_counter() - t0
        y64 = torch.cat(outs_h).cpu().numpy()
        e64 = torch.cat(outs_e).cpu().numpy()
        pairs4 = 0.0
        c4, o4 = plan4.counts()
        ex4 = w4.hybrid_xi.reshape(len(imgs4), nq, 2)
        e_idx = (ex4[..., 0] < 0) * 1 + (ex4[..., 1] < 0) * 2
        pr = np.where(e_idx >= 2, e_idx ^ 3, e_idx)
        pairs4 = float(np.take_along_axis(o4, pr, axis=1).sum())
        # the batch's precompute alone (count / scan / write launches, library stage events), priced
        # against HBM with the bytes it cannot avoid: every pixel read once, 32 B per list entry
        # written, the list offsets
        pe = [(hipevents.Event(), hipevents.Event()) for _ in range(reps)]
        for i in range(reps):
            N.check(N.ect_set_stage_events(N.STAGE_PRECOMPUTE, pe[i][0].handle, pe[i][1].handle), "stage events")
            plan4.rerun()
        torch.cuda.synchronize()
        N.ect_set_stage_events(N.STAGE_PRECOMPUTE, None, None)
        pre_ms = float(np.mean([a.elapsed_ms(b) for a, b in pe]))
        px_bytes = float(sum(im.size * im.itemsize for im in w4.images))
        entries4 = float(c4.sum() + o4.sum())
        pre_bytes = px_bytes + 32.0 * entries4 + 8.0 * (len(imgs4) + 1) * (c4.shape[1] + o4.shape[1])
        vertices4 = float(sum((im.shape[0] + 1) * (im.shape[1] + 1) for im in w4.images))
        batch = {"workload": "batch_4096: 4096 binary GRF images, sides U{28,64,128,256}, sigma U[2,8]; "
                             "ECT 128 dirs x 128 per-image thresholds; Euler-Laplace at 512 xi per image",
                 "batched_fp32_graph_ms": t_batched * 1e3, "per_image_fp64_loop_ms": t_loop * 1e3,
                 "speedup": t_loop / t_batched,
                 "hybrid_evals_per_s_batched": pairs4 / t_batched,
                 "ect_dirs_per_s_batched": len(imgs4) * len(w4.ect_dirs) / t_batched,
                 "ect_identical": bool(np.array_equal(e32, e64)),
                 "fp32_vs_fp64_normwise": float(np.abs(y32 - y64).max() / np.abs(y64).max()),
                 "precompute_ms": pre_ms, "precompute_vertices": vertices4, "precompute_list_entries": entries4,
                 "precompute_hbm_roofline": roofline.hbm_roofline(pre_bytes, pre_ms * 1e-3),
                 "precompute_vertices_per_s": vertices4 / (pre_ms * 1e-3)}
        log(f"batched {t_batched * 1e3:.3f} ms vs per-image FP64 loop {t_loop * 1e3:.1f} ms")

    res = {
        "metric": METRIC,
        "value": value,
        "unit": "ξ·crit-pt evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "grf_512: 512x512 binary Gaussian random field (sigma 8 px, median "
                               "threshold), primal cubical complex; ECT 360 dirs x 256 thresholds; "
                               "Euler-Fourier/Laplace/Bessel at 4096 xi, |xi|~U[0.01,1]; Fourier backward",
                   "graph": use_graph, "precision": "FP32 kernel values, FP64 phases and accumulation",
                   "tuning": tuning},
        "ect_dirs_per_s": len(w.ect_dirs) / sec,
        "evals_per_step": evals_per_step,
        "stage_kernel_ms": stage_ms,
        "stage_note": ("the step launches precompute (which also buckets the shared query set), "
                       "ect_hybrid_fused (the ECT inside the fused hybrid pass) and hybrid_bwd_fourier; ect and "
                       "hybrid_fused are the two passes launched separately with the step's knobs, for reference")
                      if step.combined else None,
        "bessel_small_branch_fraction": small_frac,
        "roofline": roof,
        "fp64_path_ms_per_step": None if fp64 is None else fp64 * 1e3,
        "fp32_vs_fp64_speedup": None if fp64 is None else fp64 / sec,
        "batched_vs_per_image": batch,
        "radon_and_exact": next_rows,
        "four_axes": four,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
