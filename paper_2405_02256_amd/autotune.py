"""Schedule autotuner for a plan and its queries.

Two knobs of a plan change only how the work is scheduled, never what is
computed (the ECT stays exact, hybrid sums change only in the rounding of the
chunked partial sums):

* the point-chunk length of a hybrid work item (image, orthant pair, 64-query
  tile, chunk of list entries) -- short chunks give many small work items that
  fill the 256 compute units but cost more partial sums, long ones the reverse;
* the number of directions one ECT workgroup evaluates per streamed point and,
  for shared direction sets, the number of parts each list is split into so
  that several workgroups share one group of directions; the automatic
  setting (0, 0) also lets many-image batches with short lists take the
  direction-parallel kernel.  When the ECT runs
  inside the hybrid launch (ect_hybrid_eval_multi) these are swept again on
  that combined call: there the ECT work is hidden beside the hybrid work
  items and list parts only add a chunk-sum launch, so the best setting
  differs from the one for a separate ECT launch.

The tuner times each candidate on the device with events around a few
repetitions of the real calls, keeps the fastest and stores it in a JSON cache
keyed by the device architecture, the library version and a signature of the
workload (image shapes, list sizes, query counts, kernels, precision), so a
later process with the same workload skips the sweep.
"""
from __future__ import annotations

import json
import os
import statistics
import tempfile
from dataclasses import dataclass, field

from . import _native as N

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_2405_02256_amd", "tuning.json")
# (directions per workgroup, list parts; 0 = automatic)
ECT_CANDIDATES = ((1, 1), (2, 1), (4, 1), (8, 1), (1, 0), (2, 0), (4, 0), (8, 0), (1, 2), (1, 4), (2, 2), (2, 4),
                  (0, 0))
HYBRID_ITEM_CANDIDATES = (512, 1024, 2048, 4096, 8192, 16384)


@dataclass
class Tuning:
    hybrid_chunk: int = 0
    hybrid_target_items: int = 2048
    ect_dirs_per_group: int = 0
    ect_chunks: int = 0
    timings: dict = field(default_factory=dict)

    def as_args(self):
        return (int(self.hybrid_chunk), int(self.hybrid_target_items), int(self.ect_dirs_per_group),
                int(self.ect_chunks))

    def to_json(self):
        return {"hybrid_chunk": int(self.hybrid_chunk), "hybrid_target_items": int(self.hybrid_target_items),
                "ect_dirs_per_group": int(self.ect_dirs_per_group), "ect_chunks": int(self.ect_chunks),
                "timings": self.timings}

    @staticmethod
    def from_json(d):
        return Tuning(int(d["hybrid_chunk"]), int(d["hybrid_target_items"]), int(d["ect_dirs_per_group"]),
                      int(d.get("ect_chunks", 0)), dict(d.get("timings", {})))


def signature(plan, ect_rows=0, ect_thresholds=0, hybrid_rows=0, kernels=(), precision="fp32",
              backward=None) -> str:
    """Workload key: what the schedule depends on, not the data values."""
    c, o = plan.counts()
    shapes = sorted({tuple(int(d) for d in row) for row in plan.dims})
    parts = [
        f"n{plan.ndim}", f"c{int(plan.construction)}", f"i{plan.num_images}",
        "s" + ";".join("x".join(map(str, s)) for s in shapes[:8]) + (f"+{len(shapes) - 8}" if len(shapes) > 8 else ""),
        f"cl{int(c.sum())}/{int(c.max()) if c.size else 0}", f"or{int(o.sum())}/{int(o.max()) if o.size else 0}",
        f"e{int(ect_rows)}x{int(ect_thresholds)}", f"h{int(hybrid_rows)}",
        "k" + "+".join(kernels), f"p{precision}", f"b{backward or '-'}",
    ]
    return "|".join(parts)


def device_key(device=None) -> str:
    import torch
    props = torch.cuda.get_device_properties(device if device is not None else torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", props.name)
    return f"{arch}|cu{props.multi_processor_count}|lib{N.version()}"


class Cache:
    """JSON file of {device key: {workload signature: tuning}}; writes are atomic."""

    def __init__(self, path: str | None = None):
        self.path = path or os.environ.get("ECT_TUNE_CACHE", DEFAULT_CACHE)

    def load(self) -> dict:
        try:
            with open(self.path) as f:
                d = json.load(f)
            return d if isinstance(d, dict) else {}
        except (OSError, ValueError):
            return {}

    def get(self, dev: str, sig: str) -> Tuning | None:
        e = self.load().get(dev, {}).get(sig)
        try:
            return Tuning.from_json(e) if e is not None else None
        except (KeyError, TypeError, ValueError):
            return None

    def put(self, dev: str, sig: str, t: Tuning) -> None:
        d = self.load()
        d.setdefault(dev, {})[sig] = t.to_json()
        folder = os.path.dirname(self.path) or "."
        os.makedirs(folder, exist_ok=True)
        fd, tmp = tempfile.mkstemp(dir=folder, prefix=".tuning", suffix=".json")
        with os.fdopen(fd, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def pick(timings: dict):
    """Fastest candidate; ties keep the earlier (smaller) one."""
    best, best_t = None, float("inf")
    for k, t in timings.items():
        if t < best_t:
            best, best_t = k, t
    return best


def time_call(fn, reps: int = 10, warmup: int = 2, trials: int = 5) -> float:
    """Median over trials of the mean device time (ms) of fn() on the current stream."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(trials):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        b.synchronize()
        out.append(a.elapsed_time(b) / reps)
    return statistics.median(out)


def tune(plan, ect_dirs=None, ect_thresholds=None, hybrid_xi=None, kernels=("fourier",), s=1.0,
         precision="fp32", ect_offsets=None, hybrid_offsets=None, backward_kernel=None, grad_out=None,
         cache: Cache | None = None, use_cache=True, reps=10, timer=None, dev_key: str | None = None,
         combined: bool = False, log_scale: bool = False) -> Tuning:
    """Sweep the knobs for this plan's ECT and hybrid calls, apply the fastest
    to the plan and return it (from the cache when the workload was seen).
    log_scale: the Laplace output is taken with a log-scale output, as the
    timed calls then make it (large phases would overflow without one)."""
    import torch
    timer = timer or time_call
    cache = cache or Cache()
    from .api import QuerySet
    eq = None if ect_dirs is None else (ect_dirs if isinstance(ect_dirs, QuerySet) else QuerySet(ect_dirs, ect_offsets))
    hq = None if hybrid_xi is None else (hybrid_xi if isinstance(hybrid_xi, QuerySet) else QuerySet(hybrid_xi, hybrid_offsets))
    e_rows = eq.rows(plan.num_images) if eq is not None else 0
    h_rows = hq.rows(plan.num_images) if hq is not None else 0
    M = int(ect_thresholds.shape[-1]) if ect_thresholds is not None else 0
    combined = bool(combined and e_rows > 0 and h_rows > 0)
    sig = signature(plan, e_rows, M, h_rows, tuple(kernels) if hq is not None else (), precision, backward_kernel)
    if combined:
        sig += "|one-launch"
    if log_scale:
        sig += "|log-scale"
    dev = dev_key or device_key()
    if use_cache:
        hit = cache.get(dev, sig)
        if hit is not None:
            plan.set_tuning(*hit.as_args())
            return hit

    best = Tuning()
    timings = {}
    if eq is not None and e_rows > 0:
        ect_t = {}
        out = None
        for td, ch in ECT_CANDIDATES:
            plan.set_tuning(0, best.hybrid_target_items, td, ch)
            out = plan.ect(eq, ect_thresholds, slot="ect")

            def run(o=out):
                plan.ect(eq, ect_thresholds, out=o, slot="ect")
            ect_t[(td, ch)] = timer(run, reps)
        best.ect_dirs_per_group, best.ect_chunks = pick(ect_t)
        timings["ect"] = {f"{k[0]}/{k[1]}": v for k, v in ect_t.items()}
    ls = None
    if hq is not None and h_rows > 0 and log_scale and "laplace" in kernels:
        ls = torch.empty(h_rows, dtype=torch.float64, device=plan.device)
    if hq is not None and h_rows > 0:
        hy_t = {}
        kernels = tuple(kernels)
        for items in HYBRID_ITEM_CANDIDATES:
            plan.set_tuning(0, items, best.ect_dirs_per_group, best.ect_chunks)
            if len(kernels) > 1:
                outs = plan.hybrid_multi(hq, kernels, s, precision, log_scale_out=ls)
            else:
                outs = {kernels[0]: plan.hybrid(hq, kernels[0], s, precision, log_scale_out=ls)}
            fwd = outs.get(backward_kernel) if backward_kernel else None
            if fwd is not None and grad_out is None:
                grad_out = torch.ones_like(fwd)
            gxi = torch.empty((hq.vecs.shape[0], plan.ndim), dtype=torch.float64, device=plan.device)
            gs = torch.empty((), dtype=torch.float64, device=plan.device)

            def run(outs=outs, fwd=fwd):
                if len(kernels) > 1:
                    plan.hybrid_multi(hq, kernels, s, precision, outs=outs, log_scale_out=ls)
                else:
                    plan.hybrid(hq, kernels[0], s, precision, out=outs[kernels[0]], log_scale_out=ls)
                if fwd is not None:
                    plan.hybrid_backward(hq, fwd, grad_out, backward_kernel, s, precision, grad_xi=gxi, grad_s=gs)
            hy_t[items] = timer(run, reps)
        best.hybrid_target_items = pick(hy_t)
        timings["hybrid"] = {str(k): v for k, v in hy_t.items()}
    if combined:
        co_t = {}
        for td, ch in ECT_CANDIDATES:
            plan.set_tuning(0, best.hybrid_target_items, td, ch)
            eo, ho = plan.ect_hybrid_multi(eq, ect_thresholds, hq, kernels, s, precision, log_scale_out=ls)
            fwd = ho.get(backward_kernel) if backward_kernel else None
            if fwd is not None and grad_out is None:
                grad_out = torch.ones_like(fwd)
            gxi = torch.empty((hq.vecs.shape[0], plan.ndim), dtype=torch.float64, device=plan.device)
            gs = torch.empty((), dtype=torch.float64, device=plan.device)

            def run(eo=eo, ho=ho, fwd=fwd):
                plan.ect_hybrid_multi(eq, ect_thresholds, hq, kernels, s, precision, ect_out=eo, outs=ho,
                                      log_scale_out=ls)
                if fwd is not None:
                    plan.hybrid_backward(hq, fwd, grad_out, backward_kernel, s, precision, grad_xi=gxi, grad_s=gs)
            co_t[(td, ch)] = timer(run, reps)
        best.ect_dirs_per_group, best.ect_chunks = pick(co_t)
        timings["ect_hybrid"] = {f"{k[0]}/{k[1]}": v for k, v in co_t.items()}
    best.timings = timings
    plan.set_tuning(*best.as_args())
    if use_cache:
        cache.put(dev, sig, best)
    return best
