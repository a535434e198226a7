"""Whole-path orchestration: one pass over a batch with every buffer preallocated.

``Step`` binds a ``Plan`` to its query sets and output buffers so that one
call to ``run()`` enqueues the complete hot path on the current stream --
precompute kernels (classification and ordered compaction), sign-vector
bucketing, the exact ECT, the hybrid transforms for every requested kernel
(fused into one pass over the (query, point) pairs by default) and,
optionally, one backward pass -- without allocating, copying or
synchronising.  ``capture()`` records that sequence once into a HIP graph
(through torch.cuda.CUDAGraph) so that a replay costs one launch.

The ECT and the hybrid transforms only read the precomputed lists.  By
default (``combined=True``) the step evaluates both with one call
(ect_hybrid_eval_multi), which for a shared direction set puts the ECT
workgroups into the launch of the fused hybrid pass: the short, latency-bound
ECT work then fills compute units beside the long hybrid work items instead of
running before them.  With ``concurrent=True`` the ECT branch instead runs on
a side stream (its own workspace) between an event after the precompute and a
join before the step ends; in a captured graph the fork and join become graph
edges.
"""
from __future__ import annotations

import torch

from .api import Plan, QuerySet


class Step:
    def __init__(self, plan: Plan, ect_dirs=None, ect_thresholds=None, hybrid_xi=None, kernels=("fourier",),
                 s: float = 1.0, precision: str = "fp32", ect_offsets=None, hybrid_offsets=None,
                 backward_kernel: str | None = None, grad_out: torch.Tensor | None = None,
                 log_scale_laplace: bool = False, rerun_precompute: bool = True, fused: bool = True,
                 concurrent: bool = False, reuse_prepared: bool = True, combined: bool = True):
        self.plan = plan
        self.reuse_prepared = reuse_prepared
        dev = plan.device
        self.rerun_precompute = rerun_precompute
        self.ect_q = None if ect_dirs is None else QuerySet(ect_dirs, ect_offsets)
        self.ect_thr = None if ect_thresholds is None else ect_thresholds.to(device=dev, dtype=torch.float64).contiguous()
        self.hy_q = None if hybrid_xi is None else QuerySet(hybrid_xi, hybrid_offsets)
        self.kernels = tuple(kernels) if self.hy_q is not None else ()
        self.s = float(s)
        self.precision = precision
        self.log_scale_laplace = log_scale_laplace
        self.fused = fused
        if self.ect_q is not None:
            self.ect_q.validate(plan.num_images, plan.ndim)
            rows = self.ect_q.rows(plan.num_images)
            self.ect_out = torch.empty((rows, self.ect_thr.shape[-1]), dtype=torch.int32, device=dev)
        self.hy_out = {}
        self.hy_ls = {}
        if self.hy_q is not None:
            self.hy_q.validate(plan.num_images, plan.ndim)
            rows = self.hy_q.rows(plan.num_images)
            for k in self.kernels:
                shape = (rows, 2) if k == "fourier" else (rows,)
                self.hy_out[k] = torch.empty(shape, dtype=torch.float64, device=dev)
                if k == "laplace" and log_scale_laplace:
                    self.hy_ls[k] = torch.empty(rows, dtype=torch.float64, device=dev)
        self.backward_kernel = backward_kernel
        if backward_kernel is not None:
            if backward_kernel not in self.kernels:
                raise ValueError("backward kernel must be one of the forward kernels")
            self.grad_out = grad_out.to(device=dev, dtype=torch.float64).contiguous()
            self.grad_xi = torch.empty((self.hy_q.vecs.shape[0], plan.ndim), dtype=torch.float64, device=dev)
            self.grad_s = torch.empty((), dtype=torch.float64, device=dev)
        self.graph = None
        self.concurrent = concurrent and self.ect_q is not None and self.hy_q is not None
        self.combined = (combined and not self.concurrent and self.ect_q is not None and self.hy_q is not None
                         and fused)
        if self.concurrent:
            self.side = torch.cuda.Stream(device=dev)
            self._fork = torch.cuda.Event()
            self._join = torch.cuda.Event()

    def run(self, stream=None) -> None:
        p = self.plan
        main = stream if stream is not None else torch.cuda.current_stream()
        if self.rerun_precompute:
            if self.combined and self.hy_q.offsets is None:
                # the shared query set is bucketed in the compaction launch
                p.rerun_prepare(self.hy_q, main)
            else:
                p.rerun(main)
        if self.combined:
            p.ect_hybrid_multi(self.ect_q, self.ect_thr, self.hy_q, self.kernels, self.s, self.precision,
                               ect_out=self.ect_out, outs=self.hy_out, log_scale_out=self.hy_ls.get("laplace"),
                               stream=main)
        else:
            self._ect(main)
            self._hybrid(main)
        stream = main
        if self.backward_kernel is not None:
            # the forward calls just bucketed this query set into the same workspace
            p.hybrid_backward(self.hy_q, self.hy_out[self.backward_kernel], self.grad_out, self.backward_kernel,
                              self.s, self.precision, stream=stream, grad_xi=self.grad_xi, grad_s=self.grad_s,
                              reuse_prepared=self.reuse_prepared)
        if self.concurrent:
            main.wait_event(self._join)

    def _ect(self, main) -> None:
        p = self.plan
        if self.ect_q is None:
            return
        if self.concurrent:
            self._fork.record(main)
            self.side.wait_event(self._fork)
            p.ect(self.ect_q, self.ect_thr, out=self.ect_out, stream=self.side, slot="ect")
            self._join.record(self.side)
        else:
            p.ect(self.ect_q, self.ect_thr, out=self.ect_out, stream=main)

    def _hybrid(self, stream) -> None:
        p = self.plan
        if self.fused and len(self.kernels) > 1:
            p.hybrid_multi(self.hy_q, self.kernels, self.s, self.precision, outs=self.hy_out,
                           log_scale_out=self.hy_ls.get("laplace"), stream=stream)
            return
        for k in self.kernels:
            if k in self.hy_ls:
                p.hybrid(self.hy_q, k, self.s, self.precision, out=self.hy_out[k], log_scale_out=self.hy_ls[k],
                         stream=stream)
            else:
                p.hybrid(self.hy_q, k, self.s, self.precision, out=self.hy_out[k], stream=stream)

    def autotune(self, cache=None, use_cache: bool = True, reps: int = 20):
        """Pick the plan's schedule knobs for this step's queries (before capture())."""
        from . import autotune as AT
        return AT.tune(self.plan, self.ect_q, self.ect_thr, self.hy_q, self.kernels, self.s, self.precision,
                       backward_kernel=self.backward_kernel,
                       grad_out=self.grad_out if self.backward_kernel is not None else None,
                       cache=cache, use_cache=use_cache, reps=reps, combined=self.combined,
                       log_scale=self.log_scale_laplace)

    def capture(self) -> "torch.cuda.CUDAGraph":
        """Record run() into a graph (after one eager run sized every workspace).

        The graph keeps the evaluation workspace it recorded alive, so later
        eager calls on the plan that need a larger one cannot free it."""
        self.run()
        torch.cuda.synchronize()
        self.graph_ws = dict(self.plan._eval_ws)
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                self.run()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = g
        return g

    def replay(self) -> None:
        self.graph.replay()
