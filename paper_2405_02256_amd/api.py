"""PyTorch-facing layer over the C ABI: device memory and streams only.

``Plan`` owns the workspace tensors of one precomputed batch and exposes the
evaluation calls; ``HybridTransform`` is the autograd Function whose backward
is the library's hand-written vector-Jacobian product.  Every numeric step
runs in libect.so on the GPU.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _native as N

_DTYPES = {torch.uint8: N.U8, torch.int16: N.I16, torch.int32: N.I32}


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _device_scale(s, device):
    """A device float64 scalar for the *_s entry points (None when s is a Python number)."""
    if not torch.is_tensor(s):
        return None
    t = s.detach()
    if t.numel() != 1 or t.device != device:
        raise ValueError("a tensor scale must be one element on the plan's device")
    return t.reshape(()).to(torch.float64).contiguous()


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class QuerySet:
    """FP64 query vectors on the device: shared (one set for every image) or ragged."""

    def __init__(self, vecs: torch.Tensor, offsets: torch.Tensor | None = None):
        if vecs.dtype != torch.float64 or not vecs.is_cuda or vecs.dim() != 2:
            raise ValueError("query vectors must be a CUDA float64 tensor [rows][ndim]")
        self.vecs = vecs.contiguous()
        self.offsets = None if offsets is None else offsets.to(device=vecs.device, dtype=torch.int64).contiguous()

    def validate(self, num_images: int, ndim: int) -> None:
        """Check shapes once per (num_images, ndim); the offsets check reads them back to the host,
        so a set used inside graph capture must have been validated before."""
        if getattr(self, "_checked", None) == (num_images, ndim):
            return
        if self.vecs.shape[1] != ndim:
            raise ValueError(f"query vectors have {self.vecs.shape[1]} columns, expected {ndim}")
        if self.offsets is not None:
            o = self.offsets.cpu().numpy()
            if o.shape != (num_images + 1,) or o[0] != 0 or o[-1] != self.vecs.shape[0] or (np.diff(o) < 0).any():
                raise ValueError("ragged offsets must be [num_images+1], start at 0, be non-decreasing and "
                                 "end at the number of rows")
        self._checked = (num_images, ndim)

    def rows(self, num_images: int) -> int:
        return self.vecs.shape[0] if self.offsets is not None else self.vecs.shape[0] * num_images

    def c(self) -> N.QuerySet:
        return N.QuerySet(_dptr(self.vecs), _dptr(self.offsets), self.vecs.shape[0])


class Plan:
    """Critical-point lists of a batch of images (ect_precompute).

    images: list of integer tensors on one CUDA device (numpy axis order: the
    last index is embedding axis 0), or one tensor for a single image.
    """

    def __init__(self, images, construction: int = N.PRIMAL, origin=None, spacing=None, stream=None):
        if isinstance(images, torch.Tensor):
            images = [images]
        if not images:
            raise ValueError("empty batch")
        dev = images[0].device
        dt = images[0].dtype
        if dt not in _DTYPES or not images[0].is_cuda:
            raise ValueError("images must be CUDA uint8/int16/int32 tensors")
        ndim = images[0].dim()
        if ndim not in (2, 3, 4) or any(im.dim() != ndim or im.dtype != dt or im.device != dev for im in images):
            raise ValueError("every image must have the same ndim (2, 3 or 4), dtype and device")
        self.ndim = ndim
        self.construction = int(construction)
        self.tuning = (0, 2048, 0, 0)
        self.num_images = len(images)
        self.device = dev
        flat = [im.reshape(-1) for im in images]
        self.pixels = torch.cat(flat) if len(flat) > 1 else flat[0].contiguous()
        self.dims = np.array([list(reversed(im.shape)) for im in images], dtype=np.int32)
        offs = np.zeros(len(images), dtype=np.int64)
        if len(images) > 1:
            offs[1:] = np.cumsum([f.numel() for f in flat[:-1]])
        self.pixel_offsets = offs
        self.origin = None if origin is None else np.ascontiguousarray(np.asarray(origin, np.float64).reshape(-1, ndim))
        self.spacing = None if spacing is None else np.ascontiguousarray(np.asarray(spacing, np.float64).reshape(-1, ndim))
        if self.origin is not None and self.origin.shape[0] == 1 and self.num_images > 1:
            self.origin = np.ascontiguousarray(np.repeat(self.origin, self.num_images, 0))
        if self.spacing is not None and self.spacing.shape[0] == 1 and self.num_images > 1:
            self.spacing = np.ascontiguousarray(np.repeat(self.spacing, self.num_images, 0))
        self._batch = N.ImageBatch(
            ndim, len(images), self.dims.ctypes.data_as(N.P(N.c_i32)),
            self.pixel_offsets.ctypes.data_as(N.P(N.c_i64)), _dptr(self.pixels), _DTYPES[dt], construction,
            None if self.origin is None else self.origin.ctypes.data_as(N.P(N.c_f64)),
            None if self.spacing is None else self.spacing.ctypes.data_as(N.P(N.c_f64)))
        st = _stream(stream)
        need = ctypes.c_size_t(0)
        status, _ = N.ect_precompute(self._batch, None, need, st)
        N.check(status, "ect_precompute(size)")
        self.ws = _workspace(need.value, dev)
        have = ctypes.c_size_t(self.ws.numel())
        status, handle = N.ect_precompute(self._batch, ctypes.c_void_p(_dptr(self.ws)), have, st)
        N.check(status, "ect_precompute")
        self.handle = handle
        self._eval_ws = {}

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "handle", None):
            N.ect_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ------------------------------------------------------------
    def _ws(self, nbytes: int, slot: str = "main") -> torch.Tensor:
        """Evaluation workspace `slot`: calls that may run at the same time on
        different streams must use different slots."""
        ws = self._eval_ws.get(slot)
        if ws is None or ws.numel() < nbytes:
            ws = self._eval_ws[slot] = _workspace(nbytes, self.device)
        return ws

    def rerun_prepare(self, xi, stream=None, slot: str = "main") -> None:
        """rerun(), bucketing the shared query set xi in the same launch for the next forward hybrid call
        on this workspace slot (ect_plan_rerun_prepare); plans it does not apply to are just re-run."""
        q = xi if isinstance(xi, QuerySet) else QuerySet(xi)
        q.validate(self.num_images, self.ndim)
        if q.offsets is not None:
            raise ValueError("rerun_prepare takes a shared query set")
        st = _stream(stream)
        need = ctypes.c_size_t(0)
        N.check(N.ect_plan_rerun_prepare(self.handle, q.c(), None, need, st), "ect_plan_rerun_prepare(size)")
        ws = self._ws(need.value, slot)
        have = ctypes.c_size_t(ws.numel())
        N.check(N.ect_plan_rerun_prepare(self.handle, q.c(), ctypes.c_void_p(_dptr(ws)), have, st),
                "ect_plan_rerun_prepare")

    def set_tuning(self, hybrid_chunk: int = 0, hybrid_target_items: int = 2048, ect_dirs_per_group: int = 0,
                   ect_chunks: int = 0):
        """Schedule knobs (0 = automatic): hybrid point chunk, hybrid work items,
        directions per ECT workgroup, parts per list for shared ECT sets."""
        N.check(N.ect_plan_set_tuning(self.handle, hybrid_chunk, hybrid_target_items, ect_dirs_per_group,
                                      ect_chunks), "ect_plan_set_tuning")
        self.tuning = (hybrid_chunk, hybrid_target_items, ect_dirs_per_group, ect_chunks)

    def rerun(self, stream=None):
        N.check(N.ect_plan_rerun(self.handle, _stream(stream)), "ect_plan_rerun")

    def counts(self):
        nc, no = 1 << self.ndim, 1 << (self.ndim - 1)
        c = np.zeros((self.num_images, nc), np.int64)
        o = np.zeros((self.num_images, no), np.int64)
        N.check(N.ect_plan_counts(self.handle, c.ctypes.data_as(N.P(N.c_i64)), o.ctypes.data_as(N.P(N.c_i64))),
                "ect_plan_counts")
        return c, o

    def export(self, image: int, kind: int, lst: int, stream=None):
        """(coords [count][ndim] vertex indices, values [count]) of one list (kind 0 classical, 1 ordinary)."""
        cnt = ctypes.c_int64(0)
        st = _stream(stream)
        N.check(N.ect_plan_export(self.handle, image, kind, lst, None, None, 0, ctypes.byref(cnt), st),
                "ect_plan_export(count)")
        n = cnt.value
        coords = np.zeros((max(n, 1), self.ndim), np.int32)
        vals = np.zeros(max(n, 1), np.int32)
        N.check(N.ect_plan_export(self.handle, image, kind, lst, coords.ctypes.data_as(N.P(N.c_i32)),
                                  vals.ctypes.data_as(N.P(N.c_i32)), n, ctypes.byref(cnt), st), "ect_plan_export")
        return coords[:n], vals[:n]

    def check(self, stream=None) -> int:
        f = ctypes.c_uint32(0)
        N.check(N.ect_plan_check(self.handle, ctypes.byref(f), _stream(stream)), "ect_plan_check")
        return f.value

    # -- evaluation ---------------------------------------------------------
    def ect(self, dirs, thresholds: torch.Tensor, offsets=None, out=None, stream=None, slot: str = "main") -> torch.Tensor:
        """int32 [rows][M]: ECT at every direction and threshold (thresholds [M] or [num_images][M])."""
        return self._thresholds(N.ect_eval, "ect_eval", dirs, thresholds, offsets, out, stream, slot)

    def radon(self, dirs, thresholds: torch.Tensor, offsets=None, out=None, stream=None,
              slot: str = "main") -> torch.Tensor:
        """int32 [rows][M]: Radon transform (slice Euler characteristic) at every direction and threshold."""
        return self._thresholds(N.radon_eval, "radon_eval", dirs, thresholds, offsets, out, stream, slot)

    def _thresholds(self, fn, name, dirs, thresholds, offsets, out, stream, slot):
        q = dirs if isinstance(dirs, QuerySet) else QuerySet(dirs, offsets)
        q.validate(self.num_images, self.ndim)
        thr = thresholds.to(device=self.device, dtype=torch.float64).contiguous()
        per_image = 1 if thr.dim() == 2 else 0
        if thr.dim() not in (1, 2) or (per_image and thr.shape[0] != self.num_images):
            raise ValueError("thresholds must be [M] or [num_images][M]")
        M = thr.shape[-1]
        rows = q.rows(self.num_images)
        if out is None:
            out = torch.empty((rows, M), dtype=torch.int32, device=self.device)
        st = _stream(stream)
        need = ctypes.c_size_t(0)
        N.check(fn(self.handle, q.c(), _dptr(thr), M, per_image, _dptr(out), None, need, st), name + "(size)")
        ws = self._ws(need.value, slot)
        have = ctypes.c_size_t(ws.numel())
        N.check(fn(self.handle, q.c(), _dptr(thr), M, per_image, _dptr(out), ctypes.c_void_p(_dptr(ws)), have, st),
                name)
        return out

    def exact(self, dirs, kind: str = "ect", offsets=None, stream=None, slot: str = "main",
              reuse: "ExactRepresentation | None" = None) -> "ExactRepresentation":
        """Exact representation of every query row (ect_exact_layout, then ect_exact): kind "ect" gives
        (T, E), "radon" gives (T, E', Tc, Ec).  Reads the total size back to the host once.  With
        `reuse` (a representation of the same kind, plan contents and query set) its layout and arrays
        are rebuilt in place: no layout call, no host read-back."""
        kinds = {"ect": N.EXACT_ECT, "radon": N.EXACT_RADON}
        if kind not in kinds:
            raise ValueError(f"kind must be one of {sorted(kinds)}")
        k = kinds[kind]
        q = dirs if isinstance(dirs, QuerySet) else QuerySet(dirs, offsets)
        q.validate(self.num_images, self.ndim)
        rows = q.rows(self.num_images)
        st = _stream(stream)
        if reuse is not None:
            if reuse.kind != k or reuse.rows != rows:
                raise ValueError("reuse needs a representation of the same kind and number of rows")
            need = ctypes.c_size_t(0)
            args = (self.handle, q.c(), k, _dptr(reuse.row_off), reuse.capacity, _dptr(reuse.T), _dptr(reuse.E),
                    _dptr(reuse.length))
            N.check(N.ect_exact(*args, None, need, st), "ect_exact(size)")
            ws = self._ws(need.value, slot)
            have = ctypes.c_size_t(ws.numel())
            N.check(N.ect_exact(*args, ctypes.c_void_p(_dptr(ws)), have, st), "ect_exact")
            return reuse
        row_off = torch.empty(rows + 1, dtype=torch.int64, device=self.device)
        need = ctypes.c_size_t(0)
        N.check(N.ect_exact_layout(self.handle, q.c(), k, _dptr(row_off), None, need, st), "ect_exact_layout(size)")
        ws = self._ws(need.value, slot)
        have = ctypes.c_size_t(ws.numel())
        N.check(N.ect_exact_layout(self.handle, q.c(), k, _dptr(row_off), ctypes.c_void_p(_dptr(ws)), have, st),
                "ect_exact_layout")
        with torch.cuda.stream(stream) if stream is not None else _nullctx():
            capacity = int(row_off[rows].item())
        T = torch.empty(max(capacity, 1), dtype=torch.float64, device=self.device)
        E = torch.empty(max(capacity, 1), dtype=torch.int32, device=self.device)
        length = torch.empty((rows, 2) if k == N.EXACT_RADON else (rows,), dtype=torch.int64, device=self.device)
        need = ctypes.c_size_t(0)
        N.check(N.ect_exact(self.handle, q.c(), k, _dptr(row_off), capacity, _dptr(T), _dptr(E), _dptr(length),
                            None, need, st), "ect_exact(size)")
        ws = self._ws(need.value, slot)
        have = ctypes.c_size_t(ws.numel())
        N.check(N.ect_exact(self.handle, q.c(), k, _dptr(row_off), capacity, _dptr(T), _dptr(E), _dptr(length),
                            ctypes.c_void_p(_dptr(ws)), have, st), "ect_exact")
        return ExactRepresentation(k, row_off, T, E, length, capacity)

    def hybrid(self, xi, kernel: str = "fourier", s: float = 1.0, precision: str = "fp32", offsets=None,
               log_scale: bool = False, out=None, stream=None, log_scale_out=None, slot: str = "main"):
        """float64 [rows] (Fourier: [rows][2]); with log_scale (Laplace) returns (out, log_scale)."""
        q = xi if isinstance(xi, QuerySet) else QuerySet(xi, offsets)
        q.validate(self.num_images, self.ndim)
        k = N.KERNELS[kernel]
        rows = q.rows(self.num_images)
        if out is None:
            out = torch.empty((rows, 2) if k == N.FOURIER else (rows,), dtype=torch.float64, device=self.device)
        if log_scale_out is not None:
            log_scale = True
        ls = log_scale_out if log_scale_out is not None else (
            torch.empty(rows, dtype=torch.float64, device=self.device) if log_scale else None)
        st = _stream(stream)
        sd = _device_scale(s, self.device)
        need = ctypes.c_size_t(0)
        if sd is not None:
            # the kernels read the scale from device memory (no host copy)
            ptrs = [_dptr(out) if k == kk else 0 for kk in (N.FOURIER, N.LAPLACE, N.BESSEL)]
            N.check(N.hybrid_eval_multi_s(self.handle, 1 << k, _dptr(sd), N.PRECISIONS[precision], q.c(), *ptrs,
                                          _dptr(ls), None, need, st), "hybrid_eval_multi_s(size)")
            ws = self._ws(need.value, slot)
            have = ctypes.c_size_t(ws.numel())
            N.check(N.hybrid_eval_multi_s(self.handle, 1 << k, _dptr(sd), N.PRECISIONS[precision], q.c(), *ptrs,
                                          _dptr(ls), ctypes.c_void_p(_dptr(ws)), have, st), "hybrid_eval_multi_s")
            return (out, ls) if log_scale else out
        N.check(N.hybrid_eval(self.handle, k, s, N.PRECISIONS[precision], q.c(), _dptr(out), _dptr(ls), None,
                              need, st), "hybrid_eval(size)")
        ws = self._ws(need.value, slot)
        have = ctypes.c_size_t(ws.numel())
        N.check(N.hybrid_eval(self.handle, k, s, N.PRECISIONS[precision], q.c(), _dptr(out), _dptr(ls),
                              ctypes.c_void_p(_dptr(ws)), have, st), "hybrid_eval")
        return (out, ls) if log_scale else out

    def hybrid_multi(self, xi, kernels=("fourier", "laplace", "bessel"), s: float = 1.0, precision: str = "fp32",
                     offsets=None, outs=None, log_scale_out=None, stream=None, slot: str = "main") -> dict:
        """Several kernels in one pass: {kernel: output} (outputs as hybrid())."""
        q = xi if isinstance(xi, QuerySet) else QuerySet(xi, offsets)
        q.validate(self.num_images, self.ndim)
        rows = q.rows(self.num_images)
        outs = dict(outs or {})
        mask = 0
        for k in kernels:
            mask |= 1 << N.KERNELS[k]
            if k not in outs:
                outs[k] = torch.empty((rows, 2) if k == "fourier" else (rows,), dtype=torch.float64,
                                      device=self.device)
        st = _stream(stream)
        ptrs = [_dptr(outs.get(k)) for k in ("fourier", "laplace", "bessel")]
        sd = _device_scale(s, self.device)
        fn, sv, name = ((N.hybrid_eval_multi_s, _dptr(sd), "hybrid_eval_multi_s") if sd is not None
                        else (N.hybrid_eval_multi, s, "hybrid_eval_multi"))
        need = ctypes.c_size_t(0)
        N.check(fn(self.handle, mask, sv, N.PRECISIONS[precision], q.c(), *ptrs, _dptr(log_scale_out), None, need,
                   st), name + "(size)")
        ws = self._ws(need.value, slot)
        have = ctypes.c_size_t(ws.numel())
        N.check(fn(self.handle, mask, sv, N.PRECISIONS[precision], q.c(), *ptrs, _dptr(log_scale_out),
                   ctypes.c_void_p(_dptr(ws)), have, st), name)
        return {k: outs[k] for k in kernels}

    def ect_hybrid_multi(self, dirs, thresholds: torch.Tensor, xi, kernels=("fourier", "laplace", "bessel"),
                         s: float = 1.0, precision: str = "fp32", dir_offsets=None, xi_offsets=None, ect_out=None,
                         outs=None, log_scale_out=None, stream=None, slot: str = "main"):
        """(ect, {kernel: output}): ect() and hybrid_multi() in one call (ect_hybrid_eval_multi); a shared
        direction set with small threshold arrays runs both in one launch.  Outputs equal the separate calls'."""
        qd = dirs if isinstance(dirs, QuerySet) else QuerySet(dirs, dir_offsets)
        qd.validate(self.num_images, self.ndim)
        qx = xi if isinstance(xi, QuerySet) else QuerySet(xi, xi_offsets)
        qx.validate(self.num_images, self.ndim)
        thr = thresholds.to(device=self.device, dtype=torch.float64).contiguous()
        per_image = 1 if thr.dim() == 2 else 0
        if thr.dim() not in (1, 2) or (per_image and thr.shape[0] != self.num_images):
            raise ValueError("thresholds must be [M] or [num_images][M]")
        M = thr.shape[-1]
        if ect_out is None:
            ect_out = torch.empty((qd.rows(self.num_images), M), dtype=torch.int32, device=self.device)
        rows = qx.rows(self.num_images)
        outs = dict(outs or {})
        mask = 0
        for k in kernels:
            mask |= 1 << N.KERNELS[k]
            if k not in outs:
                outs[k] = torch.empty((rows, 2) if k == "fourier" else (rows,), dtype=torch.float64,
                                      device=self.device)
        st = _stream(stream)
        ptrs = [_dptr(outs.get(k)) for k in ("fourier", "laplace", "bessel")]
        head = (self.handle, qd.c(), _dptr(thr), M, per_image, _dptr(ect_out), mask, s, N.PRECISIONS[precision],
                qx.c(), *ptrs, _dptr(log_scale_out))
        need = ctypes.c_size_t(0)
        N.check(N.ect_hybrid_eval_multi(*head, None, need, st), "ect_hybrid_eval_multi(size)")
        ws = self._ws(need.value, slot)
        have = ctypes.c_size_t(ws.numel())
        N.check(N.ect_hybrid_eval_multi(*head, ctypes.c_void_p(_dptr(ws)), have, st), "ect_hybrid_eval_multi")
        return ect_out, {k: outs[k] for k in kernels}

    def hybrid_backward(self, xi, out: torch.Tensor, grad_out: torch.Tensor, kernel: str = "fourier", s: float = 1.0,
                        precision: str = "fp32", offsets=None, stream=None, grad_xi=None, grad_s=None,
                        slot: str = "main", reuse_prepared: bool = False):
        """(grad_xi, grad_s): VJP of hybrid() (shared sets sum grad_xi over images).

        reuse_prepared: the last forward call on this plan used the same query
        set (same QuerySet object or tensors, unchanged) and workspace slot,
        on the same stream, so its bucketing is reused."""
        q = xi if isinstance(xi, QuerySet) else QuerySet(xi, offsets)
        q.validate(self.num_images, self.ndim)
        k = N.KERNELS[kernel]
        rows = q.rows(self.num_images)
        if out.shape[0] != rows or grad_out.shape != out.shape:
            raise ValueError("out and grad_out must have the forward output's shape")
        gxi = grad_xi if grad_xi is not None else torch.empty((q.vecs.shape[0], self.ndim), dtype=torch.float64,
                                                              device=self.device)
        gs = grad_s if grad_s is not None else torch.empty((), dtype=torch.float64, device=self.device)
        out = out.to(torch.float64).contiguous()
        go = grad_out.to(torch.float64).contiguous()
        st = _stream(stream)
        sd = _device_scale(s, self.device)
        fn, sv, name = ((N.hybrid_eval_backward_s, _dptr(sd), "hybrid_eval_backward_s") if sd is not None
                        else (N.hybrid_eval_backward, s, "hybrid_eval_backward"))
        need = ctypes.c_size_t(0)
        N.check(fn(self.handle, k, sv, N.PRECISIONS[precision], q.c(), _dptr(out), _dptr(go), _dptr(gxi), _dptr(gs),
                   None, need, st), name + "(size)")
        ws = self._ws(need.value, slot)
        have = ctypes.c_size_t(ws.numel())
        N.check(fn(self.handle, k, sv, N.PRECISIONS[precision], q.c(), _dptr(out), _dptr(go), _dptr(gxi), _dptr(gs),
                   ctypes.c_void_p(_dptr(ws)), have, st, N.BWD_REUSE_PREPARED if reuse_prepared else 0), name)
        return gxi, gs


class _nullctx:
    def __enter__(self):
        return self

    def __exit__(self, *exc):
        return False


class ExactRepresentation:
    """Device arrays written by ect_exact: row r starts at row_off[r]; ECT rows hold (T, E) of length
    length[r], Radon rows (T, E') of length length[r, 0] followed by (Tc, Ec) of length length[r, 1]."""

    def __init__(self, kind: int, row_off, T, E, length, capacity: int):
        self.kind, self.row_off, self.T, self.E, self.length, self.capacity = kind, row_off, T, E, length, capacity
        self.rows = row_off.shape[0] - 1

    def to_host(self):
        """Per-row numpy arrays: [(T, E)] or [(T, E', Tc, Ec)]."""
        off = self.row_off.cpu().numpy()
        T, E, L = self.T.cpu().numpy(), self.E.cpu().numpy(), self.length.cpu().numpy()
        out = []
        for r in range(self.rows):
            b = int(off[r])
            if self.kind == N.EXACT_ECT:
                n = int(L[r])
                out.append((T[b:b + n], E[b:b + n]))
            else:
                no, nc = int(L[r, 0]), int(L[r, 1])
                out.append((T[b:b + no], E[b:b + no], T[b + no:b + no + nc], E[b + no:b + no + nc]))
        return out

    def eval(self, thresholds: torch.Tensor, out=None, stream=None) -> torch.Tensor:
        """int32 [rows][M] by binary search (ect_exact_eval); thresholds [M] or [rows][M], any order."""
        thr = thresholds.to(device=self.T.device, dtype=torch.float64).contiguous()
        per_row = 1 if thr.dim() == 2 else 0
        if thr.dim() not in (1, 2) or (per_row and thr.shape[0] != self.rows):
            raise ValueError("thresholds must be [M] or [rows][M]")
        M = thr.shape[-1]
        if out is None:
            out = torch.empty((self.rows, M), dtype=torch.int32, device=self.T.device)
        N.check(N.ect_exact_eval(self.kind, self.rows, _dptr(self.row_off), _dptr(self.T), _dptr(self.E),
                                 _dptr(self.length), self.capacity, _dptr(thr), M, per_row, _dptr(out),
                                 _stream(stream)), "ect_exact_eval")
        return out


class HybridTransform(torch.autograd.Function):
    """y = HT_s(xi) for every image of a plan, differentiable in xi and in the scale s.

    xi: [count][ndim] shared by every image (float32 or float64; converted to
    float64 losslessly at the boundary).  s: a number, or a one-element tensor
    on the plan's device, which the kernels read from device memory (no host
    synchronisation, so a training step with a learnable scale can be
    captured into a HIP graph).  Returns float64 [num_images*count] (Fourier:
    [num_images*count][2]); the backward pass calls the library's
    vector-Jacobian product kernel.
    """

    @staticmethod
    def forward(ctx, xi, s, plan: Plan, kernel: str = "fourier", precision: str = "fp32"):
        xi64 = xi.detach().to(torch.float64).contiguous()
        ctx.s_is_tensor = torch.is_tensor(s)
        sarg = _device_scale(s, plan.device) if ctx.s_is_tensor else float(s)
        y = plan.hybrid(xi64, kernel, sarg, precision)
        ctx.plan, ctx.kernel, ctx.precision, ctx.sarg = plan, kernel, precision, sarg
        ctx.xi_dtype = xi.dtype
        ctx.s_dtype = s.dtype if ctx.s_is_tensor else None
        ctx.s_shape = s.shape if ctx.s_is_tensor else None
        ctx.save_for_backward(xi64, y)
        return y

    @staticmethod
    def backward(ctx, gy):
        xi64, y = ctx.saved_tensors
        gxi, gs = ctx.plan.hybrid_backward(xi64, y, gy.contiguous(), ctx.kernel, ctx.sarg, ctx.precision)
        return (gxi.to(ctx.xi_dtype), (gs.to(ctx.s_dtype).reshape(ctx.s_shape) if ctx.s_is_tensor else None), None,
                None, None)
