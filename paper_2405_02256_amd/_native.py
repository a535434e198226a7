"""ctypes binding of libect.so (argument marshalling only).

Every compute step runs in the HIP kernels of libect.so.  If the library is
missing this module raises: there is no CPU fallback on the product path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libect.so")

c_i32, c_i64, c_f64, c_u32, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint32, ctypes.c_void_p
P = ctypes.POINTER

ECT_OK, ECT_E_INVALID, ECT_E_NOMEM, ECT_E_DEVICE, ECT_E_UNSUPPORTED, ECT_E_RANGE, ECT_E_SCRATCH = range(7)
NOALLOC_SCRATCH_BYTES = 64 << 20
PRIMAL, DUAL = 0, 1
U8, I16, I32 = 0, 1, 2
FOURIER, LAPLACE, BESSEL = 0, 1, 2
FP32, FP64 = 0, 1
KERNELS = {"fourier": FOURIER, "laplace": LAPLACE, "bessel": BESSEL}
PRECISIONS = {"fp32": FP32, "fp64": FP64}

DEVERR_THRESHOLDS = 0x2
DEVERR_NONFINITE = 0x4
DEVERR_LOOKBACK = 0x8
DEVERR_OVERFLOW = 0x10
DEVERR_CAPACITY = 0x20
DEVERR_LAYOUT = 0x40
DEVERR_SCALE = 0x80
EXACT_ECT, EXACT_RADON = 0, 1
BWD_REUSE_PREPARED = 0x1


class ImageBatch(ctypes.Structure):
    _fields_ = [("ndim", c_i32), ("num_images", c_i32), ("dims", P(c_i32)), ("pixel_offsets", P(c_i64)),
                ("pixels", c_vp), ("dtype", c_i32), ("construction", c_i32), ("origin", P(c_f64)),
                ("spacing", P(c_f64))]


class QuerySet(ctypes.Structure):
    _fields_ = [("vecs", c_vp), ("offsets", c_vp), ("count", c_i64)]


class EctError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} (status {status})")


_lib = None


def lib():
    """Load libect.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2405_02256_amd.build` "
                           "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    L.ect_version.restype = ctypes.c_char_p
    L.ect_status_string.restype = ctypes.c_char_p
    L.ect_status_string.argtypes = [c_i32]
    L.ect_precompute.argtypes = [P(ImageBatch), c_vp, P(ctypes.c_size_t), c_vp, P(c_vp)]
    L.ect_plan_rerun.argtypes = [c_vp, c_vp]
    L.ect_plan_rerun_prepare.argtypes = [c_vp, QuerySet, c_vp, P(ctypes.c_size_t), c_vp]
    L.ect_eval.argtypes = [c_vp, QuerySet, c_vp, c_i32, c_i32, c_vp, c_vp, P(ctypes.c_size_t), c_vp]
    L.radon_eval.argtypes = [c_vp, QuerySet, c_vp, c_i32, c_i32, c_vp, c_vp, P(ctypes.c_size_t), c_vp]
    L.hybrid_eval.argtypes = [c_vp, c_i32, c_f64, c_i32, QuerySet, c_vp, c_vp, c_vp, P(ctypes.c_size_t), c_vp]
    L.hybrid_eval_noalloc.argtypes = [c_vp, c_i32, c_f64, c_i32, QuerySet, c_vp, c_vp, c_vp]
    L.hybrid_eval_multi.argtypes = [c_vp, c_u32, c_f64, c_i32, QuerySet, c_vp, c_vp, c_vp, c_vp, c_vp,
                                    P(ctypes.c_size_t), c_vp]
    L.ect_hybrid_eval_multi.argtypes = [c_vp, QuerySet, c_vp, c_i32, c_i32, c_vp, c_u32, c_f64, c_i32, QuerySet,
                                        c_vp, c_vp, c_vp, c_vp, c_vp, P(ctypes.c_size_t), c_vp]
    L.hybrid_eval_multi_s.argtypes = [c_vp, c_u32, c_vp, c_i32, QuerySet, c_vp, c_vp, c_vp, c_vp, c_vp,
                                      P(ctypes.c_size_t), c_vp]
    L.hybrid_eval_backward_s.argtypes = [c_vp, c_i32, c_vp, c_i32, QuerySet, c_vp, c_vp, c_vp, c_vp, c_u32,
                                         c_vp, P(ctypes.c_size_t), c_vp]
    L.hybrid_eval_backward.argtypes = [c_vp, c_i32, c_f64, c_i32, QuerySet, c_vp, c_vp, c_vp, c_vp, c_u32,
                                       c_vp, P(ctypes.c_size_t), c_vp]
    L.ect_plan_counts.argtypes = [c_vp, P(c_i64), P(c_i64)]
    L.ect_plan_export.argtypes = [c_vp, c_i32, c_i32, c_i32, P(c_i32), P(c_i32), c_i64, P(c_i64), c_vp]
    L.ect_plan_check.argtypes = [c_vp, P(c_u32), c_vp]
    L.ect_plan_destroy.argtypes = [c_vp]
    L.ect_plan_set_tuning.argtypes = [c_vp, c_i64, c_i64, c_i32, c_i32]
    L.ect_set_stage_events.argtypes = [c_i32, c_vp, c_vp]
    L.ect_exact_layout.argtypes = [c_vp, QuerySet, c_i32, c_vp, c_vp, P(ctypes.c_size_t), c_vp]
    L.ect_exact.argtypes = [c_vp, QuerySet, c_i32, c_vp, c_i64, c_vp, c_vp, c_vp, c_vp, P(ctypes.c_size_t), c_vp]
    L.ect_exact_eval.argtypes = [c_i32, c_i64, c_vp, c_vp, c_vp, c_vp, c_i64, c_vp, c_i32, c_i32, c_vp, c_vp]
    for name in ("ect_precompute", "ect_plan_rerun", "ect_plan_rerun_prepare", "ect_eval", "radon_eval", "hybrid_eval", "hybrid_eval_noalloc",
                 "hybrid_eval_multi", "hybrid_eval_multi_s", "hybrid_eval_backward_s",
                 "ect_hybrid_eval_multi", "hybrid_eval_backward", "ect_exact_layout", "ect_exact", "ect_exact_eval",
                 "ect_plan_counts", "ect_plan_export", "ect_plan_check", "ect_plan_destroy", "ect_plan_set_tuning",
                 "ect_set_stage_events"):
        getattr(L, name).restype = c_i32
    _lib = L
    return L


def status_string(status: int) -> str:
    return lib().ect_status_string(int(status)).decode()


def check(status: int, where: str) -> None:
    if status != ECT_OK:
        raise EctError(status, where)


def version() -> str:
    return lib().ect_version().decode()


# Thin same-name wrappers around the C entry points (raw pointers as ints).

def ect_precompute(batch: ImageBatch, ws, ws_bytes: ctypes.c_size_t, stream: int) -> int:
    plan = c_vp()
    st = lib().ect_precompute(ctypes.byref(batch), ws, ctypes.byref(ws_bytes), c_vp(stream), ctypes.byref(plan))
    return st, plan.value


def ect_plan_rerun(plan: int, stream: int) -> int:
    return lib().ect_plan_rerun(c_vp(plan), c_vp(stream))


def ect_eval(plan, dirs: QuerySet, thresholds, M, per_image, out, ws, ws_bytes: ctypes.c_size_t, stream) -> int:
    return lib().ect_eval(c_vp(plan), dirs, c_vp(thresholds), int(M), int(per_image), c_vp(out), ws,
                          ctypes.byref(ws_bytes), c_vp(stream))


def radon_eval(plan, dirs: QuerySet, thresholds, M, per_image, out, ws, ws_bytes: ctypes.c_size_t, stream) -> int:
    return lib().radon_eval(c_vp(plan), dirs, c_vp(thresholds), int(M), int(per_image), c_vp(out), ws,
                            ctypes.byref(ws_bytes), c_vp(stream))


def ect_exact_layout(plan, dirs: QuerySet, kind, row_off, ws, ws_bytes: ctypes.c_size_t, stream) -> int:
    return lib().ect_exact_layout(c_vp(plan), dirs, int(kind), c_vp(row_off), ws, ctypes.byref(ws_bytes),
                                  c_vp(stream))


def ect_exact(plan, dirs: QuerySet, kind, row_off, capacity, T, E, length, ws, ws_bytes: ctypes.c_size_t,
              stream) -> int:
    return lib().ect_exact(c_vp(plan), dirs, int(kind), c_vp(row_off), int(capacity), c_vp(T), c_vp(E),
                           c_vp(length), ws, ctypes.byref(ws_bytes), c_vp(stream))


def ect_exact_eval(kind, rows, row_off, T, E, length, capacity, thresholds, M, per_row, out, stream) -> int:
    return lib().ect_exact_eval(int(kind), int(rows), c_vp(row_off), c_vp(T), c_vp(E), c_vp(length),
                                int(capacity), c_vp(thresholds), int(M), int(per_row), c_vp(out), c_vp(stream))


def hybrid_eval(plan, kernel, s, precision, xi: QuerySet, out, log_scale, ws, ws_bytes: ctypes.c_size_t,
                stream) -> int:
    return lib().hybrid_eval(c_vp(plan), int(kernel), float(s), int(precision), xi, c_vp(out),
                             c_vp(log_scale) if log_scale else None, ws, ctypes.byref(ws_bytes), c_vp(stream))


def hybrid_eval_noalloc(plan, kernel, s, precision, xi: QuerySet, out, log_scale, stream) -> int:
    return lib().hybrid_eval_noalloc(c_vp(plan), int(kernel), float(s), int(precision), xi, c_vp(out),
                                     c_vp(log_scale) if log_scale else None, c_vp(stream))


def hybrid_eval_multi(plan, mask, s, precision, xi: QuerySet, out_f, out_l, out_b, log_scale, ws,
                      ws_bytes: ctypes.c_size_t, stream) -> int:
    return lib().hybrid_eval_multi(c_vp(plan), int(mask), float(s), int(precision), xi,
                                   c_vp(out_f) if out_f else None, c_vp(out_l) if out_l else None,
                                   c_vp(out_b) if out_b else None, c_vp(log_scale) if log_scale else None, ws,
                                   ctypes.byref(ws_bytes), c_vp(stream))


def hybrid_eval_multi_s(plan, mask, s_ptr, precision, xi: QuerySet, out_f, out_l, out_b, log_scale, ws,
                        ws_bytes: ctypes.c_size_t, stream) -> int:
    return lib().hybrid_eval_multi_s(c_vp(plan), int(mask), c_vp(s_ptr), int(precision), xi,
                                     c_vp(out_f) if out_f else None, c_vp(out_l) if out_l else None,
                                     c_vp(out_b) if out_b else None, c_vp(log_scale) if log_scale else None, ws,
                                     ctypes.byref(ws_bytes), c_vp(stream))


def hybrid_eval_backward_s(plan, kernel, s_ptr, precision, xi: QuerySet, out, grad_out, grad_xi, grad_s, ws,
                           ws_bytes: ctypes.c_size_t, stream, flags: int = 0) -> int:
    return lib().hybrid_eval_backward_s(c_vp(plan), int(kernel), c_vp(s_ptr), int(precision), xi, c_vp(out),
                                        c_vp(grad_out), c_vp(grad_xi), c_vp(grad_s) if grad_s else None, int(flags),
                                        ws, ctypes.byref(ws_bytes), c_vp(stream))


def ect_plan_rerun_prepare(plan, xi: QuerySet, ws, ws_bytes: ctypes.c_size_t, stream) -> int:
    return lib().ect_plan_rerun_prepare(c_vp(plan), xi, ws, ctypes.byref(ws_bytes), c_vp(stream))


def ect_hybrid_eval_multi(plan, dirs: QuerySet, thresholds, M, per_image, ect_out, mask, s, precision,
                          xi: QuerySet, out_f, out_l, out_b, log_scale, ws, ws_bytes: ctypes.c_size_t, stream) -> int:
    return lib().ect_hybrid_eval_multi(c_vp(plan), dirs, c_vp(thresholds), int(M), int(per_image), c_vp(ect_out),
                                       int(mask), float(s), int(precision), xi,
                                       c_vp(out_f) if out_f else None, c_vp(out_l) if out_l else None,
                                       c_vp(out_b) if out_b else None, c_vp(log_scale) if log_scale else None, ws,
                                       ctypes.byref(ws_bytes), c_vp(stream))


def hybrid_eval_backward(plan, kernel, s, precision, xi: QuerySet, out, grad_out, grad_xi, grad_s, ws,
                         ws_bytes: ctypes.c_size_t, stream, flags: int = 0) -> int:
    return lib().hybrid_eval_backward(c_vp(plan), int(kernel), float(s), int(precision), xi, c_vp(out),
                                      c_vp(grad_out), c_vp(grad_xi), c_vp(grad_s) if grad_s else None,
                                      int(flags), ws, ctypes.byref(ws_bytes), c_vp(stream))


def ect_plan_counts(plan, classical, ordinary) -> int:
    return lib().ect_plan_counts(c_vp(plan), classical, ordinary)


def ect_plan_export(plan, image, kind, lst, coords, values, capacity, count, stream) -> int:
    return lib().ect_plan_export(c_vp(plan), int(image), int(kind), int(lst), coords, values, int(capacity),
                                 count, c_vp(stream))


def ect_plan_check(plan, flags, stream) -> int:
    return lib().ect_plan_check(c_vp(plan), flags, c_vp(stream))


def ect_plan_destroy(plan) -> int:
    return lib().ect_plan_destroy(c_vp(plan))


def ect_plan_set_tuning(plan, hybrid_chunk: int, hybrid_target_items: int, ect_dirs_per_group: int,
                        ect_chunks: int = 0) -> int:
    return lib().ect_plan_set_tuning(c_vp(plan), int(hybrid_chunk), int(hybrid_target_items),
                                     int(ect_dirs_per_group), int(ect_chunks))


STAGE_PRECOMPUTE, STAGE_ECT, STAGE_HYBRID, STAGE_HYBRID_BWD = 0, 1, 2, 3


def ect_set_stage_events(stage: int, before, after) -> int:
    """before/after: raw hipEvent_t handles (ints) or None."""
    return lib().ect_set_stage_events(int(stage), c_vp(before) if before else None, c_vp(after) if after else None)
