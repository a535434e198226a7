"""C-ABI boundary checks that need no GPU: the library loads, exports every
entry point that include/ect.h declares, and rejects malformed arguments on
the host before touching the device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ect.h")


@pytest.fixture(scope="module")
def N():
    from paper_2405_02256_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        from paper_2405_02256_amd import build
        build.build(verbose=False)
    _native.lib()
    return _native


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", src, flags=re.M)))


def test_header_declares_the_four_calls():
    names = declared_functions()
    for n in ("ect_precompute", "ect_eval", "hybrid_eval", "hybrid_eval_backward"):
        assert n in names


def test_library_exports_every_declared_symbol(N):
    out = subprocess.run(["nm", "-D", "--defined-only", N.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    # nothing but the C ABI is exported
    extra = sorted(exported - set(declared_functions()))
    assert not extra, extra


def test_status_strings_and_version(N):
    assert N.version() == "0.1.0"
    for st in range(7):
        assert N.status_string(st)
    assert N.status_string(99) == "unknown status"


def _batch(N, ndim=2, dims=((4, 5),), dtype=0, cons=0, pixels=0x1000):
    d = np.array(dims, np.int32)
    offs = np.zeros(len(dims), np.int64)
    b = N.ImageBatch(ndim, len(dims), d.ctypes.data_as(N.P(N.c_i32)), offs.ctypes.data_as(N.P(N.c_i64)),
                     pixels, dtype, cons, None, None)
    return b, (d, offs)


def test_precompute_size_query_and_validation(N):
    b, keep = _batch(N)
    need = ctypes.c_size_t(0)
    st, plan = N.ect_precompute(b, None, need, 0)
    assert st == N.ECT_OK and plan is None and need.value > 0
    # larger images need more
    b2, keep2 = _batch(N, dims=((40, 50),))
    need2 = ctypes.c_size_t(0)
    assert N.ect_precompute(b2, None, need2, 0)[0] == N.ECT_OK and need2.value > need.value
    # four axes are accepted (16 classical + 8 ordinary lists of 8-byte entries)
    b4, keep4 = _batch(N, ndim=4, dims=((3, 4, 2, 5),))
    need4 = ctypes.c_size_t(0)
    assert N.ect_precompute(b4, None, need4, 0)[0] == N.ECT_OK and need4.value > 24 * 8 * (4 * 5 * 3 * 6)
    # the packed vertex index needs 3 x 11 bits for 1025^3 vertices: refused
    b5, keep5 = _batch(N, ndim=3, dims=((1024, 1024, 1024),))
    assert N.ect_precompute(b5, None, ctypes.c_size_t(0), 0)[0] == N.ECT_E_UNSUPPORTED
    # 1023^3 pixels (1024^3 vertices) fit in 30 bits
    b6, keep6 = _batch(N, ndim=3, dims=((1023, 1023, 1023),))
    assert N.ect_precompute(b6, None, ctypes.c_size_t(0), 0)[0] == N.ECT_OK
    for kw in (dict(ndim=5, dims=((2, 2, 2, 2, 2),)), dict(ndim=1, dims=((3,),)), dict(dims=((0, 5),)),
               dict(dtype=7), dict(cons=3), dict(pixels=0)):
        bb, k = _batch(N, **kw)
        assert N.ect_precompute(bb, None, ctypes.c_size_t(0), 0)[0] == N.ECT_E_INVALID, kw
    # workspace too small
    small = ctypes.c_size_t(need.value - 1)
    assert N.ect_precompute(b, ctypes.c_void_p(0x100000), small, 0)[0] == N.ECT_E_NOMEM
    # misaligned workspace
    assert N.ect_precompute(b, ctypes.c_void_p(0x100001), ctypes.c_size_t(need.value), 0)[0] == N.ECT_E_INVALID


def test_eval_calls_reject_null_plan(N):
    q = N.QuerySet(0x1000, None, 4)
    need = ctypes.c_size_t(0)
    assert N.ect_eval(None, q, 0x2000, 4, 0, 0x3000, None, need, 0) == N.ECT_E_INVALID
    assert N.radon_eval(None, q, 0x2000, 4, 0, 0x3000, None, need, 0) == N.ECT_E_INVALID
    assert N.hybrid_eval(None, 0, 1.0, 0, q, 0x3000, 0, None, need, 0) == N.ECT_E_INVALID
    assert N.hybrid_eval_backward(None, 0, 1.0, 0, q, 1, 2, 3, 0, None, need, 0) == N.ECT_E_INVALID
    assert N.hybrid_eval_noalloc(None, 0, 1.0, 0, q, 0x3000, 0, 0) == N.ECT_E_INVALID
    assert N.ect_exact_layout(None, q, 0, 0x4000, None, need, 0) == N.ECT_E_INVALID
    assert N.ect_exact(None, q, 0, 0x4000, 16, 0x5000, 0x6000, 0x7000, None, need, 0) == N.ECT_E_INVALID
    assert N.ect_hybrid_eval_multi(None, q, 0x2000, 4, 0, 0x3000, 1, 1.0, 0, q, 0x4000, 0, 0, 0, None, need,
                                   0) == N.ECT_E_INVALID
    assert N.ect_plan_rerun_prepare(None, q, None, need, 0) == N.ECT_E_INVALID
    assert N.ect_plan_destroy(None) == N.ECT_E_INVALID
    assert N.ect_plan_rerun(None, 0) == N.ECT_E_INVALID


def test_exact_eval_validation(N):
    """Host checks of ect_exact_eval (no plan involved): bad kind, sizes and null pointers are
    rejected before any launch; zero rows is a no-op."""
    args = dict(rows=3, row_off=0x1000, T=0x2000, E=0x3000, length=0x4000, capacity=64, thresholds=0x5000, M=4,
                per_row=0, out=0x6000, stream=0)

    def call(**kw):
        a = dict(args, **kw)
        return N.ect_exact_eval(a.pop("kind", 0), **a)

    assert call(kind=2) == N.ECT_E_INVALID
    assert call(M=0) == N.ECT_E_INVALID
    assert call(rows=-1) == N.ECT_E_INVALID
    assert call(capacity=-1) == N.ECT_E_INVALID
    assert call(T=0) == N.ECT_E_INVALID
    assert call(rows=0, T=0, E=0) == N.ECT_OK


def test_tuning_validation(N):
    assert N.ect_plan_set_tuning(None, 0, 2048, 0, 0) == N.ECT_E_INVALID


def test_product_path_refuses_without_library(tmp_path, monkeypatch):
    from paper_2405_02256_amd import _native
    monkeypatch.setattr(_native, "_lib", None)
    monkeypatch.setattr(_native, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _native.lib()
