"""Error gates for floating-point parity against the FP64 oracle.

Hybrid transforms are sums of many terms of both signs that cancel heavily
(their condition number sum|term| / |sum| reaches 10^4 on binary fields), so
a plain per-query relative tolerance cannot describe FP32 arithmetic.  The FP32
gate per query is

    |y - y_ref| <= 1e-5 |y_ref| + 8 * 2^-24 * S2,     S2 = sqrt(sum_x |D(x) kbar_s(<xi,x>)|^2),

i.e. 1e-5 relative plus eight FP32 rounding units of the root-sum-square of
the terms (the size of the rounding error of an FP32 evaluation of every term
when the errors are independent); in addition the normwise error
max|y - y_ref| / max|y_ref| must stay below 1e-5.  The FP64 gate is
|y - y_ref| <= 1e-11 * S1 with S1 = sum_x |D(x) kbar_s(<xi,x>)|.

S1 and S2 come from the oracle's own critical values, never from the GPU.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O


def _vertex_coords(shape_np, construction, origin=None, spacing=None):
    dims = np.array(list(reversed(shape_np)))
    Nn = dims if construction == O.PRIMAL else dims - 1
    V = Nn + 1
    o = -0.5 * Nn if origin is None else np.asarray(origin, float)
    h = np.ones(len(V)) if spacing is None else np.asarray(spacing, float)
    ks = np.array(np.meshgrid(*[np.arange(v) for v in V], indexing="ij")).reshape(len(V), -1).T
    # linear vertex index with axis 0 fastest: sort by (k_{n-1}, ..., k_0)
    order = np.lexsort(ks.T)
    ks = ks[order]
    return ks * h + o


def term_scales(img, xi, kernel, s, construction=O.PRIMAL, origin=None, spacing=None, shift=None):
    """(S1, S2) per query from the oracle's ordinary critical values."""
    img = np.asarray(img)
    xi = np.asarray(xi, float).reshape(-1, img.ndim)
    _, od = O.critical_values(img, construction)
    x = _vertex_coords(img.shape, construction, origin, spacing)
    S1 = np.zeros(len(xi))
    S2 = np.zeros(len(xi))
    for q in range(len(xi)):
        e = sum(1 << a for a in range(img.ndim) if not (xi[q, a] >= 0))
        D = od[:, e]
        nz = np.nonzero(D)[0]
        u = x[nz] @ xi[q]
        z = s * u
        if kernel == "fourier":
            t = np.abs(D[nz]) / abs(s) * np.ones_like(z)
        elif kernel == "laplace":
            m = 0.0 if shift is None else shift[q]
            t = np.abs(D[nz]) * np.exp(-z - m) / abs(s)
        else:
            t = np.abs(D[nz] * O.ji0_array(z)) / abs(s)
        S1[q] = t.sum()
        S2[q] = np.sqrt((t * t).sum())
    return S1, S2


def fp32_gate(y, ref, S2, normwise=True):
    """Return (ok, worst ratio, normwise error, strict max relative error).

    normwise=False drops the set-wide criterion, for sets of a few queries
    whose largest value may itself be a cancellation to ~0."""
    y = np.asarray(y)
    ref = np.asarray(ref)
    err = np.abs(y - ref)
    tol = 1e-5 * np.abs(ref) + 8 * 2.0 ** -24 * S2
    ratio = float((err / np.maximum(tol, 1e-300)).max()) if err.size else 0.0
    norm = float(err.max() / max(np.abs(ref).max(), 1e-300)) if err.size else 0.0
    strict = float((err / np.maximum(np.abs(ref), 1e-300)).max()) if err.size else 0.0
    return ratio <= 1.0 and (norm <= 1e-5 or not normwise), ratio, norm, strict


def fp64_gate(y, ref, S1):
    err = np.abs(np.asarray(y) - np.asarray(ref))
    tol = 1e-11 * np.maximum(S1, 1e-300)
    ratio = float((err / tol).max()) if err.size else 0.0
    return ratio <= 1.0, ratio
