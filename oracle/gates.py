"""Error gates for floating-point parity against the FP64 oracle.  TEST INFRASTRUCTURE ONLY
(used by the tests and by the cpu_baseline leg of bench.py, like the oracle itself).

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

Laplace values reach e^(+-900) on the large-phase workloads, so they are
gated in shifted form: both sides are brought to the oracle's shift m_ref
(HT e^-m_ref) and S2 is taken over the shifted terms.

Gradients use the same gate per query AND per component: for dHT/dxi_a the
terms are D x_a kappa(s u) paired with the cotangent, so a wrong small
component cannot hide under a large one; the d/ds contribution propagates
the component scales and the forward output's scale through its formula.

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


def _rss(t):
    """Root sum of squares without overflow (terms scaled by their largest)."""
    t = np.abs(np.asarray(t, float))
    if t.size == 0:
        return 0.0
    m = t.max()
    if m == 0.0 or not np.isfinite(m):
        return float(m)
    return float(m * np.sqrt(((t / m) ** 2).sum()))


class _Lists:
    """The oracle's ordinary lists (D, coordinates) per sign vector, built once per image."""

    def __init__(self, img, construction, origin, spacing):
        self.n = img.ndim
        _, self.od = O.critical_values(img, construction)
        self.x = _vertex_coords(img.shape, construction, origin, spacing)
        self.cache = {}

    def __call__(self, xi_q):
        e = sum(1 << a for a in range(self.n) if not (xi_q[a] >= 0))
        if e not in self.cache:
            D = self.od[:, e]
            nz = np.nonzero(D)[0]
            self.cache[e] = (D[nz].astype(float), self.x[nz])
        return self.cache[e]


def _bessel_envelope(z):
    """|J0(z)| <= min(1, sqrt(2 / (pi |z|))): the size of J0 that an FP32
    evaluation's absolute error scales with."""
    az = np.abs(z)
    return np.minimum(1.0, np.sqrt(2.0 / (np.pi * np.maximum(az, 1e-300))))


def _forward_terms(kernel, D, z, s, m=0.0):
    if kernel == "fourier":
        return np.abs(D) / abs(s) * np.ones_like(z)
    if kernel == "laplace":
        return np.abs(D) * np.exp(-z - m) / abs(s)
    return np.abs(D * O.ji0_array(z)) / abs(s)


def term_scales(img, xi, kernel, s, construction=O.PRIMAL, origin=None, spacing=None, shift=None):
    """(S1, S2) per query from the oracle's ordinary critical values.

    Laplace with shift m: the terms of HT * exp(-m), i.e. the scale of the
    oracle's shifted output."""
    img = np.asarray(img)
    xi = np.asarray(xi, float).reshape(-1, img.ndim)
    lists = _Lists(img, construction, origin, spacing)
    S1 = np.zeros(len(xi))
    S2 = np.zeros(len(xi))
    for q in range(len(xi)):
        D, xs = lists(xi[q])
        z = s * (xs @ xi[q])
        t = _forward_terms(kernel, D, z, s, 0.0 if shift is None else shift[q])
        S1[q] = t.sum()
        S2[q] = _rss(t)
    return S1, S2


def grad_scales(img, xi, kernel, s, gout, construction=O.PRIMAL, origin=None, spacing=None):
    """Error scales of the backward pass at each query, from the oracle's critical values.

    Returns (S2x [q][n], S1x [q][n], S2s [q], S1s [q]): per component a the
    root sum of squares (and sum) of the terms |D x_a kappa(s u) g| of
    dHT/dxi_a paired with the cotangent g, and for the d/ds contribution of
    the query (sum_a xi_a G_a - <g, HT>) / s the same scales propagated
    through that expression (the forward output's own term scale included)."""
    img = np.asarray(img)
    n = img.ndim
    xi = np.asarray(xi, float).reshape(-1, n)
    g = np.asarray(gout)
    if kernel == "fourier":
        g = g.reshape(len(xi), 2)
        gm = np.abs(g[:, 0]) + np.abs(g[:, 1])
    else:
        gm = np.abs(g.reshape(len(xi)))
    lists = _Lists(img, construction, origin, spacing)
    S2x = np.zeros((len(xi), n))
    S1x = np.zeros((len(xi), n))
    S2s = np.zeros(len(xi))
    S1s = np.zeros(len(xi))
    for q in range(len(xi)):
        D, xs = lists(xi[q])
        z = s * (xs @ xi[q])
        if kernel == "fourier":
            k = np.ones_like(z)
        elif kernel == "laplace":
            k = np.exp(-z)
        else:
            k = _bessel_envelope(z)
        base = np.abs(D) * k * gm[q]
        for a in range(n):
            t = base * np.abs(xs[:, a])
            S2x[q, a] = _rss(t)
            S1x[q, a] = t.sum()
        fwd = _forward_terms(kernel, D, z, s) * gm[q]
        S2s[q] = (np.abs(xi[q]) @ S2x[q] + _rss(fwd)) / abs(s)
        S1s[q] = (np.abs(xi[q]) @ S1x[q] + fwd.sum()) / abs(s)
    return S2x, S1x, S2s, S1s


def fp32_gate(y, ref, S2, normwise=True):
    """Return (ok, worst ratio, normwise error, strict max relative error).

    normwise=False drops the set-wide criterion, for sets of a few queries
    whose largest value may itself be a cancellation to ~0."""
    y = np.asarray(y)
    ref = np.asarray(ref)
    err = np.abs(y - ref)
    tol = 1e-5 * np.abs(ref) + 8 * 2.0 ** -24 * np.asarray(S2)
    ratio = float((err / np.maximum(tol, 1e-300)).max()) if err.size else 0.0
    norm = float(err.max() / max(np.abs(ref).max(), 1e-300)) if err.size else 0.0
    strict = float((err / np.maximum(np.abs(ref), 1e-300)).max()) if err.size else 0.0
    return ratio <= 1.0 and (norm <= 1e-5 or not normwise), ratio, norm, strict


def fp64_gate(y, ref, S1):
    err = np.abs(np.asarray(y) - np.asarray(ref))
    tol = 1e-11 * np.maximum(np.asarray(S1), 1e-300)
    ratio = float((err / tol).max()) if err.size else 0.0
    return ratio <= 1.0, ratio


def combine_rss(*scales):
    """Scales of sums over independent parts (e.g. images sharing a query set)."""
    return np.sqrt(sum(np.asarray(a, float) ** 2 for a in scales))


def laplace_shifted(img, xi, s, construction=O.PRIMAL, origin=None, spacing=None):
    """(HT e^-m_ref, m_ref, S2 of the shifted terms) from the oracle."""
    ref, m = O.hybrid(img, xi, "laplace", s, construction, origin=origin, spacing=spacing, with_shift=True)
    _, S2 = term_scales(img, xi, "laplace", s, construction, origin, spacing, shift=m)
    return ref, m, S2


def grad_gate(g, ref, S2, normwise=True):
    """fp32_gate applied to every (query, component) of a gradient."""
    return fp32_gate(np.asarray(g).ravel(), np.asarray(ref).ravel(), np.asarray(S2).ravel(), normwise)


def g9_stats(y, ref, S2, S1=None) -> dict:
    """Error statistics of a set of results against the oracle: the worst ratio
    to the per-query gate (<= 1 passes), the normwise error
    max|err| / max|ref|, the strict per-query relative error and, with S1,
    the largest condition number S1 / |ref| of the set."""
    y = np.asarray(y).ravel()
    ref = np.asarray(ref).ravel()
    S2 = np.asarray(S2, float).ravel()
    ok, ratio, norm, strict = fp32_gate(y, ref, S2)
    out = {"checked": int(y.size), "max_gate_ratio": ratio, "normwise": norm, "strict_rel_max": strict,
           "pass": bool(ok)}
    if S1 is not None:
        out["cond_max"] = float((np.asarray(S1, float).ravel() / np.maximum(np.abs(ref), 1e-300)).max())
    return out
