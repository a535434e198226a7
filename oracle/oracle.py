"""Python face of the FP64 CPU oracle.  TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  It shares no code with the GPU library:
the heavy definitions live in ``oracle.c`` (built here with gcc), and a few
literal small-case forms are written out below in plain numpy/Python loops.

Functions and the definitions they follow:

* ``cell_values``          weighted cubical complex from an image (Sec. 4.1 for
                           the primal rule, Sec. 5 for the dual rule).
* ``euler_characteristic`` chi = sum (-1)^dim phi (Sec. 2.1).
* ``ect``                  ECT(xi,t) = chi(phi restricted to {xi <= t}) (Sec. 2.2),
                           over every cell.
* ``ect_literal``          the same sum evaluated threshold by threshold (tiny).
* ``hybrid``               HT(xi) = integral kappa R dt in its cell form (Sec. 2.2
                           with Lemma A.1).
* ``hybrid_integral``      HT as the literal integral of kappa against the Radon
                           transform, the latter read off the ECT (tiny inputs).
* ``hybrid_grad``          analytic derivative of the cell form in xi and s.
* ``critical_values``      lower/upper-star Euler characteristics (Sec. 3).
* ``critical_values_literal``  the same from the definition of the lower star
                           (cells whose maximum of a generic xi of the given sign
                           vector is attained at the vertex), tiny inputs.
* ``ji0``                  integral_0^z J0(t) dt by Gauss-Legendre panels.

Images have 1 to 4 axes (n-dimensional arrays, Sec. 4.1; all 2^n sign vectors,
Sec. 4.2).

Status: every function is pinned by the CPU tests in ``tests/test_oracle_*.py``
against closed forms, the worked example of Appendix A, invariants and brute
force on tiny inputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.c")

PRIMAL, DUAL = 0, 1
KERNELS = {"fourier": 0, "laplace": 1, "bessel": 2}


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (no contraction of a*b+c into fma)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", tmp, SRC_PATH, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
            build(force=True)
        L = ctypes.CDLL(LIB_PATH)
        i32p = ctypes.POINTER(ctypes.c_int32)
        f64p = ctypes.POINTER(ctypes.c_double)
        L.oracle_cell_values.argtypes = [ctypes.c_int, i32p, i32p, ctypes.c_int, i32p]
        L.oracle_euler_characteristic.argtypes = [ctypes.c_int, i32p, i32p, ctypes.c_int]
        L.oracle_euler_characteristic.restype = ctypes.c_longlong
        L.oracle_ect.argtypes = [ctypes.c_int, i32p, i32p, ctypes.c_int, f64p, f64p,
                                 ctypes.c_int, f64p, ctypes.c_int, f64p, i32p]
        L.oracle_hybrid.argtypes = [ctypes.c_int, i32p, i32p, ctypes.c_int, f64p, f64p,
                                    ctypes.c_int, f64p, ctypes.c_int, ctypes.c_double, f64p, f64p]
        L.oracle_hybrid_grad.argtypes = [ctypes.c_int, i32p, i32p, ctypes.c_int, f64p, f64p,
                                         ctypes.c_int, f64p, ctypes.c_int, ctypes.c_double,
                                         f64p, f64p, f64p]
        L.oracle_critical_values.argtypes = [ctypes.c_int, i32p, i32p, ctypes.c_int, i32p, i32p]
        L.oracle_ji0.argtypes = [ctypes.c_double]
        L.oracle_ji0.restype = ctypes.c_double
        L.oracle_ji0_array.argtypes = [ctypes.c_longlong, f64p, f64p]
        L.oracle_max_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _dims(img):
    """Embedding-axis extents of a numpy image (axis 0 = numpy's last index)."""
    return np.array(list(reversed(img.shape)), dtype=np.int32)


def grid_shape(img, construction):
    """numpy shape of the cell grid (2N_a+1 per axis, numpy order)."""
    d = _dims(img)
    N = d if construction == PRIMAL else d - 1
    return tuple(int(x) for x in reversed(2 * N + 1))


def vertex_shape(img, construction):
    d = _dims(img)
    N = d if construction == PRIMAL else d - 1
    return tuple(int(x) for x in reversed(N + 1))


def default_origin(img, construction):
    d = _dims(img).astype(np.float64)
    N = d if construction == PRIMAL else d - 1
    return -0.5 * N


def set_threads(t: int) -> None:
    lib().oracle_set_threads(int(t))


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def cell_values(img, construction=PRIMAL) -> np.ndarray:
    img = np.asarray(img)
    dims, dp = _i32(_dims(img))
    px, pp = _i32(img)
    out = np.zeros(grid_shape(img, construction), dtype=np.int32)
    rc = lib().oracle_cell_values(img.ndim, dp, pp, construction,
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc:
        raise ValueError(f"oracle_cell_values failed ({rc})")
    return out


def euler_characteristic(img, construction=PRIMAL) -> int:
    img = np.asarray(img)
    dims, dp = _i32(_dims(img))
    px, pp = _i32(img)
    return int(lib().oracle_euler_characteristic(img.ndim, dp, pp, construction))


def ect(img, dirs, thresholds, construction=PRIMAL, origin=None, spacing=None) -> np.ndarray:
    img = np.asarray(img)
    n = img.ndim
    dims, dp = _i32(_dims(img))
    px, pp = _i32(img)
    dirs, dirp = _f64(np.asarray(dirs, dtype=np.float64).reshape(-1, n))
    thr, tp = _f64(thresholds)
    org, op = _f64(origin)
    spc, sp = _f64(spacing)
    out = np.zeros((dirs.shape[0], thr.shape[0]), dtype=np.int32)
    rc = lib().oracle_ect(n, dp, pp, construction, op, sp, dirs.shape[0], dirp, thr.shape[0], tp,
                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc:
        raise ValueError(f"oracle_ect failed ({rc})")
    return out


def radon(img, dirs, thresholds, construction=PRIMAL, origin=None, spacing=None) -> np.ndarray:
    """R(xi, t) = chi of the slice {<xi,.> = t} from the cells (Sec. 2.2), int32 [dirs][thresholds]."""
    img = np.asarray(img)
    n = img.ndim
    dims, dp = _i32(_dims(img))
    px, pp = _i32(img)
    dirs, dirp = _f64(np.asarray(dirs, dtype=np.float64).reshape(-1, n))
    thr, tp = _f64(thresholds)
    org, op = _f64(origin)
    spc, sp = _f64(spacing)
    out = np.zeros((dirs.shape[0], thr.shape[0]), dtype=np.int32)
    rc = lib().oracle_radon(n, dp, pp, construction, op, sp, dirs.shape[0], dirp, thr.shape[0], tp,
                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc:
        raise ValueError(f"oracle_radon failed ({rc})")
    return out


def vertex_projections(img, xi, construction=PRIMAL, origin=None, spacing=None) -> np.ndarray:
    """Canonical FP64 projections of every vertex on xi, in linear vertex order."""
    img = np.asarray(img)
    n = img.ndim
    dims, dp = _i32(_dims(img))
    xi, xp = _f64(np.asarray(xi, dtype=np.float64).reshape(n))
    org, op = _f64(origin)
    spc, sp = _f64(spacing)
    nv = int(np.prod(vertex_shape(img, construction)))
    out = np.zeros(nv, dtype=np.float64)
    rc = lib().oracle_vertex_projections(n, dp, construction, op, sp, xp,
                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc:
        raise ValueError(f"oracle_vertex_projections failed ({rc})")
    return out


def _sign_index(xi):
    return sum(1 << a for a in range(len(xi)) if not (xi[a] >= 0.0))


def _sorted_jumps(u, vals):
    """Distinct values of u in ascending order and the sum of vals at each."""
    order = np.argsort(u, kind="stable")
    us, vs = u[order], vals[order].astype(np.int64)
    if us.size == 0:
        return us, vs
    head = np.ones(us.size, dtype=bool)
    head[1:] = us[1:] != us[:-1]
    starts = np.nonzero(head)[0]
    return us[starts], np.add.reduceat(vs, starts)


def ect_exact(img, xi, construction=PRIMAL, origin=None, spacing=None):
    """Exact ECT(xi, .) as (T, E) (Sec. 4.3): T = [-inf] + the sorted distinct projections of the
    classical critical points of eps(xi), E = [0] + the cumulative sums of their critical values
    (equal projections merged), so that ECT(xi, t) = E[i] for the largest T[i] <= t."""
    xi = np.asarray(xi, dtype=np.float64)
    lw, _ = critical_values(img, construction)
    D = lw[:, _sign_index(xi)]
    nz = np.nonzero(D)[0]
    u = vertex_projections(img, xi, construction, origin, spacing)[nz]
    t, v = _sorted_jumps(u, D[nz])
    return np.concatenate([[-np.inf], t]), np.concatenate([[0], np.cumsum(v)]).astype(np.int64)


def radon_exact(img, xi, construction=PRIMAL, origin=None, spacing=None):
    """Exact R(xi, .) as (T, E', Tc, Ec) (Sec. 4.3) with the sign the definition gives:
    R = sum over classical points of Delta^- 1_{u} - sum over ordinary points of D 1_(u, inf).
    T, E': [-inf] + sorted distinct ordinary projections and the cumulative sums of -D;
    Tc: sorted distinct classical projections; Ec[i] = E'[i0] + the classical values at Tc[i],
    with i0 the largest index such that T[i0] < Tc[i] (the open interval excludes u itself)."""
    xi = np.asarray(xi, dtype=np.float64)
    lw, od = critical_values(img, construction)
    e = _sign_index(xi)
    u_all = vertex_projections(img, xi, construction, origin, spacing)
    Do = od[:, e]
    nzo = np.nonzero(Do)[0]
    to, vo = _sorted_jumps(u_all[nzo], -Do[nzo])
    T = np.concatenate([[-np.inf], to])
    Ep = np.concatenate([[0], np.cumsum(vo)]).astype(np.int64)
    Dc = lw[:, e]
    nzc = np.nonzero(Dc)[0]
    tc, vc = _sorted_jumps(u_all[nzc], Dc[nzc])
    i0 = np.searchsorted(T, tc, side="left") - 1
    Ec = Ep[i0] + vc
    return T, Ep, tc, Ec.astype(np.int64)


def eval_ect_exact(T, E, t):
    """ECT(xi, t) = E[i] for the largest i with T[i] <= t (binary search)."""
    return E[np.searchsorted(T, np.asarray(t, dtype=np.float64), side="right") - 1]


def eval_radon_exact(T, Ep, Tc, Ec, t):
    """R(xi, t): Ec at a classical projection, else E'[i] for the largest i with T[i] < t."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    out = Ep[np.searchsorted(T, t, side="left") - 1].copy()
    k = np.searchsorted(Tc, t, side="left")
    hit = (k < Tc.size) & (Tc[np.minimum(k, max(Tc.size - 1, 0))] == t) if Tc.size else np.zeros(t.size, bool)
    out[hit] = Ec[k[hit]]
    return out


def hybrid(img, xi, kernel, s=1.0, construction=PRIMAL, origin=None, spacing=None,
           with_shift=False):
    """HT at each xi.  Fourier returns complex; Laplace with_shift returns (HT*exp(-m), m)."""
    img = np.asarray(img)
    n = img.ndim
    dims, dp = _i32(_dims(img))
    px, pp = _i32(img)
    xi, xp = _f64(np.asarray(xi, dtype=np.float64).reshape(-1, n))
    org, op = _f64(origin)
    spc, sp = _f64(spacing)
    k = KERNELS[kernel]
    q = xi.shape[0]
    out = np.zeros((q, 2) if k == 0 else (q,), dtype=np.float64)
    shift = np.zeros(q, dtype=np.float64) if with_shift else None
    rc = lib().oracle_hybrid(n, dp, pp, construction, op, sp, q, xp, k, float(s),
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             shift.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if with_shift else None)
    if rc:
        raise ValueError(f"oracle_hybrid failed ({rc})")
    if k == 0:
        out = out[:, 0] + 1j * out[:, 1]
    if with_shift:
        return out, shift
    return out


def hybrid_grad(img, xi, kernel, s, gout, construction=PRIMAL, origin=None, spacing=None):
    """(grad_xi [q][n], grad_s) of sum_q <gout_q, HT(xi_q)> (real pairing, Fourier as (Re, Im))."""
    img = np.asarray(img)
    n = img.ndim
    dims, dp = _i32(_dims(img))
    px, pp = _i32(img)
    xi, xp = _f64(np.asarray(xi, dtype=np.float64).reshape(-1, n))
    org, op = _f64(origin)
    spc, sp = _f64(spacing)
    k = KERNELS[kernel]
    q = xi.shape[0]
    g = np.asarray(gout)
    if k == 0 and np.iscomplexobj(g):
        g = np.stack([g.real, g.imag], axis=-1)
    g, gp = _f64(g.reshape(q, 2) if k == 0 else g.reshape(q))
    gxi = np.zeros((q, n), dtype=np.float64)
    gs = ctypes.c_double(0.0)
    rc = lib().oracle_hybrid_grad(n, dp, pp, construction, op, sp, q, xp, k, float(s), gp,
                                  gxi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  ctypes.byref(gs))
    if rc:
        raise ValueError(f"oracle_hybrid_grad failed ({rc})")
    return gxi, gs.value


def critical_values(img, construction=PRIMAL):
    """(lower[v][e], ordinary[v][e]) over vertices in linear order (axis 0 fastest).

    Sign-vector index e: bit a set means eps_a = -1.
    """
    img = np.asarray(img)
    n = img.ndim
    dims, dp = _i32(_dims(img))
    px, pp = _i32(img)
    nv = int(np.prod(vertex_shape(img, construction)))
    lw = np.zeros((nv, 1 << n), dtype=np.int32)
    od = np.zeros((nv, 1 << n), dtype=np.int32)
    rc = lib().oracle_critical_values(n, dp, pp, construction,
                                      lw.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      od.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc:
        raise ValueError(f"oracle_critical_values failed ({rc})")
    return lw, od


def critical_lists(img, construction=PRIMAL):
    """Per sign vector e: (classical {vertex: value}, ordinary {vertex: value}), zeros dropped."""
    lw, od = critical_values(img, construction)
    out = []
    for e in range(lw.shape[1]):
        c = {int(v): int(lw[v, e]) for v in np.nonzero(lw[:, e])[0]}
        o = {int(v): int(od[v, e]) for v in np.nonzero(od[:, e])[0]}
        out.append((c, o))
    return out


def ji0(z: float) -> float:
    return float(lib().oracle_ji0(float(z)))


def ji0_array(z) -> np.ndarray:
    z, zp = _f64(np.asarray(z, dtype=np.float64).reshape(-1))
    out = np.zeros_like(z)
    lib().oracle_ji0_array(z.size, zp, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


# ---------------------------------------------------------------------------
# Literal small-case forms (pure Python / numpy loops)
# ---------------------------------------------------------------------------

def _cells_literal(img, construction):
    """Yield (coords tuple in axis order, dim, value, list of vertex coords k) for every cell."""
    phi = cell_values(img, construction)
    n = img.ndim
    it = np.ndindex(*reversed(phi.shape))
    for c in it:  # c in embedding-axis order
        val = int(phi[tuple(reversed(c))])
        dim = sum(x & 1 for x in c)
        ranges = [((x - 1) // 2, (x + 1) // 2) if x & 1 else (x // 2,) for x in c]
        verts = [tuple(v) for v in np.array(np.meshgrid(*ranges, indexing="ij")).reshape(n, -1).T]
        yield c, dim, val, verts


def _project(xi, x):
    """Canonical projection fma(xi_{n-1}, x_{n-1}, ... fma(xi_1, x_1, xi_0*x_0))."""
    u = float(xi[0]) * float(x[0])
    for a in range(1, len(x)):
        u = _fma(float(xi[a]), float(x[a]), u)
    return u


def _fma(a, b, c):
    """Correctly rounded a*b+c in FP64 via exact rational arithmetic."""
    from fractions import Fraction
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def _vertex_x(k, origin, spacing):
    return [_fma(spacing[a], float(k[a]), origin[a]) for a in range(len(k))]


def ect_literal(img, dirs, thresholds, construction=PRIMAL, origin=None, spacing=None):
    """ECT by summing (-1)^dim phi over cells whose vertices all satisfy <xi,v> <= t, per t."""
    img = np.asarray(img)
    n = img.ndim
    origin = default_origin(img, construction) if origin is None else np.asarray(origin, float)
    spacing = np.ones(n) if spacing is None else np.asarray(spacing, float)
    cells = [(dim, val, verts) for _, dim, val, verts in _cells_literal(img, construction) if val != 0]
    out = np.zeros((len(dirs), len(thresholds)), dtype=np.int64)
    for d, xi in enumerate(dirs):
        proj = {}   # each vertex projected once per direction
        for _, _, verts in cells:
            for v in verts:
                if v not in proj:
                    proj[v] = _project(xi, _vertex_x(v, origin, spacing))
        for j, t in enumerate(thresholds):
            tot = 0
            for dim, val, verts in cells:
                if all(proj[v] <= t for v in verts):
                    tot += (-1) ** dim * val
            out[d, j] = tot
    return out


def critical_values_literal(img, construction=PRIMAL, generic=None):
    """Critical values from the star definitions with one generic xi per orthant.

    LwSt(xi, x): cells containing x on which max xi = xi(x); UpSt: min xi = xi(x).
    A generic xi of sign vector eps has nonzero, pairwise incommensurable entries.
    """
    img = np.asarray(img)
    n = img.ndim
    base = np.array([1.0, np.sqrt(2.0), np.sqrt(3.0), np.sqrt(5.0)])[:n] if generic is None else np.asarray(generic)
    cells = list(_cells_literal(img, construction))
    vshape = vertex_shape(img, construction)
    V = list(reversed(vshape))
    nv = int(np.prod(V))
    lw = np.zeros((nv, 1 << n), dtype=np.int64)
    up = np.zeros((nv, 1 << n), dtype=np.int64)
    for e in range(1 << n):
        eps = np.array([-1.0 if (e >> a) & 1 else 1.0 for a in range(n)])
        xi = eps * base
        for _, dim, val, verts in cells:
            if val == 0:
                continue
            proj = [float(np.dot(xi, np.array(v, float))) for v in verts]
            top = verts[int(np.argmax(proj))]
            bot = verts[int(np.argmin(proj))]
            sgn = (-1) ** dim * val
            vt = sum(top[a] * int(np.prod(V[:a])) for a in range(n))
            vb = sum(bot[a] * int(np.prod(V[:a])) for a in range(n))
            lw[vt, e] += sgn
            up[vb, e] += sgn
    return lw, up - lw


def radon_from_ect(img, xi, t, construction=PRIMAL, origin=None, spacing=None):
    """R(xi,t) = ECT(xi,t) + ECT(-xi,-t) - chi, at every t (ties included).

    {xi = t} = {xi <= t} minus the open set {xi < t}; the open sublevel set of xi
    at t is the complement of the closed sublevel set of -xi at -t, and chi is
    additive over this partition of the cells' relative interiors.  The canonical
    projection on -xi is exactly the negated projection on xi, so a vertex at t
    lies in both closed sublevel sets.
    """
    xi = np.asarray(xi, float)
    e1 = ect(img, xi[None], np.array([t]), construction, origin, spacing)[0, 0]
    e2 = ect(img, (-xi)[None], np.array([-t]), construction, origin, spacing)[0, 0]
    return int(e1) + int(e2) - euler_characteristic(img, construction)


def hybrid_integral(img, xi, kernel, s=1.0, construction=PRIMAL, origin=None, spacing=None):
    """HT(xi) = integral kappa_s(t) R(xi,t) dt with R piecewise constant between vertex projections.

    On each open interval (b_k, b_{k+1}) between consecutive distinct vertex
    projections, R is constant, so the integral of kappa_s over it is
    kbar_s(b_{k+1}) - kbar_s(b_k).  R vanishes outside [b_0, b_K].
    """
    img = np.asarray(img)
    n = img.ndim
    origin = default_origin(img, construction) if origin is None else np.asarray(origin, float)
    spacing = np.ones(n) if spacing is None else np.asarray(spacing, float)
    V = list(reversed(vertex_shape(img, construction)))
    pts = sorted({_project(xi, _vertex_x(k, origin, spacing))
                  for k in np.ndindex(*V)})
    kb = _kbar(kernel, s)
    tot = 0.0 + 0.0j
    for a, b in zip(pts[:-1], pts[1:]):
        r = radon_from_ect(img, xi, 0.5 * (a + b), construction, origin, spacing)
        if r:
            tot += r * (kb(b) - kb(a))
    return tot if kernel == "fourier" else tot.real


def _kbar(kernel, s):
    if s == 0:
        # kappa_0 is the constant kappa(0) = 1 for every kernel; its primitive is t
        return (lambda t: t + 0j) if kernel == "fourier" else (lambda t: t)
    if kernel == "fourier":
        return lambda t: (np.sin(s * t) + 1j * np.cos(s * t)) / s
    if kernel == "laplace":
        return lambda t: -np.exp(-s * t) / s
    if kernel == "bessel":
        return lambda t: ji0(s * t) / s
    raise ValueError(kernel)


if __name__ == "__main__":
    build(force=True)
    print(LIB_PATH)
    sys.exit(0)
