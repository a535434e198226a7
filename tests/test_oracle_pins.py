"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test states the fact it checks.  None of them re-types an oracle formula:
they use printed values of the worked example (Appendix A), closed forms of
simple complexes, invariants implied by the lemmas, and brute force on tiny
inputs through independent literal forms.
"""
import json
import math
import os

import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_02256_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _example():
    d = json.load(open(os.path.join(GOLD, "running_example.json")))
    img = np.array(d["image_rows_axis1"], dtype=np.uint8)
    return d, img


def _paper_coords(img):
    n = img.ndim
    N = np.array(list(reversed(img.shape))) - 1  # dual: N top cells per axis
    return np.full(n, -0.5), 1.0 / N.astype(float)


def _gudhi_vertex_id(v, img):
    # vertex linear index (axis 0 fastest over dims) -> cell id of the 7x7 grid
    V = list(reversed(img.shape))
    k0, k1 = v % V[0], v // V[0]
    G0 = 2 * (V[0] - 1) + 1
    return 2 * k0 + G0 * 2 * k1


# ----------------------------------------------------------------------------
# Appendix A: the running example
# ----------------------------------------------------------------------------

def test_example_nonzero_cells():
    d, img = _example()
    phi = O.cell_values(img, O.DUAL)
    dims = [(c[0] & 1) + (c[1] & 1) for c in np.ndindex(*phi.shape)]
    nz = phi.reshape(-1) != 0
    counts = np.bincount(np.array(dims)[nz], minlength=3)
    assert counts.tolist() == [d["nonzero_cells"]["vertices"], d["nonzero_cells"]["edges"],
                               d["nonzero_cells"]["squares"]]


def test_example_table2_critical_lists():
    """Every entry of Table 2, for all four sign vectors."""
    d, img = _example()
    lists = O.critical_lists(img, O.DUAL)
    for row in d["table2"]:
        e = sum(1 << a for a, s in enumerate(row["eps"]) if s < 0)
        cls, ordn = lists[e]
        got_c = {_gudhi_vertex_id(v, img): val for v, val in cls.items()}
        got_o = {_gudhi_vertex_id(v, img): val for v, val in ordn.items()}
        assert got_c == {int(k): v for k, v in row["classical"].items()}, row["eps"]
        assert got_o == {int(k): v for k, v in row["ordinary"].items()}, row["eps"]


def test_example_ect_evaluations_and_vectorization():
    d, img = _example()
    o, h = _paper_coords(img)
    xi = np.array([d["xi"]])
    vec = d["vectorization"]
    ts = np.array([vec["a"] + i * (vec["b"] - vec["a"]) / (vec["N"] - 1) for i in range(vec["N"])])
    assert O.ect(img, xi, ts, O.DUAL, o, h)[0].tolist() == vec["values"]
    for ev in d["ect_evaluations"]:
        assert O.ect(img, xi, np.array([ev["t"]]), O.DUAL, o, h)[0, 0] == ev["ect"]


def test_example_ect_exact_representation_values():
    """The jumps of the ECT curve at xi=(2,2) sit at the printed T and reach the printed E."""
    d, img = _example()
    o, h = _paper_coords(img)
    rep = d["ect_exact_representation"]
    tol = rep["print_precision"]
    xi = np.array([d["xi"]])
    probes = [rep["T_printed"][0] - 1.0]
    for t in rep["T_printed"]:
        probes.append(t + tol)
    vals = O.ect(img, xi, np.array(probes), O.DUAL, o, h)[0].tolist()
    assert vals == rep["E"]
    # just below each jump the curve still has the previous value
    below = O.ect(img, xi, np.array(rep["T_printed"]) - tol, O.DUAL, o, h)[0].tolist()
    assert below == rep["E"][:-1]


def test_example_hybrid_from_definition():
    """kbar = exp (Laplace kernel with s = -1): the definition gives +4.714568."""
    d, img = _example()
    o, h = _paper_coords(img)
    hy = d["hybrid_exp_primitive"]
    xi = np.array([d["xi"]])
    val = O.hybrid(img, xi, "laplace", s=-1.0, construction=O.DUAL, origin=o, spacing=h)[0]
    assert abs(val - hy["value_from_definition"]) < hy["tolerance"]
    assert abs(abs(val) - abs(hy["printed"])) < 5e-4
    lit = O.hybrid_integral(img, xi[0], "laplace", s=-1.0, construction=O.DUAL, origin=o, spacing=h)
    assert abs(lit - val) < 1e-12


# ----------------------------------------------------------------------------
# Euler characteristic: closed forms
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("construction", [O.PRIMAL, O.DUAL])
def test_chi_filled_square_and_cube(construction):
    assert O.euler_characteristic(np.ones((5, 7), np.uint8), construction) == 1
    assert O.euler_characteristic(np.ones((3, 4, 5), np.uint8), construction) == 1


@pytest.mark.parametrize("construction", [O.PRIMAL, O.DUAL])
def test_chi_annulus(construction):
    img = np.ones((7, 7), np.uint8)
    img[2:5, 2:5] = 0
    assert O.euler_characteristic(img, construction) == 0


def test_chi_interior_blocks():
    """Primal-min keeps only the open interior of a block surrounded by zeros."""
    img2 = np.zeros((6, 6), np.uint8)
    img2[1:5, 2:4] = 1
    assert O.euler_characteristic(img2, O.PRIMAL) == 1      # open square: (-1)^2
    assert O.euler_characteristic(img2, O.DUAL) == 1        # closed square
    img3 = np.zeros((5, 5, 5), np.uint8)
    img3[1:4, 1:3, 2:4] = 1
    assert O.euler_characteristic(img3, O.PRIMAL) == -1     # open cube: (-1)^3
    assert O.euler_characteristic(img3, O.DUAL) == 1        # closed cube


def test_chi_two_components_and_weights():
    img = np.zeros((5, 9), np.uint8)
    img[1:4, 1:3] = 3
    img[1:4, 5:8] = 2
    assert O.euler_characteristic(img, O.DUAL) == 5
    assert O.euler_characteristic(img, O.PRIMAL) == 5


# ----------------------------------------------------------------------------
# ECT
# ----------------------------------------------------------------------------

def _rand_imgs(rng, shapes, levels):
    return [W.random_image(rng, s, levels) for s in shapes]


@pytest.mark.parametrize("construction", [O.PRIMAL, O.DUAL])
def test_ect_matches_literal_per_threshold_sum(construction):
    rng = np.random.default_rng(11)
    for img in _rand_imgs(rng, [(3, 4), (4, 3), (2, 2, 3)], 3):
        n = img.ndim
        dirs = rng.standard_normal((3, n))
        dirs[0, 0] = 0.0  # an axis-parallel direction (sign 0 case)
        R = float(np.linalg.norm(img.shape)) * 2
        thr = np.sort(np.concatenate([rng.uniform(-R, R, 5), [0.0, -0.5, 0.5]]))
        got = O.ect(img, dirs, thr, construction)
        lit = O.ect_literal(img, dirs, thr, construction)
        assert np.array_equal(got, lit)


@pytest.mark.parametrize("construction", [O.PRIMAL, O.DUAL])
def test_ect_limits(construction):
    rng = np.random.default_rng(12)
    img = W.random_image(rng, (9, 8), 4)
    chi = O.euler_characteristic(img, construction)
    dirs = rng.standard_normal((6, 2))
    got = O.ect(img, dirs, np.array([-1e6, 1e6]), construction)
    assert (got[:, 0] == 0).all() and (got[:, 1] == chi).all()


def test_ect_scaling_and_translation_bit_exact():
    rng = np.random.default_rng(13)
    img = W.random_image(rng, (10, 12), 3)
    dirs = np.round(rng.standard_normal((5, 2)) * 64) / 64   # dyadic directions
    thr = np.arange(-20, 21, 0.5)
    base = O.ect(img, dirs, thr)
    assert np.array_equal(O.ect(img, 4 * dirs, 4 * thr), base)
    v = np.array([3.0, -2.0])
    org = O.default_origin(img, O.PRIMAL) + v
    shifted = O.ect(img, dirs, thr[None, :].repeat(1, 0)[0] + 0.0, origin=org)
    # ECT_{origin+v}(xi, t + <xi,v>) = ECT_origin(xi, t)
    for d in range(dirs.shape[0]):
        w = float(dirs[d] @ v)
        assert np.array_equal(O.ect(img, dirs[d:d + 1], thr + w, origin=org)[0], base[d])
    assert shifted.shape == base.shape


def test_ect_point_reflection():
    """Rotating the image by 180 degrees equals negating the direction (centred origin)."""
    rng = np.random.default_rng(14)
    img = W.random_image(rng, (7, 10), 3)
    dirs = rng.standard_normal((4, 2))
    thr = np.linspace(-9, 9, 37)
    a = O.ect(img, dirs, thr)
    b = O.ect(img[::-1, ::-1].copy(), -dirs, thr)
    assert np.array_equal(a, b)


# ----------------------------------------------------------------------------
# Critical values (Sec. 3) and Lemma 3.1
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("construction", [O.PRIMAL, O.DUAL])
def test_critical_values_match_literal_star_definition(construction):
    rng = np.random.default_rng(21)
    for img in _rand_imgs(rng, [(4, 5), (3, 3), (2, 3, 2)], 4):
        lw, od = O.critical_values(img, construction)
        llw, lod = O.critical_values_literal(img, construction)
        assert np.array_equal(lw, llw) and np.array_equal(od, lod)


def test_critical_values_exhaustive_3x3_primal_and_2x2x2():
    for img in W.all_binary_images((3, 3)):
        lw, od = O.critical_values(img, O.PRIMAL)
        llw, lod = O.critical_values_literal(img, O.PRIMAL)
        assert np.array_equal(lw, llw) and np.array_equal(od, lod)
    for construction in (O.PRIMAL, O.DUAL):
        for img in W.all_binary_images((2, 2, 2)):
            lw, od = O.critical_values(img, construction)
            llw, lod = O.critical_values_literal(img, construction)
            assert np.array_equal(lw, llw) and np.array_equal(od, lod)


@pytest.mark.parametrize("construction", [O.PRIMAL, O.DUAL])
def test_critical_value_invariants(construction):
    """sum Delta^- = chi for every eps; sum Delta^ord = 0; Delta^ord(-eps) = -Delta^ord(eps)."""
    rng = np.random.default_rng(22)
    for img in _rand_imgs(rng, [(12, 9), (5, 6, 4)], 5):
        chi = O.euler_characteristic(img, construction)
        lw, od = O.critical_values(img, construction)
        ne = lw.shape[1]
        assert (lw.sum(axis=0) == chi).all()
        assert (od.sum(axis=0) == 0).all()
        for e in range(ne):
            assert np.array_equal(od[:, e], -od[:, (ne - 1) ^ e])


def _vertex_coords(img, construction, origin=None):
    V = list(reversed(O.vertex_shape(img, construction)))
    o = O.default_origin(img, construction) if origin is None else origin
    ks = np.array(list(np.ndindex(*reversed(V))))[:, ::-1]  # axis 0 fastest
    return ks + o[None, :]


def _canon(xi, x):
    u = xi[0] * x[:, 0]
    for a in range(1, x.shape[1]):
        u = np.array([O._fma(float(xi[a]), float(xx), float(uu)) for xx, uu in zip(x[:, a], u)])
    return u


def _sign_index(xi):
    return sum(1 << a for a in range(len(xi)) if not (xi[a] >= 0))


@pytest.mark.parametrize("shape,construction", [((4, 4), O.DUAL), ((3, 3), O.PRIMAL),
                                                ((2, 2, 2), O.PRIMAL), ((2, 2, 2), O.DUAL)])
def test_lemma31_ect_from_classical_points_exhaustive(shape, construction):
    """ECT(xi,.) = sum over classical points of Delta^- 1[u, inf), bit for bit."""
    rng = np.random.default_rng(31)
    imgs = W.all_binary_images(shape)
    if len(imgs) > 4096:
        imgs = imgs[rng.choice(len(imgs), 1500, replace=False)]
    n = len(shape)
    dirs = rng.standard_normal((4, n))
    dirs[1, 0] = 0.0
    dirs[2, -1] = -0.0
    thr = np.sort(np.concatenate([rng.uniform(-3, 3, 6), [0.0]]))
    x = _vertex_coords(imgs[0], construction)
    us = [_canon(d, x) for d in dirs]
    for img in imgs:
        ref = O.ect(img, dirs, thr, construction)
        lw, _ = O.critical_values(img, construction)
        for d in range(len(dirs)):
            e = _sign_index(dirs[d])
            got = [(lw[:, e] * (us[d] <= t)).sum() for t in thr]
            assert got == ref[d].tolist()


@pytest.mark.parametrize("kernel", ["fourier", "laplace", "bessel"])
@pytest.mark.parametrize("construction", [O.PRIMAL, O.DUAL])
def test_lemma31_hybrid_from_ordinary_points(kernel, construction):
    """HT(xi) = + sum over ordinary points of Delta^ord kbar_s(<xi,x>) (definition's sign)."""
    rng = np.random.default_rng(32)
    s = 0.7
    for img in _rand_imgs(rng, [(6, 5), (3, 4, 3)], 4):
        n = img.ndim
        xi = rng.standard_normal((5, n))
        ref = O.hybrid(img, xi, kernel, s, construction)
        _, od = O.critical_values(img, construction)
        x = _vertex_coords(img, construction)
        for q in range(len(xi)):
            u = x @ xi[q]
            D = od[:, _sign_index(xi[q])]
            z = s * u
            if kernel == "fourier":
                val = (D * (np.sin(z) + 1j * np.cos(z))).sum() / s
            elif kernel == "laplace":
                val = (D * -np.exp(-z)).sum() / s
            else:
                val = sum(int(Di) * float(mp.quad(lambda t: mp.besselj(0, t), [0, zi]))
                          for Di, zi in zip(D, z) if Di) / s
            assert abs(val - ref[q]) <= 1e-11 * max(1.0, np.abs(D).sum())


# ----------------------------------------------------------------------------
# Hybrid transforms: closed forms and symmetries
# ----------------------------------------------------------------------------

def _box_extremes(img, construction, xi, origin=None):
    x = _vertex_coords(img, construction, origin)
    u = x @ xi
    return u.max(), u.min()


def _kbar(kernel, s, t):
    if kernel == "fourier":
        return (math.sin(s * t) + 1j * math.cos(s * t)) / s
    if kernel == "laplace":
        return -math.exp(-s * t) / s
    return float(mp.quad(lambda y: mp.besselj(0, y), [0, s * t])) / s


@pytest.mark.parametrize("kernel", ["fourier", "laplace", "bessel"])
def test_hybrid_closed_box(kernel):
    """A closed box (all-ones image): HT = kbar(M) - kbar(m) over the box's vertex projections."""
    rng = np.random.default_rng(41)
    for shape in [(5, 8), (3, 4, 2)]:
        img = np.ones(shape, np.uint8)
        for construction in (O.PRIMAL, O.DUAL):
            xi = rng.standard_normal((3, len(shape))) * 0.4
            got = O.hybrid(img, xi, kernel, 1.3, construction)
            for q in range(3):
                M, m = _box_extremes(img, construction, xi[q])
                want = _kbar(kernel, 1.3, M) - _kbar(kernel, 1.3, m)
                assert abs(got[q] - want) < 1e-12


@pytest.mark.parametrize("kernel", ["fourier", "laplace"])
def test_hybrid_open_box_primal(kernel):
    """Primal interior block = open box: HT = (-1)^(n-1) (kbar(M) - kbar(m)), M, m over the block."""
    rng = np.random.default_rng(42)
    for shape, sl in [((7, 8), (slice(2, 5), slice(1, 6))),
                      ((5, 6, 5), (slice(1, 3), slice(2, 5), slice(1, 4)))]:
        img = np.zeros(shape, np.uint8)
        img[sl] = 1
        n = len(shape)
        xi = rng.standard_normal((3, n)) * 0.5
        got = O.hybrid(img, xi, kernel, 1.0, O.PRIMAL)
        o = O.default_origin(img, O.PRIMAL)
        # block vertices: pixel range [start, stop) -> vertex range [start, stop]
        rngs = [np.arange(s_.start, s_.stop + 1) for s_ in reversed(sl)]  # axis order
        pts = np.array(np.meshgrid(*rngs, indexing="ij")).reshape(n, -1).T + o
        for q in range(3):
            u = pts @ xi[q]
            want = (-1) ** (n - 1) * (_kbar(kernel, 1.0, u.max()) - _kbar(kernel, 1.0, u.min()))
            assert abs(got[q] - want) < 1e-12


def test_hybrid_symmetries():
    rng = np.random.default_rng(43)
    img = W.random_image(rng, (11, 9), 4)
    xi = rng.standard_normal((6, 2)) * 0.3
    F = O.hybrid(img, xi, "fourier", 1.0)
    # conjugate symmetry
    assert np.allclose(O.hybrid(img, -xi, "fourier", 1.0), np.conj(F), atol=1e-12, rtol=0)
    # scale: HT_s(xi) = HT_1(s xi) / s
    for kern in ("fourier", "laplace", "bessel"):
        a = O.hybrid(img, xi, kern, 2.5)
        b = O.hybrid(img, 2.5 * xi, kern, 1.0) / 2.5
        assert np.allclose(a, b, atol=1e-12, rtol=1e-12)
    # translation phase
    v = np.array([1.5, -4.0])
    org = O.default_origin(img, O.PRIMAL) + v
    Ft = O.hybrid(img, xi, "fourier", 1.0, origin=org)
    assert np.allclose(Ft, F * np.exp(-1j * (xi @ v)), atol=1e-11, rtol=0)
    L = O.hybrid(img, xi, "laplace", 1.0)
    Lt = O.hybrid(img, xi, "laplace", 1.0, origin=org)
    assert np.allclose(Lt, L * np.exp(-(xi @ v)), atol=1e-11, rtol=1e-11)


@pytest.mark.parametrize("construction", [O.PRIMAL, O.DUAL])
@pytest.mark.parametrize("kernel", ["fourier", "laplace", "bessel"])
def test_hybrid_cell_form_equals_literal_integral(kernel, construction):
    rng = np.random.default_rng(44)
    for img in _rand_imgs(rng, [(3, 4), (2, 3, 2)], 3):
        n = img.ndim
        for _ in range(2):
            xi = rng.standard_normal(n) * 0.8
            a = O.hybrid(img, xi[None], kernel, 0.9, construction)[0]
            b = O.hybrid_integral(img, xi, kernel, 0.9, construction)
            assert abs(a - b) < 1e-11


def test_laplace_shift_rescales_exactly():
    rng = np.random.default_rng(45)
    img = W.random_image(rng, (20, 16), 3)
    xi = rng.standard_normal((8, 2))
    plain = O.hybrid(img, xi, "laplace", 1.0)
    out, m = O.hybrid(img, xi, "laplace", 1.0, with_shift=True)
    assert np.allclose(out * np.exp(m), plain, rtol=1e-12, atol=0)
    assert (np.abs(out) <= 64).all()   # every term is at most |phi| after the shift


# ----------------------------------------------------------------------------
# Ji0 and gradients
# ----------------------------------------------------------------------------

def test_ji0_against_mpmath_and_limits():
    for z in [0.0, 1e-3, 0.5, 2.404825557695773, 7.9, 10.0, 33.3, 250.0, 887.0]:
        ref = float(mp.quad(lambda t: mp.besselj(0, t), mp.linspace(0, z, int(z) + 2)))
        assert abs(O.ji0(z) - ref) < 5e-15 * max(1.0, z / 50)
        assert O.ji0(-z) == -O.ji0(z)
    assert abs(O.ji0(5000.0) - 1.0) < 0.02
    assert abs(O.ji0(10.0) - 1.06701130395674) < 1e-13


@pytest.mark.parametrize("kernel", ["fourier", "laplace", "bessel"])
def test_gradient_matches_central_differences(kernel):
    rng = np.random.default_rng(51)
    img = W.random_image(rng, (10, 9), 2)
    xi = W.polar_vectors(rng, 5, 0.05, 0.5, axis_gap=0.05)
    s = 1.1
    g = rng.standard_normal((5, 2)) if kernel == "fourier" else rng.standard_normal(5)
    if kernel == "fourier":
        gc = g[:, 0] + 1j * g[:, 1]
    gxi, gs = O.hybrid_grad(img, xi, kernel, s, g)

    def loss(xv, sv):
        y = O.hybrid(img, xv, kernel, sv)
        if kernel == "fourier":
            return float((gc.real * y.real + gc.imag * y.imag).sum())
        return float((g * y).sum())

    h = 1e-5
    for q in range(5):
        for a in range(2):
            xp, xm = xi.copy(), xi.copy()
            xp[q, a] += h
            xm[q, a] -= h
            fd = (loss(xp, s) - loss(xm, s)) / (2 * h)
            assert abs(fd - gxi[q, a]) <= 1e-6 * max(1.0, abs(fd))
    fd_s = (loss(xi, s + h) - loss(xi, s - h)) / (2 * h)
    assert abs(fd_s - gs) <= 1e-6 * max(1.0, abs(fd_s))


def test_lemma31_laplace_large_phases_cancellation():
    """At phases ~10^3 every critical point can sit far below the maximal vertex; the cell
    form must still equal the critical-point sum (here summed with correctly rounded fsum)."""
    rng = np.random.default_rng(606)
    img = W.quantised_volume(rng, 16, 2.0)
    xi = W.sphere_vectors(rng, 24, 0.5, 20.0)
    org = np.zeros(3)
    out, m = O.hybrid(img, xi, "laplace", 1.0, origin=org, with_shift=True)
    _, od = O.critical_values(img, O.PRIMAL)
    x = _vertex_coords(img, O.PRIMAL, org)
    for q in range(len(xi)):
        D = od[:, _sign_index(xi[q])]
        nz = np.nonzero(D)[0]
        u = x[nz] @ xi[q]
        terms = [-float(d) * math.exp(-uu - m[q]) for d, uu in zip(D[nz], u)]
        ref = math.fsum(terms)
        scale = math.fsum(abs(t) for t in terms)
        # Sum2 bound: a relative 1e-12 of the critical-point terms plus a doubled-precision
        # residue (~2^-106) of the O(1) cell terms that cancel at non-critical vertices
        assert abs(out[q] - ref) <= 1e-12 * scale + 1e-28, (q, out[q], ref, scale)


# ----------------------------------------------------------------------------
# Exact representations (Sec. 4.3) and the Radon transform (Sec. 2.2)
# ----------------------------------------------------------------------------

def test_example_ect_exact_pairs():
    """(T, E) of the example at xi = (2,2): jumps at the printed T, values E (merging the two points
    that share -2/3)."""
    d, img = _example()
    o, h = _paper_coords(img)
    rep = d["ect_exact_representation"]
    T, E = O.ect_exact(img, np.array(d["xi"]), O.DUAL, o, h)
    assert T[0] == -np.inf and E.tolist() == rep["E"]
    assert np.allclose(T[1:], rep["T_printed"], atol=rep["print_precision"])


def test_example_radon_exact_ordinary_jumps():
    """The ordinary jumps of the example's Radon transform sit where the paper prints them; the
    values carry the sign the definition gives (the negated E' of the printed example), and the
    point values at the classical projections agree with the slice Euler characteristic."""
    d, img = _example()
    o, h = _paper_coords(img)
    xi = np.array(d["xi"])
    T, Ep, Tc, Ec = O.radon_exact(img, xi, O.DUAL, o, h)
    assert np.allclose(T[1:], [-2.0 / 3.0, 2.0 / 3.0, 4.0 / 3.0], atol=1e-12)
    assert Ep.tolist() == [0, 2, 1, 0]
    assert np.allclose(Tc, [-2.0, -2.0 / 3.0, 0.0], atol=1e-12)
    assert Ec.tolist() == O.radon(img, xi[None], Tc, O.DUAL, o, h)[0].tolist()


def _tie_thresholds(img, xi, construction, origin=None, spacing=None, extra=0, rng=None):
    u = O.vertex_projections(img, xi, construction, origin, spacing)
    t = np.unique(u)
    if extra:
        t = np.concatenate([t, rng.uniform(t.min() - 1, t.max() + 1, extra)])
    mids = (t[1:] + t[:-1]) / 2 if t.size > 1 else t
    return np.sort(np.concatenate([t, mids]))


@pytest.mark.parametrize("construction", [O.PRIMAL, O.DUAL])
def test_radon_identity_with_ect_at_every_tie(construction):
    """R(xi,t) = ECT(xi,t) + ECT(-xi,-t) - chi holds at every t, ties included (a vertex at t is in
    both closed sublevel sets; a cell with min < t < max is in neither)."""
    rng = np.random.default_rng(71)
    for shape in [(5, 6), (4, 3, 5)]:
        img = W.random_image(rng, shape, 4)
        chi = O.euler_characteristic(img, construction)
        n = img.ndim
        dirs = [rng.standard_normal(n), np.eye(n)[0], -np.eye(n)[n - 1], np.round(rng.standard_normal(n) * 2) / 2]
        for xi in dirs:
            t = _tie_thresholds(img, xi, construction, extra=7, rng=rng)
            r = O.radon(img, xi[None], t, construction)[0].astype(np.int64)
            e1 = O.ect(img, xi[None], t, construction)[0].astype(np.int64)
            e2 = O.ect(img, -xi[None], -t[::-1], construction)[0][::-1].astype(np.int64)
            assert np.array_equal(r, e1 + e2 - chi), (shape, xi)


def test_radon_closed_square_and_reflection():
    """One pixel of value 3 (primal): the slice of the closed square has chi 1 on [min, max], 0 off
    it; R(-xi, -t) = R(xi, t)."""
    img = np.array([[3]], dtype=np.int32)
    xi = np.array([0.7, -1.3])
    corners = [np.dot(xi, [a, b]) for a in (-0.5, 0.5) for b in (-0.5, 0.5)]
    lo, hi = min(corners), max(corners)
    t = np.array([lo - 1, lo, (lo + hi) / 2, hi, hi + 0.25])
    assert O.radon(img, xi[None], t)[0].tolist() == [0, 3, 3, 3, 0]
    assert O.radon(img, -xi[None], -t[::-1])[0].tolist() == [0, 3, 3, 3, 0][::-1]


@pytest.mark.parametrize("construction", [O.PRIMAL, O.DUAL])
def test_exact_representations_evaluate_to_the_transforms(construction):
    """(T, E) evaluated by binary search equals the ECT of the cells, and (T, E', Tc, Ec) equals the
    Radon transform of the cells, at every tie and between them."""
    rng = np.random.default_rng(72)
    for shape in [(6, 7), (3, 4, 4)]:
        img = W.random_image(rng, shape, 5)
        n = img.ndim
        for xi in [rng.standard_normal(n), np.eye(n)[1] * -1.0, np.full(n, 0.5)]:
            t = _tie_thresholds(img, xi, construction, extra=5, rng=rng)
            T, E = O.ect_exact(img, xi, construction)
            assert np.array_equal(O.eval_ect_exact(T, E, t), O.ect(img, xi[None], t, construction)[0])
            rep = O.radon_exact(img, xi, construction)
            assert np.array_equal(O.eval_radon_exact(*rep, t), O.radon(img, xi[None], t, construction)[0])
            assert np.all(np.diff(T) > 0) and np.all(np.diff(rep[2]) > 0)


# ----------------------------------------------------------------------------
# s = 0: the constant kernel kappa_0 = kappa(0) = 1 (primitive t)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("kernel", ["fourier", "laplace", "bessel"])
def test_hybrid_at_zero_scale(kernel):
    """HT_0(xi) = integral of R(xi, t) dt: a closed box gives M - m, the literal integral agrees on a
    random image, and HT_s tends to it as s -> 0 (the limit of Lemma 3.1's sum, as sum D = 0)."""
    rng = np.random.default_rng(49)
    box = np.ones((4, 6), np.uint8)
    xi = rng.standard_normal((3, 2)) * 0.5
    got = O.hybrid(box, xi, kernel, 0.0)
    for q in range(3):
        M, m = _box_extremes(box, O.PRIMAL, xi[q])
        assert abs(got[q] - (M - m)) < 1e-12
    img = W.random_image(rng, (4, 3), 3)
    x = rng.standard_normal(2) * 0.7
    a = O.hybrid(img, x[None], kernel, 0.0)[0]
    assert abs(a - O.hybrid_integral(img, x, kernel, 0.0)) < 1e-11
    assert abs(O.hybrid(img, x[None], kernel, 1e-7)[0] - a) < 1e-5 * max(1.0, abs(a))
    if kernel == "fourier":
        assert a.imag == 0.0
