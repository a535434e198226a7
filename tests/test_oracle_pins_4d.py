"""Pins of the oracle on four-dimensional images (n-dimensional arrays, Sec. 4.1;
all 2^n sign vectors, Sec. 4.2): closed forms of chi, the ECT summed threshold
by threshold, the lower/upper stars from their definition, the invariants of the
critical values, Lemma 3.1 for the ECT and the hybrid transforms, closed boxes,
the literal integral of the hybrid transform, the Radon identity at every tie and
the exact representations.  Tiny inputs: the literal forms loop over cells in
Python."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_02256_amd import workloads as W

CONS = [O.PRIMAL, O.DUAL]


def _vertex_coords(img, construction):
    V = list(reversed(O.vertex_shape(img, construction)))
    o = O.default_origin(img, construction)
    ks = np.array(list(np.ndindex(*reversed(V))))[:, ::-1]  # axis 0 fastest
    return ks + o[None, :]


def _sign_index(xi):
    return sum(1 << a for a in range(len(xi)) if not (xi[a] >= 0))


@pytest.mark.parametrize("construction", CONS)
def test_chi_4d_boxes(construction):
    assert O.euler_characteristic(np.ones((3, 4, 2, 3), np.uint8), construction) == 1
    # a planar annulus (embedding axes 0, 1) times a 3 x 2 box has chi 0
    ring = np.ones((2, 3, 5, 5), np.uint8)
    ring[:, :, 1:4, 1:4] = 0
    assert O.euler_characteristic(ring, construction) == 0


def test_chi_4d_interior_block():
    """Primal-min keeps only the open interior of a block surrounded by zeros:
    an open 4-box has chi (-1)^4 = 1, and so does the closed one (dual)."""
    img = np.zeros((4, 5, 4, 5), np.uint8)
    img[1:3, 1:4, 1:3, 2:4] = 1
    assert O.euler_characteristic(img, O.PRIMAL) == 1
    assert O.euler_characteristic(img, O.DUAL) == 1
    img[1:3, 1:4, 1:3, 2:4] = 3
    assert O.euler_characteristic(img, O.PRIMAL) == 3


@pytest.mark.parametrize("construction", CONS)
def test_ect_4d_matches_literal_per_threshold_sum(construction):
    rng = np.random.default_rng(411)
    for shape in [(2, 2, 2, 2), (2, 1, 3, 2)]:
        img = W.random_image(rng, shape, 3)
        dirs = rng.standard_normal((3, 4))
        dirs[0, 1] = 0.0
        dirs[1, 3] = -0.0
        thr = np.sort(np.concatenate([rng.uniform(-3, 3, 5), [0.0, 0.5]]))
        assert np.array_equal(O.ect(img, dirs, thr, construction), O.ect_literal(img, dirs, thr, construction))


@pytest.mark.parametrize("construction", CONS)
def test_ect_4d_limits(construction):
    rng = np.random.default_rng(412)
    img = W.random_image(rng, (4, 3, 5, 3), 4)
    chi = O.euler_characteristic(img, construction)
    got = O.ect(img, rng.standard_normal((5, 4)), np.array([-1e6, 1e6]), construction)
    assert (got[:, 0] == 0).all() and (got[:, 1] == chi).all()


@pytest.mark.parametrize("construction", CONS)
def test_critical_values_4d_match_literal_star_definition(construction):
    rng = np.random.default_rng(413)
    for shape in [(2, 2, 2, 2), (3, 2, 2, 1)]:
        for _ in range(3):
            img = W.random_image(rng, shape, 3)
            lw, od = O.critical_values(img, construction)
            llw, lod = O.critical_values_literal(img, construction)
            assert lw.shape[1] == 16
            assert np.array_equal(lw, llw) and np.array_equal(od, lod)
    # binary 2x2x2x2 images, a seeded sample of the 65536
    imgs = W.all_binary_images((2, 2, 2, 2))
    for img in imgs[rng.choice(len(imgs), 24, replace=False)]:
        lw, od = O.critical_values(img, construction)
        llw, lod = O.critical_values_literal(img, construction)
        assert np.array_equal(lw, llw) and np.array_equal(od, lod)


@pytest.mark.parametrize("construction", CONS)
def test_critical_value_invariants_4d(construction):
    rng = np.random.default_rng(414)
    img = W.random_image(rng, (5, 4, 3, 4), 5)
    chi = O.euler_characteristic(img, construction)
    lw, od = O.critical_values(img, construction)
    assert (lw.sum(axis=0) == chi).all()
    assert (od.sum(axis=0) == 0).all()
    for e in range(16):
        assert np.array_equal(od[:, e], -od[:, 15 ^ e])


@pytest.mark.parametrize("construction", CONS)
def test_lemma31_ect_4d_from_classical_points(construction):
    """ECT(xi,.) = sum over classical points of Delta^- 1[u, inf) on random 4D images."""
    rng = np.random.default_rng(415)
    for shape in [(3, 2, 3, 2), (2, 3, 2, 3)]:
        img = W.random_image(rng, shape, 4)
        dirs = rng.standard_normal((6, 4))
        dirs[1, 2] = 0.0
        thr = np.sort(rng.uniform(-4, 4, 9))
        ref = O.ect(img, dirs, thr, construction)
        lw, _ = O.critical_values(img, construction)
        for d in range(len(dirs)):
            u = O.vertex_projections(img, dirs[d], construction)
            e = _sign_index(dirs[d])
            assert [(lw[:, e] * (u <= t)).sum() for t in thr] == ref[d].tolist()


@pytest.mark.parametrize("kernel", ["fourier", "laplace"])
@pytest.mark.parametrize("construction", CONS)
def test_lemma31_hybrid_4d_from_ordinary_points(kernel, construction):
    rng = np.random.default_rng(416)
    s = 0.8
    img = W.random_image(rng, (3, 2, 3, 2), 4)
    xi = rng.standard_normal((5, 4))
    ref = O.hybrid(img, xi, kernel, s, construction)
    _, od = O.critical_values(img, construction)
    x = _vertex_coords(img, construction)
    for q in range(len(xi)):
        z = s * (x @ xi[q])
        D = od[:, _sign_index(xi[q])]
        val = (D * (np.sin(z) + 1j * np.cos(z))).sum() / s if kernel == "fourier" else (D * -np.exp(-z)).sum() / s
        assert abs(val - ref[q]) <= 1e-11 * max(1.0, np.abs(D).sum())


@pytest.mark.parametrize("kernel", ["fourier", "laplace"])
def test_hybrid_closed_4d_box(kernel):
    rng = np.random.default_rng(417)
    img = np.ones((2, 3, 2, 4), np.uint8)
    for construction in CONS:
        xi = rng.standard_normal((3, 4)) * 0.4
        got = O.hybrid(img, xi, kernel, 1.3, construction)
        x = _vertex_coords(img, construction)
        for q in range(3):
            u = x @ xi[q]
            kb = (lambda t: (math.sin(1.3 * t) + 1j * math.cos(1.3 * t)) / 1.3) if kernel == "fourier" \
                else (lambda t: -math.exp(-1.3 * t) / 1.3)
            assert abs(got[q] - (kb(u.max()) - kb(u.min()))) < 1e-12


@pytest.mark.parametrize("construction", CONS)
def test_hybrid_4d_cell_form_equals_literal_integral(construction):
    rng = np.random.default_rng(418)
    img = W.random_image(rng, (2, 2, 2, 2), 3)
    for kernel in ("fourier", "laplace", "bessel"):
        xi = rng.standard_normal(4) * 0.8
        a = O.hybrid(img, xi[None], kernel, 0.9, construction)[0]
        b = O.hybrid_integral(img, xi, kernel, 0.9, construction)
        assert abs(a - b) < 1e-11


def _ties(img, xi, construction):
    u = np.unique(O.vertex_projections(img, xi, construction))
    mids = (u[1:] + u[:-1]) / 2 if u.size > 1 else u
    return np.sort(np.concatenate([u, mids, [u.min() - 1, u.max() + 1]]))


@pytest.mark.parametrize("construction", CONS)
def test_radon_4d_identity_and_exact_representations(construction):
    """R = ECT(xi,t) + ECT(-xi,-t) - chi at every vertex projection and between them, and both exact
    representations evaluate to the transforms there."""
    rng = np.random.default_rng(419)
    img = W.random_image(rng, (3, 4, 2, 3), 4)
    chi = O.euler_characteristic(img, construction)
    for xi in [rng.standard_normal(4), np.eye(4)[2], -np.eye(4)[0], np.round(rng.standard_normal(4) * 2) / 2]:
        t = _ties(img, xi, construction)
        r = O.radon(img, xi[None], t, construction)[0].astype(np.int64)
        e1 = O.ect(img, xi[None], t, construction)[0].astype(np.int64)
        e2 = O.ect(img, -xi[None], -t[::-1], construction)[0][::-1].astype(np.int64)
        assert np.array_equal(r, e1 + e2 - chi), xi
        T, E = O.ect_exact(img, xi, construction)
        assert np.array_equal(O.eval_ect_exact(T, E, t), e1)
        assert np.array_equal(O.eval_radon_exact(*O.radon_exact(img, xi, construction), t), r)
