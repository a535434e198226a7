"""GPU parity on four-dimensional images (n-dimensional arrays, Sec. 4.1; all
2^4 sign vectors, Sec. 4.2): the critical-point lists (16 classical, 8
ordinary), the ECT and the Radon transform at thresholds (bit-exact, ties
included), the hybrid transforms and their backward pass (the FP32 and FP64
gates of tests/gates.py) and the exact representations, against the FP64
oracle.  A batch of 1200 small 4D images runs the count/scan/write compaction
(more tiles than the chip holds at once); its lists are checked through the
ECT limits (0 below every projection, chi above) on every image and exactly on
a sample.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_02256_amd import workloads as W

from oracle.gates import fp32_gate, fp64_gate, term_scales

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_02256_amd import api as A
    return A


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))


def _check_lists(plan, i, img, construction):
    """Every list of image i equals the oracle's nonzero critical values in linear vertex order."""
    lw, od = O.critical_values(img, construction)
    V = list(reversed(O.vertex_shape(img, construction)))
    ks = np.array(np.meshgrid(*[np.arange(v) for v in V], indexing="ij")).reshape(4, -1).T
    ks = ks[np.lexsort(ks.T)]
    for kind, vals in ((0, lw), (1, od[:, :8])):
        for e in range(vals.shape[1]):
            nz = np.nonzero(vals[:, e])[0]
            coords, v = plan.export(i, kind, e)
            assert np.array_equal(coords, ks[nz]) and np.array_equal(v, vals[nz, e]), (i, kind, e)


def _dirs(rng, k):
    d = rng.standard_normal((k, 4))
    d[0] = [1.0, 0.0, 0.0, 0.0]
    d[1] = [0.0, -0.0, -1.0, 0.0]
    d[2] = np.round(d[2] * 2) / 2
    d[3, 1] = 0.0
    return d


def _ties(img, xi, construction, limit=2000):
    u = np.unique(O.vertex_projections(img, xi, construction))
    mids = (u[1:] + u[:-1]) / 2 if u.size > 1 else u
    t = np.sort(np.concatenate([u, mids, [u.min() - 1, u.max() + 1]]))
    return t[np.linspace(0, t.size - 1, min(limit, t.size)).astype(np.int64)]


@pytest.mark.parametrize("construction", [O.PRIMAL, O.DUAL])
def test_lists_4d(api, construction):
    rng = np.random.default_rng(601)
    imgs = [W.random_image(rng, (5, 4, 6, 3), 4), W.random_image(rng, (3, 3, 3, 3), 3),
            (W.random_image(rng, (7, 6, 5, 6), 2)).astype(np.uint8)]
    plan = api.Plan([T(im) for im in imgs], construction=construction)
    for i, im in enumerate(imgs):
        _check_lists(plan, i, im, construction)


@pytest.mark.parametrize("construction", [O.PRIMAL, O.DUAL])
def test_ect_and_radon_4d_at_every_tie(api, construction):
    rng = np.random.default_rng(602)
    img = W.random_image(rng, (6, 5, 4, 5), 4)
    plan = api.Plan(T(img), construction=construction)
    dirs = _dirs(rng, 12)
    R = float(np.sum(img.shape))
    thr = np.sort(np.concatenate([rng.uniform(-R, R, 60), np.arange(-R, R, 0.5)]))
    assert np.array_equal(plan.ect(T(dirs), T(thr)).cpu().numpy(), O.ect(img, dirs, thr, construction))
    assert np.array_equal(plan.radon(T(dirs), T(thr)).cpu().numpy(), O.radon(img, dirs, thr, construction))
    for xi in dirs[:6]:
        t = _ties(img, xi, construction)
        assert np.array_equal(plan.ect(T(xi[None]), T(t)).cpu().numpy(), O.ect(img, xi[None], t, construction))
        assert np.array_equal(plan.radon(T(xi[None]), T(t)).cpu().numpy(), O.radon(img, xi[None], t, construction))


def test_ect_4d_ragged_batch_per_image_thresholds(api):
    rng = np.random.default_rng(603)
    imgs = [W.random_image(rng, s, 3) for s in [(4, 5, 3, 4), (2, 2, 2, 2), (5, 3, 4, 3)]]
    plan = api.Plan([T(im) for im in imgs])
    M = 40
    thr = np.stack([np.linspace(-8, 8, M) + 0.25 * i for i in range(3)])
    counts = [9, 0, 20]
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    dirs = rng.standard_normal((offs[-1], 4))
    dirs[::5] = np.round(dirs[::5])
    for fn, ofn in ((plan.ect, O.ect), (plan.radon, O.radon)):
        got = fn(T(dirs), T(thr), offsets=T(offs)).cpu().numpy()
        for i, im in enumerate(imgs):
            if counts[i]:
                assert np.array_equal(got[offs[i]:offs[i + 1]], ofn(im, dirs[offs[i]:offs[i + 1]], thr[i])), i


@pytest.mark.parametrize("kernel", ["fourier", "laplace", "bessel"])
def test_hybrid_4d(api, kernel):
    rng = np.random.default_rng(604)
    img = W.random_image(rng, (6, 5, 6, 4), 3)
    xi = rng.standard_normal((150, 4)) * 0.4
    for construction in (O.PRIMAL, O.DUAL):
        plan = api.Plan(T(img), construction=construction)
        ref = O.hybrid(img, xi, kernel, 0.9, construction)
        S1, S2 = term_scales(img, xi, kernel, 0.9, construction)
        for precision in ("fp32", "fp64"):
            y = plan.hybrid(T(xi), kernel, 0.9, precision).cpu().numpy()
            y = y[:, 0] + 1j * y[:, 1] if kernel == "fourier" else y
            if precision == "fp32":
                ok, ratio, norm, strict = fp32_gate(y, ref, S2)
                assert ok, (construction, ratio, norm, strict)
            else:
                ok, ratio = fp64_gate(y, ref, S1)
                assert ok, (construction, ratio)


@pytest.mark.parametrize("kernel", ["fourier", "laplace"])
def test_backward_4d(api, kernel):
    rng = np.random.default_rng(605)
    imgs = [W.random_image(rng, (5, 4, 5, 4), 3), W.random_image(rng, (4, 4, 3, 5), 3)]
    plan = api.Plan([T(im) for im in imgs])
    xi = rng.standard_normal((30, 4)) * 0.3
    y = plan.hybrid(T(xi), kernel, 1.0, "fp64")
    g = rng.standard_normal(tuple(y.shape))
    gxi, gs = plan.hybrid_backward(T(xi), y, T(g), kernel, 1.0, "fp64")
    gxi, gs = gxi.cpu().numpy(), float(gs.cpu())
    rows = g.reshape(2, 30, *g.shape[1:])
    rgx = np.zeros((30, 4))
    rgs = 0.0
    for i, im in enumerate(imgs):
        a, b = O.hybrid_grad(im, xi, kernel, 1.0, rows[i])
        rgx += a
        rgs += b
    assert np.abs(gxi - rgx).max() <= 1e-9 * max(np.abs(rgx).max(), 1.0)
    assert abs(gs - rgs) <= 1e-9 * max(abs(rgs), np.abs(rgx).max(), 1.0)


@pytest.mark.parametrize("construction", [O.PRIMAL, O.DUAL])
def test_exact_4d(api, construction):
    rng = np.random.default_rng(606)
    img = W.random_image(rng, (5, 6, 4, 5), 4)
    plan = api.Plan(T(img), construction=construction)
    dirs = _dirs(rng, 10)
    for kind in ("ect", "radon"):
        rows = plan.exact(T(dirs), kind).to_host()
        for r, xi in enumerate(dirs):
            exp = O.ect_exact(img, xi, construction) if kind == "ect" else O.radon_exact(img, xi, construction)
            for g, e in zip(rows[r], exp):
                assert np.array_equal(g, e), (kind, r)


def test_large_4d_batch_uses_the_counting_compaction(api):
    rng = np.random.default_rng(607)
    imgs = [W.random_image(rng, (4, 4, 4, 4), 3) for _ in range(1200)]
    plan = api.Plan([T(im) for im in imgs])
    dirs = _dirs(rng, 6)
    got = plan.ect(T(dirs), T(np.array([-1e6, 1e6]))).cpu().numpy().reshape(len(imgs), len(dirs), 2)
    chi = np.array([O.euler_characteristic(im) for im in imgs])
    assert (got[:, :, 0] == 0).all()
    assert (got[:, :, 1] == chi[:, None]).all()
    for i in rng.choice(len(imgs), 6, replace=False):
        _check_lists(plan, int(i), imgs[i], O.PRIMAL)
    assert plan.check() == 0
