"""GPU parity of the Radon transform at thresholds (slice Euler characteristic,
Sec. 2.2, evaluated through Lemma 3.1 with the sign the definition gives)
against the FP64 CPU oracle, which counts the cells of each slice directly.

Bar: bit-exact.  Thresholds are placed on the vertex projections themselves
(computed by the oracle with the canonical expression) and between them, so
every tie case of the classical point term and of the open rays of the
ordinary term is exercised.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_02256_amd import workloads as W

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


def tie_thresholds(img, xi, construction, origin=None, spacing=None, extra=0, rng=None, limit=4096):
    """Distinct vertex projections on xi, the midpoints between them and a few
    random values, sorted (at most `limit`, evenly subsampled)."""
    u = np.unique(O.vertex_projections(img, xi, construction, origin, spacing))
    mids = (u[1:] + u[:-1]) / 2 if u.size > 1 else u
    t = np.concatenate([u, mids])
    if extra:
        t = np.concatenate([t, rng.uniform(u.min() - 1, u.max() + 1, extra)])
    t = np.sort(t)
    if t.size > limit:
        t = t[np.linspace(0, t.size - 1, limit).astype(np.int64)]
    return t


def test_radon_running_example(api):
    img = W.RUNNING_EXAMPLE
    o, h = [-0.5, -0.5], [1 / 3, 1 / 3]
    plan = api.Plan(T(img), construction=O.DUAL, origin=o, spacing=h)
    for xi in (np.array([2.0, 2.0]), np.array([1.0, -0.5]), np.array([-1.0, 0.0])):
        t = tie_thresholds(img, xi, O.DUAL, o, h)
        got = plan.radon(T(xi[None]), T(t)).cpu().numpy()
        assert np.array_equal(got, O.radon(img, xi[None], t, O.DUAL, o, h)), xi


@pytest.mark.parametrize("construction", [O.PRIMAL, O.DUAL])
def test_radon_at_every_tie_2d_3d(api, construction):
    """One direction per call with thresholds on its own vertex projections:
    random, axis, negated axis, signed-zero and half-integer directions."""
    rng = np.random.default_rng(801)
    for shape in [(23, 31), (9, 12, 7)]:
        img = W.random_image(rng, shape, 5)
        n = img.ndim
        plan = api.Plan(T(img), construction=construction)
        dirs = [rng.standard_normal(n), np.eye(n)[0], -np.eye(n)[n - 1],
                np.round(rng.standard_normal(n) * 2) / 2, np.array([-0.0] * (n - 1) + [1.0]),
                np.full(n, 0.5)]
        for xi in dirs:
            t = tie_thresholds(img, xi, construction, extra=9, rng=rng)
            got = plan.radon(T(xi[None]), T(t)).cpu().numpy()
            assert np.array_equal(got, O.radon(img, xi[None], t, construction)), (shape, xi)


@pytest.mark.parametrize("construction", [O.PRIMAL, O.DUAL])
def test_radon_shared_set_on_a_quarter_grid(api, construction):
    """A shared direction set whose axis and lattice directions hit the
    quarter-integer thresholds exactly, next to random ones that do not."""
    rng = np.random.default_rng(802)
    for shape in [(40, 37), (11, 8, 13)]:
        img = W.random_image(rng, shape, 4)
        n = img.ndim
        lattice = [np.eye(n)[a] * s for a in range(n) for s in (1.0, -1.0)]
        lattice += [np.ones(n), np.array([1.0, -1.0] + [0.5] * (n - 2)), np.full(n, -0.5)]
        dirs = np.concatenate([np.array(lattice), rng.standard_normal((13, n))])
        R = float(np.sum(shape)) + 2
        t = np.arange(-R, R + 0.125, 0.25)
        plan = api.Plan(T(img), construction=construction)
        got = plan.radon(T(dirs), T(t)).cpu().numpy()
        assert np.array_equal(got, O.radon(img, dirs, t, construction)), shape


def test_radon_ragged_batch_per_image_thresholds(api):
    rng = np.random.default_rng(803)
    sides = [28, 64, 5, 1, 45]
    imgs = [W.binary_field(rng, (s, s), 3.0) if s > 4 else W.random_image(rng, (s, s), 2) for s in sides]
    plan = api.Plan([T(im) for im in imgs])
    M = 61
    thr = np.stack([np.arange(M) * 0.5 - s / 2 - 1 for s in sides])
    counts = [7, 0, 12, 3, 20]
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    dirs = rng.standard_normal((offs[-1], 2))
    dirs[::3] = np.round(dirs[::3])          # lattice directions tie on the half-integers
    got = plan.radon(T(dirs), T(thr), offsets=T(offs)).cpu().numpy()
    for i, im in enumerate(imgs):
        if counts[i]:
            ref = O.radon(im, dirs[offs[i]:offs[i + 1]], thr[i])
            assert np.array_equal(got[offs[i]:offs[i + 1]], ref), i
    sd = np.concatenate([W.circle_dirs(8), np.eye(2)])
    got = plan.radon(T(sd), T(thr)).cpu().numpy().reshape(len(imgs), len(sd), M)
    for i, im in enumerate(imgs):
        assert np.array_equal(got[i], O.radon(im, sd, thr[i])), i


def test_radon_grf512_identity_and_sampled_rows(api):
    """Full 512 x 512 field with its 360 directions: every row satisfies
    R(xi, t) = ECT(xi, t) + ECT(-xi, -t) - chi (the ECTs from the GPU path,
    chi from the oracle), sampled rows equal the oracle, and one direction is
    checked at its own vertex projections."""
    w = W.grf_512(2, n_xi=8)
    img = w.images[0]
    plan = api.Plan(T(img))
    dirs, t = w.ect_dirs, w.ect_thresholds
    r = plan.radon(T(dirs), T(t)).cpu().numpy().astype(np.int64)
    e1 = plan.ect(T(dirs), T(t)).cpu().numpy().astype(np.int64)
    e2 = plan.ect(T(-dirs), T(-t[::-1])).cpu().numpy()[:, ::-1].astype(np.int64)
    chi = O.euler_characteristic(img)
    assert np.array_equal(r, e1 + e2 - chi)
    sel = np.arange(0, len(dirs), 45)
    assert np.array_equal(r[sel], O.radon(img, dirs[sel], t))
    xi = np.array([1.0, 0.0])
    tt = tie_thresholds(img, xi, O.PRIMAL)
    got = plan.radon(T(xi[None]), T(tt)).cpu().numpy()
    assert np.array_equal(got, O.radon(img, xi[None], tt))


def test_radon_large_threshold_count_and_tiny(api):
    rng = np.random.default_rng(804)
    img = W.random_image(rng, (30, 30), 3)
    thr = np.linspace(-25, 25, 4096)
    dirs = np.concatenate([rng.standard_normal((6, 2)), np.eye(2)])
    plan = api.Plan(T(img))
    got = plan.radon(T(dirs), T(thr)).cpu().numpy()
    assert np.array_equal(got, O.radon(img, dirs, thr))
    for tiny in (np.array([[3]], np.int32), np.zeros((1, 1), np.int32), np.zeros((2, 2, 2), np.int32)):
        p = api.Plan(T(tiny))
        d = np.eye(tiny.ndim)[:1]
        tt = np.array([-1.0, -0.5, 0.0, 0.5, 1.0])
        assert np.array_equal(p.radon(T(d), T(tt)).cpu().numpy(), O.radon(tiny, d, tt)), tiny.shape


def test_radon_non_finite_and_unsorted(api):
    rng = np.random.default_rng(805)
    img = W.random_image(rng, (17, 19), 4)
    plan = api.Plan(T(img))
    dirs = W.circle_dirs(6)
    dirs[2] = [np.nan, 0.0]
    thr = np.arange(-15.0, 15.0, 0.5)
    got = plan.radon(T(dirs), T(thr)).cpu().numpy()
    fin = np.isfinite(dirs).all(axis=1)
    assert (got[~fin] == 0).all()
    assert np.array_equal(got[fin], O.radon(img, dirs[fin], thr))
    assert plan.check() & 0x4
    bad = np.array([0.0, 1.0, 0.5])
    assert (plan.radon(T(dirs[fin]), T(bad)).cpu().numpy() == 0).all()
    assert plan.check() & 0x2
