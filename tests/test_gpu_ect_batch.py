"""The direction-parallel ECT kernel for shared direction sets over many
images with short lists (one workgroup per (image, sign vector), lanes own
directions), against the oracle and against the point-parallel kernel, bit
for bit: ragged image sizes, several passes of a sign bucket's directions,
axis and signed-zero directions, a non-finite direction, per-image
thresholds with one unsorted row, three and four axes."""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_02256_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_02256_amd import _native as N
    from paper_2405_02256_amd import api as A
    return A, N


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))


def _uses_batch_kernel(A, N, plan, dirs, thr):
    """The batch path buckets the set in a workspace; the point-parallel path on an unsplit shared set
    needs none."""
    q = A.QuerySet(T(dirs))
    need = ctypes.c_size_t(0)
    out = torch.empty((q.rows(plan.num_images), thr.shape[-1]), dtype=torch.int32, device="cuda:0")
    N.check(N.ect_eval(plan.handle, q.c(), A._dptr(thr), thr.shape[-1], 1 if thr.dim() == 2 else 0,
                       A._dptr(out), None, need, A._stream()), "ect_eval(size)")
    return need.value > 0


def _check(A, N, imgs, dirs, thr_np, expect_batch=True):
    plan = A.Plan([T(im) for im in imgs])
    thr = T(thr_np)
    assert _uses_batch_kernel(A, N, plan, dirs, thr) == expect_batch
    got = plan.ect(T(dirs), thr).cpu().numpy().reshape(len(imgs), len(dirs), -1)
    flags = plan.check()
    plan.set_tuning(0, 2048, 8, 1)                      # the point-parallel kernel
    assert not _uses_batch_kernel(A, N, plan, dirs, thr)
    ref_gpu = plan.ect(T(dirs), thr).cpu().numpy().reshape(len(imgs), len(dirs), -1)
    assert plan.check() == flags
    assert np.array_equal(got, ref_gpu)
    fin = np.isfinite(dirs).all(axis=1)
    for i, im in enumerate(imgs):
        t = thr_np[i] if thr_np.ndim == 2 else thr_np
        if np.all(np.diff(t) >= 0):
            assert np.array_equal(got[i][fin], O.ect(im, dirs[fin], t)), i
            assert (got[i][~fin] == 0).all()
        else:
            assert (got[i] == 0).all(), i
    return flags


def test_batch_ect_2d_ragged(mods):
    A, N = mods
    rng = np.random.default_rng(2501)
    sides = rng.integers(3, 40, size=300)
    imgs = [W.binary_field(rng, (int(s), int(s + 3)), 2.0) if s > 6 else W.random_image(rng, (int(s), 5), 3)
            for s in sides]
    dirs = rng.standard_normal((150, 2))                 # ~37 directions per sign vector: two passes each
    dirs[0] = [1.0, 0.0]
    dirs[1] = [-0.0, 1.0]
    dirs[2] = [0.0, -0.0]
    dirs[3] = [-1.0, -0.0]
    dirs[4] = [np.nan, 0.5]
    M = 100
    thr = np.stack([W.even_thresholds(float(max(s, 5)), M) for s in sides])
    thr[7, 10], thr[7, 11] = thr[7, 11], thr[7, 10]     # one image's thresholds out of order
    flags = _check(A, N, imgs, dirs, thr)
    assert flags & N.DEVERR_NONFINITE and flags & N.DEVERR_THRESHOLDS


def test_batch_ect_short_and_long_lists(mods):
    """Lists from a few points to a few thousand (one partial stage of the
    streamed list, or several), passes of 16 and of 1 to 3 directions."""
    A, N = mods
    rng = np.random.default_rng(2504)
    sides = rng.choice([9, 14, 30, 60, 120, 200], size=144)   # enough images for the batch kernel
    imgs = [W.binary_field(rng, (int(s), int(s) + 5), 2.5) for s in sides]
    dirs = rng.standard_normal((70, 2))                  # ~17 directions per sign vector
    dirs[0] = [1.0, 0.0]
    M = 64
    thr = np.stack([W.even_thresholds(float(s), M) for s in sides])
    _check(A, N, imgs, dirs, thr)
    _check(A, N, imgs, dirs[:9], thr)                     # one to three directions per sign vector


def test_batch_ect_shared_thresholds_one_direction_per_bucket_and_max_m(mods):
    A, N = mods
    rng = np.random.default_rng(2502)
    imgs = [W.binary_field(rng, (20, 24), 3.0) for _ in range(200)]
    dirs = W.circle_dirs(4) + 1e-3                        # one direction per sign vector
    _check(A, N, imgs, dirs, np.linspace(-18.0, 18.0, 256))
    # above the largest threshold count the point-parallel kernel runs
    _check(A, N, imgs[:140], W.circle_dirs(16), np.linspace(-18.0, 18.0, 257), expect_batch=False)


def test_batch_ect_3d_and_4d(mods):
    A, N = mods
    rng = np.random.default_rng(2503)
    vols = [W.random_image(rng, tuple(int(v) for v in rng.integers(2, 8, size=3)), 4) for _ in range(80)]
    d3 = rng.standard_normal((40, 3))
    d3[0] = [0.0, 0.0, 1.0]
    _check(A, N, vols, d3, np.linspace(-8.0, 8.0, 64))
    hv = [W.random_image(rng, tuple(int(v) for v in rng.integers(2, 4, size=4)), 3) for _ in range(40)]
    d4 = rng.standard_normal((24, 4))
    _check(A, N, hv, d4, np.linspace(-5.0, 5.0, 40))


def test_batch_ect_ties_uneven_and_offset_thresholds(mods):
    """Projections that land exactly on thresholds (axis and diagonal directions over half-integer vertex
    coordinates and thresholds on the half-integer grid), thresholds that are far from evenly spaced, and a
    coordinate frame far from the origin: every bin is the first threshold at or above the projection."""
    A, N = mods
    rng = np.random.default_rng(2504)
    imgs = [W.binary_field(rng, (18, 15), 2.5) for _ in range(200)]
    dirs = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, 1.0], [-1.0, 1.0], [1.0, -2.0], [-0.5, -0.5],
                     [2.0, 1.0], [0.0, -1.0], [-1.0, 0.0], [0.25, 0.75]])
    _check(A, N, imgs, dirs, np.arange(-20.0, 20.25, 0.5))
    uneven = np.sort(rng.uniform(-20.0, 20.0, size=90))
    uneven[40:44] = uneven[40]                            # repeated thresholds
    _check(A, N, imgs, dirs, uneven)
    # far from the origin: vertex coordinates near 1e6, thresholds around them
    org = np.array([1.0e6, -1.0e6])
    plan = A.Plan([T(im) for im in imgs], origin=np.tile(org, (len(imgs), 1)))
    thr = T(1.0e6 + np.arange(-20.0, 20.25, 0.5))
    d = np.array([[1.0, 0.0], [1.0, 1e-9], [1.0, -1e-9], [1.0, 2e-9]])   # x_0 = 1e6 + k_0 against the grid
    assert _uses_batch_kernel(A, N, plan, d, thr)
    got = plan.ect(T(d), thr).cpu().numpy().reshape(len(imgs), len(d), -1)
    for i in range(0, len(imgs), 37):
        assert np.array_equal(got[i], O.ect(imgs[i], d, thr.cpu().numpy(), origin=org)), i
