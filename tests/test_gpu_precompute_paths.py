"""The compaction paths of large plans (more than 64 x 64 tiles: count, scan,
write).  With 8- and 16-bit pixels the count pass leaves each tile's entries
packed in per-tile slots (value and vertex index in one 32-bit word) and the
last pass only places them; 32-bit pixels classify every vertex again.  Both
must give the oracle's lists exactly (Sec. 4.2: every nonzero critical value,
in vertex order), including 16-bit extremes whose critical values are the
largest the packed field has to hold, on two, three and four axes.
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


def tiles_of(imgs):
    per = 256 if imgs[0].ndim == 4 else 1024
    return sum(-(-int(np.prod([s + 1 for s in im.shape])) // per) for im in imgs)


def check_lists(plan, i, img, construction=O.PRIMAL):
    lw, od = O.critical_values(img, construction)
    n = img.ndim
    V = list(reversed(O.vertex_shape(img, construction)))
    ks = np.array(np.meshgrid(*[np.arange(v) for v in V], indexing="ij")).reshape(n, -1).T
    ks = ks[np.lexsort(ks.T)]
    for kind, vals in ((0, lw), (1, od[:, :1 << (n - 1)])):
        for e in range(vals.shape[1]):
            nz = np.nonzero(vals[:, e])[0]
            coords, v = plan.export(i, kind, e)
            assert np.array_equal(coords, ks[nz]) and np.array_equal(v, vals[nz, e]), (i, kind, e)


def test_packed_2d_u8_and_recomputed_int32_agree_with_the_oracle(api):
    rng = np.random.default_rng(1201)
    imgs = [W.binary_field(rng, (127, 129), float(rng.uniform(2, 6))).astype(np.uint8) for _ in range(300)]
    assert tiles_of(imgs) > 64 * 64
    p8 = api.Plan([T(im) for im in imgs])
    p32 = api.Plan([T(im.astype(np.int32)) for im in imgs])
    c8, o8 = p8.counts()
    c32, o32 = p32.counts()
    assert np.array_equal(c8, c32) and np.array_equal(o8, o32)
    for i in rng.choice(len(imgs), 4, replace=False):
        check_lists(p8, int(i), imgs[i])
        check_lists(p32, int(i), imgs[i])
    dirs = W.circle_dirs(16)
    thr = np.linspace(-100, 100, 64)
    assert np.array_equal(p8.ect(T(dirs), T(thr)).cpu().numpy(), p32.ect(T(dirs), T(thr)).cpu().numpy())
    assert p8.check() == 0 and p32.check() == 0


def test_packed_3d_u8_dual(api):
    rng = np.random.default_rng(1202)
    imgs = [W.random_image(rng, (24, 23, 22), 5).astype(np.uint8) for _ in range(300)]
    assert tiles_of(imgs) > 64 * 64
    plan = api.Plan([T(im) for im in imgs], construction=O.DUAL)
    for i in rng.choice(len(imgs), 3, replace=False):
        check_lists(plan, int(i), imgs[i], O.DUAL)
    assert plan.check() == 0


def test_packed_4d_int16_extremes(api):
    """16-bit pixels at both ends of their range: the critical values reach the
    packed field's bound (16 cells of +-32767 on either side of a difference)."""
    rng = np.random.default_rng(1203)
    lo, hi = np.iinfo(np.int16).min, np.iinfo(np.int16).max
    imgs = [np.where(rng.random((5, 5, 5, 5)) < 0.5, lo, hi).astype(np.int16) for _ in range(700)]
    assert tiles_of(imgs) > 64 * 64
    plan = api.Plan([T(im) for im in imgs])
    for i in rng.choice(len(imgs), 3, replace=False):
        check_lists(plan, int(i), imgs[i])
    # the same images as 32-bit pixels (classified again in the last pass)
    plan32 = api.Plan([T(im.astype(np.int32)) for im in imgs])
    c, o = plan.counts()
    c32, o32 = plan32.counts()
    assert np.array_equal(c, c32) and np.array_equal(o, o32)
    for i in rng.choice(len(imgs), 2, replace=False):
        for kind, nl in ((0, 16), (1, 8)):
            for e in range(nl):
                a, va = plan.export(int(i), kind, e)
                b, vb = plan32.export(int(i), kind, e)
                assert np.array_equal(a, b) and np.array_equal(va, vb)
    assert plan.check() == 0
