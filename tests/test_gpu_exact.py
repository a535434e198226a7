"""GPU parity of the exact representations (Sec. 4.3): the ECT as (T, E) and
the Radon transform as (T, E', Tc, Ec), built on the GPU by sorting the
projections of the critical points, against the oracle's representations
(bit-exact: T compared by value, E exactly), and their binary-search
evaluation against the oracle's transforms at every vertex projection.
"""
import ctypes

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


def ties(img, xi, construction=O.PRIMAL, origin=None, spacing=None, limit=4096):
    u = np.unique(O.vertex_projections(img, xi, construction, origin, spacing))
    mids = (u[1:] + u[:-1]) / 2 if u.size > 1 else u
    t = np.sort(np.concatenate([u, mids, [u.min() - 1.0, u.max() + 1.0]]))
    if t.size > limit:
        t = t[np.linspace(0, t.size - 1, limit).astype(np.int64)]
    return t


def check_rows(rep, imgs_of_rows, dirs, construction=O.PRIMAL, origin=None, spacing=None):
    rows = rep.to_host()
    assert len(rows) == len(dirs)
    for r, (img, xi) in enumerate(zip(imgs_of_rows, dirs)):
        if rep.kind == 0:
            Tg, Eg = rows[r]
            To, Eo = O.ect_exact(img, xi, construction, origin, spacing)
            assert np.array_equal(Tg, To) and np.array_equal(Eg, Eo), r
        else:
            Tg, Epg, Tcg, Ecg = rows[r]
            To, Epo, Tco, Eco = O.radon_exact(img, xi, construction, origin, spacing)
            assert np.array_equal(Tg, To) and np.array_equal(Epg, Epo), r
            assert np.array_equal(Tcg, Tco) and np.array_equal(Ecg, Eco), r


def test_exact_running_example(api):
    img = W.RUNNING_EXAMPLE
    o, h = [-0.5, -0.5], [1 / 3, 1 / 3]
    plan = api.Plan(T(img), construction=O.DUAL, origin=o, spacing=h)
    dirs = np.array([[2.0, 2.0], [1.0, -0.5], [-1.0, 0.0], [0.0, -3.0]])
    for kind in ("ect", "radon"):
        rep = plan.exact(T(dirs), kind)
        check_rows(rep, [img] * len(dirs), dirs, O.DUAL, o, h)
        for r, xi in enumerate(dirs):
            t = ties(img, xi, O.DUAL, o, h)
            ref = (O.ect if kind == "ect" else O.radon)(img, xi[None], t, O.DUAL, o, h)[0]
            got = rep.eval(T(np.tile(t, (len(dirs), 1)))).cpu().numpy()[r]
            assert np.array_equal(got, ref), (kind, r)


@pytest.mark.parametrize("construction", [O.PRIMAL, O.DUAL])
@pytest.mark.parametrize("kind", ["ect", "radon"])
def test_exact_random_2d_3d(api, construction, kind):
    rng = np.random.default_rng(901)
    for shape in [(33, 29), (10, 13, 9)]:
        img = W.random_image(rng, shape, 6)
        n = img.ndim
        dirs = np.concatenate([rng.standard_normal((9, n)), np.eye(n), -np.eye(n),
                               np.round(rng.standard_normal((4, n)) * 2) / 2, np.full((1, n), -0.0)])
        plan = api.Plan(T(img), construction=construction)
        rep = plan.exact(T(dirs), kind)
        check_rows(rep, [img] * len(dirs), dirs, construction)
        # evaluation at each row's own vertex projections, per-row thresholds
        tl = [ties(img, xi, construction, limit=600) for xi in dirs]
        M = min(t.size for t in tl)
        thr = np.stack([t[np.linspace(0, t.size - 1, M).astype(np.int64)] for t in tl])
        got = rep.eval(T(thr)).cpu().numpy()
        fn = O.ect if kind == "ect" else O.radon
        for r, xi in enumerate(dirs):
            assert np.array_equal(got[r], fn(img, xi[None], thr[r], construction)[0]), r


def test_exact_ragged_batch_and_degenerate_images(api):
    rng = np.random.default_rng(902)
    imgs = [W.binary_field(rng, (40, 40), 3.0), np.zeros((6, 7), np.uint8), W.random_image(rng, (1, 1), 3),
            W.binary_field(rng, (64, 30), 2.0).astype(np.uint8), np.full((3, 3), 5, np.int32)]
    imgs = [im.astype(np.int32) for im in imgs]
    plan = api.Plan([T(im) for im in imgs])
    counts = [6, 3, 0, 11, 2]
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    dirs = rng.standard_normal((offs[-1], 2))
    dirs[::4] = np.round(dirs[::4])
    img_of = [imgs[i] for i in range(len(imgs)) for _ in range(counts[i])]
    for kind in ("ect", "radon"):
        rep = plan.exact(T(dirs), kind, offsets=T(offs))
        check_rows(rep, img_of, dirs)
    # shared set over the batch
    sd = np.concatenate([W.circle_dirs(6), np.eye(2)])
    for kind in ("ect", "radon"):
        rep = plan.exact(T(sd), kind)
        check_rows(rep, [im for im in imgs for _ in range(len(sd))], np.tile(sd, (len(imgs), 1)))
    assert plan.check() == 0


def test_exact_eval_matches_threshold_kernels_grf512(api):
    """Full 512 x 512 field, 360 directions: the binary-search evaluation of
    both representations equals the threshold kernels (ect_eval, radon_eval)
    on every row, and sampled rows equal the oracle's representations."""
    w = W.grf_512(2, n_xi=8)
    img = w.images[0]
    plan = api.Plan(T(img))
    dirs, t = w.ect_dirs, w.ect_thresholds
    for kind in ("ect", "radon"):
        rep = plan.exact(T(dirs), kind)
        ref = (plan.ect if kind == "ect" else plan.radon)(T(dirs), T(t)).cpu().numpy()
        assert np.array_equal(rep.eval(T(t)).cpu().numpy(), ref), kind
        sel = np.arange(0, len(dirs), 40)
        rows = rep.to_host()
        for r in sel:
            got = rows[r]
            exp = O.ect_exact(img, dirs[r]) if kind == "ect" else O.radon_exact(img, dirs[r])
            for g, e in zip(got, exp):
                assert np.array_equal(g, e), (kind, r)


def test_exact_non_finite_direction(api):
    rng = np.random.default_rng(903)
    img = W.random_image(rng, (12, 15), 4)
    plan = api.Plan(T(img))
    dirs = np.array([[1.0, 0.3], [np.nan, 1.0], [-0.2, 0.9]])
    for kind in ("ect", "radon"):
        rep = plan.exact(T(dirs), kind)
        rows = rep.to_host()
        assert rows[1][0].tolist() == [-np.inf] and rows[1][1].tolist() == [0]
        if kind == "radon":
            assert rows[1][2].size == 0
        check_rows_sub = [(0, dirs[0]), (2, dirs[2])]
        for r, xi in check_rows_sub:
            exp = O.ect_exact(img, xi) if kind == "ect" else O.radon_exact(img, xi)
            for g, e in zip(rows[r], exp):
                assert np.array_equal(g, e), (kind, r)
        assert plan.check() & 0x4


def test_exact_rejects_offsets_without_room(api):
    """Offsets that leave a row less room than the layout gives, or reach past
    the capacity, are caught on the device: those rows get length 0 and the
    layout flag, the other rows stay exact."""
    from paper_2405_02256_amd import _native as N
    rng = np.random.default_rng(904)
    img = W.random_image(rng, (20, 20), 5)
    plan = api.Plan(T(img))
    dirs = rng.standard_normal((5, 2))
    good = plan.exact(T(dirs), "ect")
    off = good.row_off.clone()
    off[2] = off[3] - 1          # row 2 loses room (row 1 gains some)
    cap = int(off[5].item()) - 1  # row 4 reaches past the capacity
    Tt = torch.empty(cap, dtype=torch.float64, device="cuda:0")
    Et = torch.empty(cap, dtype=torch.int32, device="cuda:0")
    Lt = torch.empty(5, dtype=torch.int64, device="cuda:0")
    q = api.QuerySet(T(dirs))
    st = torch.cuda.current_stream().cuda_stream
    need = ctypes.c_size_t(0)
    N.check(N.ect_exact(plan.handle, q.c(), N.EXACT_ECT, off.data_ptr(), cap, Tt.data_ptr(), Et.data_ptr(),
                        Lt.data_ptr(), None, need, st), "size")
    ws = torch.empty(max(need.value, 256), dtype=torch.uint8, device="cuda:0")
    have = ctypes.c_size_t(ws.numel())
    N.check(N.ect_exact(plan.handle, q.c(), N.EXACT_ECT, off.data_ptr(), cap, Tt.data_ptr(), Et.data_ptr(),
                        Lt.data_ptr(), ctypes.c_void_p(ws.data_ptr()), have, st), "ect_exact")
    L = Lt.cpu().numpy()
    assert L[2] == 0 and L[4] == 0
    o = off.cpu().numpy()
    for r in (0, 1, 3):
        To, Eo = O.ect_exact(img, dirs[r])
        assert L[r] == To.size
        assert np.array_equal(Tt[o[r]:o[r] + L[r]].cpu().numpy(), To)
        assert np.array_equal(Et[o[r]:o[r] + L[r]].cpu().numpy(), Eo)
    assert plan.check() & N.DEVERR_LAYOUT


def test_exact_near_ties_in_fp32_and_long_lists(api):
    """Directions whose projections differ below FP32 resolution (the tiles
    fall back to the exact 64-bit order) and lists of 16k-26k points (several
    sorted tiles merged in the workspace, an odd number of runs included)."""
    rng = np.random.default_rng(905)
    img = W.random_image(rng, (200, 200), 8)
    dirs = np.array([[1.0, 1e-13], [1e-13, -1.0], [0.5, 0.5 + 1e-12], [-0.7, 0.3], [1.0, 0.0], [0.0, 0.0]])
    plan = api.Plan(T(img))
    for kind in ("ect", "radon"):
        rep = plan.exact(T(dirs), kind)
        check_rows(rep, [img] * len(dirs), dirs)
    small = W.random_image(rng, (40, 37), 5)
    plan2 = api.Plan(T(small))
    d2 = np.array([[1.0, 3e-14], [2e-15, 1.0], [-1.0, -1e-12], [0.0, 0.0]])
    for kind in ("ect", "radon"):
        check_rows(plan2.exact(T(d2), kind), [small] * len(d2), d2)
    # one LDS tile whose projections crowd into few buckets (a narrow image
    # seen almost along its long axis: about 21 distinct coordinates), next to
    # directions whose buckets hold a few points each
    narrow = W.random_image(rng, (300, 20), 3)
    plan3 = api.Plan(T(narrow))
    d3 = np.array([[1e-13, 1.0], [-1e-13, -1.0], [1.0, 1e-13], [0.3, -0.8], [0.0, 0.0]])
    for kind in ("ect", "radon"):
        check_rows(plan3.exact(T(d3), kind), [narrow] * len(d3), d3)


def test_exact_representation_is_strictly_increasing_grf512(api):
    w = W.grf_512(2, n_xi=8)
    plan = api.Plan(T(w.images[0]))
    for kind in ("ect", "radon"):
        for row in plan.exact(T(w.ect_dirs), kind).to_host():
            assert np.all(np.diff(row[0]) > 0)
            if kind == "radon":
                assert np.all(np.diff(row[2]) > 0)
