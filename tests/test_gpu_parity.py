"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Bar: critical lists and the ECT bit-exact; hybrid transforms within the gates
of tests/gates.py; gradients within the same gates.  Inputs are seeded; sizes
span several tiles with ragged tails, plus the degenerate cases.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_02256_amd import workloads as W

from oracle.gates import combine_rss, fp32_gate, fp64_gate, grad_gate, grad_scales, laplace_shifted, term_scales

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_02256_amd import api as A
    return A


def dev():
    return torch.device("cuda:0")


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def _oracle_lists(img, construction):
    lw, od = O.critical_values(img, construction)
    n = img.ndim
    V = list(reversed(O.vertex_shape(img, construction)))
    ks = np.array(np.meshgrid(*[np.arange(v) for v in V], indexing="ij")).reshape(n, -1).T
    ks = ks[np.lexsort(ks.T)]
    out = []
    for e in range(1 << n):
        nz = np.nonzero(lw[:, e])[0]
        out.append(("c", e, ks[nz], lw[nz, e]))
    for e in range(1 << (n - 1)):
        nz = np.nonzero(od[:, e])[0]
        out.append(("o", e, ks[nz], od[nz, e]))
    return out


def _check_lists(plan, imgs, construction):
    for i, img in enumerate(imgs):
        for kind, e, ks, vals in _oracle_lists(img, construction):
            coords, v = plan.export(i, 0 if kind == "c" else 1, e)
            assert coords.shape[0] == ks.shape[0], (i, kind, e)
            assert np.array_equal(coords, ks), (i, kind, e)
            assert np.array_equal(v, vals), (i, kind, e)


# ---------------------------------------------------------------------------
# a1-a3: classification and ordered compaction
# ---------------------------------------------------------------------------

def test_running_example_table2(api):
    img = W.RUNNING_EXAMPLE
    plan = api.Plan(T(img), construction=1)
    _check_lists(plan, [img], O.DUAL)
    assert plan.check() == 0


@pytest.mark.parametrize("construction", [O.PRIMAL, O.DUAL])
def test_lists_random_2d_3d_ragged_batch(api, construction):
    rng = np.random.default_rng(101)
    shapes2 = [(1, 1), (1, 7), (5, 3), (33, 70), (64, 64), (40, 129)]
    imgs = [W.random_image(rng, s, 4) for s in shapes2]
    plan = api.Plan([T(im) for im in imgs], construction=construction)
    _check_lists(plan, imgs, construction)
    shapes3 = [(1, 1, 1), (3, 4, 5), (17, 9, 30), (2, 33, 16)]
    imgs3 = [W.random_image(rng, s, 3) for s in shapes3]
    plan3 = api.Plan([T(im) for im in imgs3], construction=construction)
    _check_lists(plan3, imgs3, construction)


def test_lists_exhaustive_binary_3x3_and_2x2x2(api):
    imgs = list(W.all_binary_images((3, 3)))
    plan = api.Plan([T(im) for im in imgs], construction=O.PRIMAL)
    _check_lists(plan, imgs, O.PRIMAL)
    imgs3 = list(W.all_binary_images((2, 2, 2)))
    for cons in (O.PRIMAL, O.DUAL):
        plan = api.Plan([T(im) for im in imgs3], construction=cons)
        _check_lists(plan, imgs3, cons)


def test_lists_small_binary_and_int_dtypes(api):
    w = W.small_binary(1)
    img = w.images[0]
    plan = api.Plan(T(img))
    _check_lists(plan, [img], O.PRIMAL)
    rng = np.random.default_rng(7)
    big = rng.integers(-300, 300, size=(37, 41)).astype(np.int16)
    plan16 = api.Plan(T(big))
    _check_lists(plan16, [big.astype(np.int32)], O.PRIMAL)
    big32 = rng.integers(-100000, 100000, size=(12, 9, 10)).astype(np.int32)
    plan32 = api.Plan(T(big32), construction=O.DUAL)
    _check_lists(plan32, [big32], O.DUAL)


def test_list_counts_and_invariants_grf(api):
    w = W.grf_512(2, n_xi=8)
    img = w.images[0]
    plan = api.Plan(T(img))
    c, o = plan.counts()
    lw, od = O.critical_values(img, O.PRIMAL)
    assert c[0].tolist() == [int(np.count_nonzero(lw[:, e])) for e in range(4)]
    assert o[0].tolist() == [int(np.count_nonzero(od[:, e])) for e in range(2)]
    chi = O.euler_characteristic(img, O.PRIMAL)
    for e in range(4):
        _, v = plan.export(0, 0, e)
        assert v.sum() == chi
    for e in range(2):
        _, v = plan.export(0, 1, e)
        assert v.sum() == 0


# ---------------------------------------------------------------------------
# a4-a5: ECT, bit-exact
# ---------------------------------------------------------------------------

def test_ect_running_example_paper_values(api):
    img = W.RUNNING_EXAMPLE
    plan = api.Plan(T(img), construction=O.DUAL, origin=[-0.5, -0.5], spacing=[1 / 3, 1 / 3])
    out = plan.ect(T(np.array([[2.0, 2.0]])), T(np.array([-2.0, -1.0, 0.0, 1.0, 2.0])))
    assert out.cpu().numpy()[0].tolist() == [1, 1, 2, 2, 2]


def test_ect_small_binary_full(api):
    w = W.small_binary(1)
    img = w.images[0]
    plan = api.Plan(T(img))
    got = plan.ect(T(w.ect_dirs), T(w.ect_thresholds)).cpu().numpy()
    assert np.array_equal(got, O.ect(img, w.ect_dirs, w.ect_thresholds))


@pytest.mark.parametrize("ragged", [False, True])
def test_ect_non_finite_directions(api, ragged):
    """A NaN or infinite direction gets a zero row and raises the non-finite
    flag; every other row stays exact (shared sets skip bucketing, ragged sets
    are bucketed: both paths)."""
    rng = np.random.default_rng(31)
    imgs = [W.random_image(rng, (21, 17), 4), W.random_image(rng, (9, 30), 4)]
    dirs = W.circle_dirs(12)
    dirs[3] = [np.nan, 1.0]
    dirs[7] = [np.inf, -0.5]
    thr = W.even_thresholds(25.0, 30)
    plan = api.Plan([T(im) for im in imgs])
    if ragged:
        d = np.concatenate([dirs, dirs[:5]])
        offs = np.array([0, 12, 17], np.int64)
        got = plan.ect(T(d), T(thr), offsets=T(offs)).cpu().numpy()
        parts = [(0, dirs, got[:12]), (1, dirs[:5], got[12:])]
    else:
        got = plan.ect(T(dirs), T(thr)).cpu().numpy().reshape(2, 12, -1)
        parts = [(0, dirs, got[0]), (1, dirs, got[1])]
    for i, dd, g in parts:
        fin = np.isfinite(dd).all(axis=1)
        assert (g[~fin] == 0).all()
        assert np.array_equal(g[fin], O.ect(imgs[i], dd[fin], thr)), i
    assert plan.check() & 0x4


def test_rerun_on_new_contents_many_times(api):
    """Re-runs reuse the look-back words of the previous run (no reset launch):
    alternate three images of one shape through one plan, a ragged batch of
    several tiles per image, and check the ECT and a hybrid transform after
    every re-run."""
    rng = np.random.default_rng(4242)
    shapes = [(70, 90), (33, 47), (64, 64)]
    sets = [[W.binary_field(rng, sh, 2.5) if k % 2 else W.random_image(rng, sh, 5).astype(np.uint8)
             for sh in shapes] for k in range(3)]
    dirs = W.circle_dirs(24)
    thr = W.even_thresholds(60.0, 40)
    xi = W.polar_vectors(rng, 40, 0.02, 1.0)
    plan = api.Plan([T(im) for im in sets[0]])
    for it in range(7):
        cur = sets[it % 3]
        for off, im in zip(plan.pixel_offsets, cur):
            plan.pixels[int(off):int(off) + im.size].copy_(T(im).reshape(-1))
        plan.rerun()
        got = plan.ect(T(dirs), T(thr)).cpu().numpy().reshape(len(cur), len(dirs), -1)
        for i, im in enumerate(cur):
            assert np.array_equal(got[i], O.ect(im, dirs, thr)), (it, i)
        y = plan.hybrid(T(xi), "fourier", 1.0, "fp64").cpu().numpy().reshape(len(cur), len(xi), 2)
        for i, im in enumerate(cur):
            ref = O.hybrid(im, xi, "fourier", 1.0)
            S1, _ = term_scales(im, xi, "fourier", 1.0)
            ok, ratio = fp64_gate(y[i, :, 0] + 1j * y[i, :, 1], ref, S1)
            assert ok, (it, i, ratio)
    assert plan.check() == 0


@pytest.mark.parametrize("construction", [O.PRIMAL, O.DUAL])
def test_ect_random_with_axis_and_signed_zero_dirs(api, construction):
    rng = np.random.default_rng(202)
    for shape in [(20, 31), (9, 12, 7)]:
        img = W.random_image(rng, shape, 5)
        n = img.ndim
        dirs = rng.standard_normal((37, n))
        dirs[0] = 0.0
        dirs[1, 0] = -0.0
        dirs[2, :] = 0.0
        dirs[2, 0] = 1.0
        dirs[3, :] = -0.0
        dirs[3, -1] = -1.0
        R = float(np.linalg.norm(shape))
        thr = np.sort(np.concatenate([rng.uniform(-R, R, 50), [0.0, 0.0, 0.5, -0.5]]))
        plan = api.Plan(T(img), construction=construction)
        got = plan.ect(T(dirs), T(thr)).cpu().numpy()
        assert np.array_equal(got, O.ect(img, dirs, thr, construction))


def test_ect_ragged_batch_per_image_thresholds_and_dirs(api):
    rng = np.random.default_rng(303)
    sides = [28, 64, 5, 128, 1, 64]
    imgs = [W.binary_field(rng, (s, s), 3.0) if s > 4 else W.random_image(rng, (s, s), 2) for s in sides]
    plan = api.Plan([T(im) for im in imgs])
    M = 47
    thr = np.stack([W.even_thresholds(s / np.sqrt(2), M) for s in sides])
    counts = [5, 0, 17, 9, 3, 40]
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    dirs = rng.standard_normal((offs[-1], 2))
    got = plan.ect(T(dirs), T(thr), offsets=T(offs)).cpu().numpy()
    for i, im in enumerate(imgs):
        ref = O.ect(im, dirs[offs[i]:offs[i + 1]], thr[i]) if counts[i] else np.zeros((0, M), np.int32)
        assert np.array_equal(got[offs[i]:offs[i + 1]], ref), i
    # shared set for every image
    sd = W.circle_dirs(12)
    got = plan.ect(T(sd), T(thr)).cpu().numpy().reshape(len(imgs), 12, M)
    for i, im in enumerate(imgs):
        assert np.array_equal(got[i], O.ect(im, sd, thr[i])), i


def test_ect_grf512_full_config(api):
    """All 360 x 256 ECT values of the 512 x 512 field, element by element."""
    w = W.grf_512(2, n_xi=8)
    img = w.images[0]
    plan = api.Plan(T(img))
    got = plan.ect(T(w.ect_dirs), T(w.ect_thresholds)).cpu().numpy()
    assert np.array_equal(got, O.ect(img, w.ect_dirs, w.ect_thresholds))


def test_ect_large_threshold_count(api):
    rng = np.random.default_rng(404)
    img = W.random_image(rng, (30, 30), 3)
    thr = np.linspace(-25, 25, 4096)
    dirs = rng.standard_normal((10, 2))
    plan = api.Plan(T(img))
    got = plan.ect(T(dirs), T(thr)).cpu().numpy()
    assert np.array_equal(got, O.ect(img, dirs, thr))


def test_ect_unsorted_thresholds_flag(api):
    img = W.small_binary(1).images[0]
    plan = api.Plan(T(img))
    thr = np.array([0.0, 1.0, 0.5, 2.0])
    out = plan.ect(T(W.circle_dirs(4)), T(thr)).cpu().numpy()
    assert (out == 0).all()
    assert plan.check() & 0x2
    assert plan.check() == 0


# ---------------------------------------------------------------------------
# a6: hybrid transforms
# ---------------------------------------------------------------------------

def _cplx(y, kernel):
    y = np.asarray(y)
    return y[:, 0] + 1j * y[:, 1] if kernel == "fourier" else y


@pytest.mark.parametrize("kernel", ["fourier", "laplace", "bessel"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_hybrid_small_binary(api, kernel, precision):
    w = W.small_binary(1)
    img = w.images[0]
    plan = api.Plan(T(img))
    y = _cplx(plan.hybrid(T(w.hybrid_xi), kernel, 1.0, precision).cpu().numpy(), kernel)
    ref = O.hybrid(img, w.hybrid_xi, kernel, 1.0)
    S1, S2 = term_scales(img, w.hybrid_xi, kernel, 1.0)
    if precision == "fp32":
        ok, ratio, norm, strict = fp32_gate(y, ref, S2)
        assert ok, (ratio, norm, strict)
    else:
        ok, ratio = fp64_gate(y, ref, S1)
        assert ok, ratio


@pytest.fixture(scope="module")
def grf512_step(api):
    """The 512 x 512 field's step as the benchmark launches it: ECT and the fused Fourier + Laplace +
    Bessel pass in one call (ECT workgroups inside the hybrid launch), FP32."""
    w = W.grf_512(2)
    img = w.images[0]
    plan = api.Plan(T(img))
    plan.set_tuning(0, 2048, 2, 1)
    ect, outs = plan.ect_hybrid_multi(T(w.ect_dirs), T(w.ect_thresholds), T(w.hybrid_xi),
                                      ("fourier", "laplace", "bessel"), 1.0, "fp32")
    assert plan.check() == 0
    return w, plan, ect.cpu().numpy(), {k: v.cpu().numpy() for k, v in outs.items()}


def test_grf512_step_ect_full(grf512_step):
    w, _, ect, _ = grf512_step
    assert np.array_equal(ect, O.ect(w.images[0], w.ect_dirs, w.ect_thresholds))


@pytest.mark.parametrize("kernel", ["fourier", "laplace", "bessel"])
def test_grf512_step_hybrid_full(grf512_step, kernel):
    """All 4096 xi of every kernel against the oracle, per query (Laplace in shifted form)."""
    w, _, _, outs = grf512_step
    img, xi = w.images[0], w.hybrid_xi
    y = _cplx(outs[kernel], kernel)
    if kernel == "laplace":
        ref, m, S2 = laplace_shifted(img, xi, 1.0)
        y = y * np.exp(-m)
    else:
        ref = O.hybrid(img, xi, kernel, 1.0)
        _, S2 = term_scales(img, xi, kernel, 1.0)
    ok, ratio, norm, strict = fp32_gate(y, ref, S2)
    print(f"[grf512 {kernel}] max gate ratio {ratio:.3g}, normwise {norm:.3g}, strict {strict:.3g}")
    assert ok, (ratio, norm, strict)


def test_grf512_step_backward_full(grf512_step):
    """The step's Fourier backward at all 4096 xi against the oracle gradient, per query and component,
    and d/ds."""
    w, plan, _, outs = grf512_step
    img, xi = w.images[0], w.hybrid_xi
    g = np.random.default_rng(22).standard_normal((len(xi), 2))
    gx, gs = plan.hybrid_backward(T(xi), T(outs["fourier"]), T(g), "fourier", 1.0, "fp32")
    gx, gs = gx.cpu().numpy(), float(gs.cpu())
    rgx, rgs = O.hybrid_grad(img, xi, "fourier", 1.0, g)
    S2x, _, S2s, _ = grad_scales(img, xi, "fourier", 1.0, g)
    ok, ratio, norm, strict = grad_gate(gx, rgx, S2x)
    print(f"[grf512 grad] max gate ratio {ratio:.3g}, normwise {norm:.3g}")
    assert ok, (ratio, norm, strict)
    ok, ratio, _, _ = fp32_gate([gs], [rgs], [np.sqrt((S2s ** 2).sum())], normwise=False)
    assert ok, (gs, rgs, ratio)


@pytest.mark.parametrize("construction", [O.PRIMAL, O.DUAL])
@pytest.mark.parametrize("kernel", ["fourier", "laplace", "bessel"])
def test_hybrid_3d_and_dual(api, kernel, construction):
    rng = np.random.default_rng(505)
    img = W.quantised_volume(rng, 20, 2.0)
    xi = W.sphere_vectors(rng, 100, 0.01, 2.0)
    plan = api.Plan(T(img), construction=construction, origin=[0.0, 0.0, 0.0])
    org = np.zeros(3)
    for precision in ("fp32", "fp64"):
        y = _cplx(plan.hybrid(T(xi), kernel, 0.8, precision).cpu().numpy(), kernel)
        ref = O.hybrid(img, xi, kernel, 0.8, construction, origin=org)
        S1, S2 = term_scales(img, xi, kernel, 0.8, construction, origin=org)
        if precision == "fp32":
            ok, ratio, norm, strict = fp32_gate(y, ref, S2)
            assert ok, (precision, ratio, norm, strict)
        else:
            ok, ratio = fp64_gate(y, ref, S1)
            assert ok, (precision, ratio)


def test_laplace_log_scale_large_phases(api):
    rng = np.random.default_rng(606)
    img = W.quantised_volume(rng, 24, 2.0)
    xi = W.sphere_vectors(rng, 64, 0.5, 20.0)    # phases up to ~800: exp overflows FP64 unshifted
    plan = api.Plan(T(img), origin=[0.0, 0.0, 0.0])
    out, ls = plan.hybrid(T(xi), "laplace", 1.0, "fp32", log_scale=True)
    out, ls = out.cpu().numpy(), ls.cpu().numpy()
    ref, m = O.hybrid(img, xi, "laplace", 1.0, origin=np.zeros(3), with_shift=True)
    y = out * np.exp(ls - m)
    S1, S2 = term_scales(img, xi, "laplace", 1.0, origin=np.zeros(3), shift=m)
    ok, ratio, norm, strict = fp32_gate(y, ref, S2)
    assert ok, (ratio, norm, strict)


def test_hybrid_ragged_batch_and_signs(api):
    rng = np.random.default_rng(707)
    sides = [28, 64, 1, 100]
    imgs = [W.binary_field(rng, (s, s), 4.0) if s > 1 else np.ones((1, 1), np.uint8) for s in sides]
    plan = api.Plan([T(im) for im in imgs])
    counts = [70, 3, 5, 130]
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    xi = W.polar_vectors(rng, int(offs[-1]), 0.01, 1.0)
    xi[0] = [0.3, 0.0]
    xi[1] = [-0.0, -0.2]
    for kernel in ("fourier", "laplace"):
        y = _cplx(plan.hybrid(T(xi), kernel, 1.0, "fp32", offsets=T(offs)).cpu().numpy(), kernel)
        for i, im in enumerate(imgs):
            sl = slice(offs[i], offs[i + 1])
            ref = O.hybrid(im, xi[sl], kernel, 1.0)
            S1, S2 = term_scales(im, xi[sl], kernel, 1.0)
            ok, ratio, norm, strict = fp32_gate(y[sl], ref, S2)
            assert ok, (kernel, i, ratio, norm)


def test_hybrid_deterministic(api):
    w = W.grf_512(2, n_xi=1024)
    plan = api.Plan(T(w.images[0]))
    for kernel in ("fourier", "laplace", "bessel"):
        a = plan.hybrid(T(w.hybrid_xi), kernel, 1.0, "fp32").cpu().numpy()
        b = plan.hybrid(T(w.hybrid_xi), kernel, 1.0, "fp32").cpu().numpy()
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_empty_lists_and_tiny(api):
    z = np.zeros((16, 16), np.uint8)
    plan = api.Plan(T(z))
    c, o = plan.counts()
    assert c.sum() == 0 and o.sum() == 0
    xi = W.circle_dirs(70) * 0.5
    y = plan.hybrid(T(xi), "fourier", 1.0).cpu().numpy()
    assert (y == 0).all()
    e = plan.ect(T(xi), T(np.linspace(-5, 5, 9))).cpu().numpy()
    assert (e == 0).all()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_fused_multi_kernel_equals_separate_calls(api, precision):
    w = W.grf_512(2, n_xi=2048)
    plan = api.Plan(T(w.images[0]))
    xi = T(w.hybrid_xi)
    for kernels in (("fourier", "laplace", "bessel"), ("fourier", "bessel"), ("laplace", "bessel")):
        multi = plan.hybrid_multi(xi, kernels, 1.0, precision)
        for k in kernels:
            one = plan.hybrid(xi, k, 1.0, precision).cpu().numpy()
            got = multi[k].cpu().numpy()
            assert np.array_equal(got.view(np.uint64), one.view(np.uint64)), (kernels, k)


def test_large_query_sets_use_multi_workgroup_bucketing(api):
    rng = np.random.default_rng(1001)
    img = W.binary_field(rng, (40, 40), 3.0)
    plan = api.Plan(T(img))
    xi = W.polar_vectors(rng, 70000, 0.01, 1.0)          # > 65536 rows: multi-workgroup path
    y = plan.hybrid(T(xi), "fourier", 1.0).cpu().numpy()
    sel = rng.choice(len(xi), 40, replace=False)
    ref = O.hybrid(img, xi[sel], "fourier", 1.0)
    S1, S2 = term_scales(img, xi[sel], "fourier", 1.0)
    ok, ratio, norm, strict = fp32_gate(_cplx(y, "fourier")[sel], ref, S2)
    assert ok, (ratio, norm)
    dirs = W.circle_dirs(70000)
    thr = np.linspace(-30, 30, 16)
    e = plan.ect(T(dirs), T(thr)).cpu().numpy()
    assert np.array_equal(e[sel], O.ect(img, dirs[sel], thr))
    # many (image, bucket) entries: 2100 images x 2 pairs > 4096
    imgs = [W.random_image(rng, (3, 4), 2) for _ in range(2100)]
    planb = api.Plan([T(im) for im in imgs])
    counts = rng.integers(0, 4, size=len(imgs))
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    xib = W.polar_vectors(rng, int(offs[-1]), 0.05, 1.0)
    yb = planb.hybrid(T(xib), "laplace", 1.0, offsets=T(offs)).cpu().numpy()
    for i in rng.choice(len(imgs), 25, replace=False):
        if counts[i] == 0:
            continue
        sl = slice(offs[i], offs[i + 1])
        ref = O.hybrid(imgs[i], xib[sl], "laplace", 1.0)
        S1, S2 = term_scales(imgs[i], xib[sl], "laplace", 1.0)
        ok, ratio, norm, strict = fp32_gate(yb[sl], ref, S2, normwise=False)   # 1-3 queries per image
        assert ok, (i, ratio)


# ---------------------------------------------------------------------------
# a7: backward
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kernel", ["fourier", "laplace", "bessel"])
def test_backward_against_oracle_gradient(api, kernel):
    rng = np.random.default_rng(808)
    imgs = [W.binary_field(rng, (48, 48), 3.0) for _ in range(3)]
    plan = api.Plan([T(im) for im in imgs])
    xi = W.polar_vectors(rng, 40, 0.01, 0.5, axis_gap=0.02)
    y = plan.hybrid(T(xi), kernel, 1.0, "fp32")
    g = rng.standard_normal(tuple(y.shape))
    gxi, gs = plan.hybrid_backward(T(xi), y, T(g), kernel, 1.0, "fp32")
    gxi, gs = gxi.cpu().numpy(), float(gs.cpu())
    rows = g.reshape(len(imgs), 40, *g.shape[1:])
    rgx = np.zeros((40, 2))
    rgs = 0.0
    S2x, S2s = [], []
    for i, im in enumerate(imgs):
        a, b = O.hybrid_grad(im, xi, kernel, 1.0, rows[i])
        rgx += a
        rgs += b
        sx, _, ss, _ = grad_scales(im, xi, kernel, 1.0, rows[i])
        S2x.append(sx)
        S2s.append(ss)
    ok, ratio, norm, strict = grad_gate(gxi, rgx, combine_rss(*S2x))
    assert ok, (ratio, norm, strict)
    ok, ratio, _, _ = fp32_gate([gs], [rgs], [np.sqrt((combine_rss(*S2s) ** 2).sum())], normwise=False)
    assert ok, (gs, rgs, ratio)
    # FP64 backward: every component within 1e-11 of its terms' sum
    y64 = plan.hybrid(T(xi), kernel, 1.0, "fp64")
    gx64, gs64 = plan.hybrid_backward(T(xi), y64, T(g), kernel, 1.0, "fp64")
    S1x = sum(grad_scales(im, xi, kernel, 1.0, rows[i])[1] for i, im in enumerate(imgs))
    S1s = sum(grad_scales(im, xi, kernel, 1.0, rows[i])[3].sum() for i, im in enumerate(imgs))
    ok, ratio = fp64_gate(gx64.cpu().numpy(), rgx, S1x)
    assert ok, ratio
    ok, ratio = fp64_gate([float(gs64.cpu())], [rgs], [S1s])
    assert ok, ratio


def test_autograd_function_matches_finite_differences(api):
    rng = np.random.default_rng(909)
    imgs = [W.binary_field(rng, (32, 32), 3.0) for _ in range(2)]
    plan = api.Plan([T(im) for im in imgs])
    xi0 = W.polar_vectors(rng, 8, 0.05, 0.5, axis_gap=0.05)
    xi = T(xi0).clone().requires_grad_(True)
    s = torch.tensor(1.0, dtype=torch.float64, device=dev(), requires_grad=True)
    y = api.HybridTransform.apply(xi, s, plan, "laplace", "fp64")
    wts = T(rng.standard_normal(tuple(y.shape)))
    (y * wts).sum().backward()
    wnp = wts.cpu().numpy().reshape(2, 8)

    def loss(xv, sv):
        return sum(float((O.hybrid(im, xv, "laplace", sv) * wnp[i]).sum()) for i, im in enumerate(imgs))

    h = 1e-3
    for q in range(8):
        for a in range(2):
            xp, xm = xi0.copy(), xi0.copy()
            xp[q, a] += h
            xm[q, a] -= h
            fd = (loss(xp, 1.0) - loss(xm, 1.0)) / (2 * h)
            assert abs(fd - float(xi.grad[q, a])) <= 1e-2 * max(1.0, abs(fd))
    fds = (loss(xi0, 1.0 + h) - loss(xi0, 1.0 - h)) / (2 * h)
    assert abs(fds - float(s.grad)) <= 1e-2 * max(1.0, abs(fds))


@pytest.mark.parametrize("kernel", ["fourier", "laplace"])
def test_autograd_function_fp32_against_oracle_gradient(api, kernel):
    """The FP32 autograd path (float32 xi, learnable s) against the oracle gradient, per query and
    component, and against central differences of the oracle forward."""
    rng = np.random.default_rng(910)
    imgs = [W.binary_field(rng, (40, 40), 3.0) for _ in range(3)]
    plan = api.Plan([T(im) for im in imgs])
    xi0 = W.polar_vectors(rng, 24, 0.05, 0.5, axis_gap=0.05).astype(np.float32)
    xi = torch.from_numpy(xi0).to(dev()).requires_grad_(True)
    s = torch.tensor(0.9, dtype=torch.float64, device=dev(), requires_grad=True)
    y = api.HybridTransform.apply(xi, s, plan, kernel, "fp32")
    wts = rng.standard_normal(tuple(y.shape))
    (y * T(wts)).sum().backward()
    gx, gsv = xi.grad.cpu().numpy().astype(np.float64), float(s.grad.cpu())
    assert xi.grad.dtype == torch.float32
    x64 = xi0.astype(np.float64)
    wr = wts.reshape(len(imgs), 24, *wts.shape[1:])
    rgx = np.zeros((24, 2))
    rgs = 0.0
    S2x, S2s = [], []
    for i, im in enumerate(imgs):
        a, b = O.hybrid_grad(im, x64, kernel, 0.9, wr[i])
        rgx += a
        rgs += b
        sx, _, ss, _ = grad_scales(im, x64, kernel, 0.9, wr[i])
        S2x.append(sx)
        S2s.append(ss)
    ok, ratio, norm, strict = grad_gate(gx, rgx, combine_rss(*S2x))   # float32 rounding: within 1e-5 rel
    assert ok, (ratio, norm, strict)
    ok, ratio, _, _ = fp32_gate([gsv], [rgs], [np.sqrt((combine_rss(*S2s) ** 2).sum())], normwise=False)
    assert ok, (gsv, rgs, ratio)

    def loss(xv, sv):
        tot = 0.0
        for i, im in enumerate(imgs):
            r = O.hybrid(im, xv, kernel, sv)
            r = np.stack([r.real, r.imag], -1) if kernel == "fourier" else r
            tot += float((r * wr[i]).sum())
        return tot

    h = 1e-3
    for q in range(0, 24, 6):
        for a in range(2):
            xp, xm = x64.copy(), x64.copy()
            xp[q, a] += h
            xm[q, a] -= h
            fd = (loss(xp, 0.9) - loss(xm, 0.9)) / (2 * h)
            assert abs(fd - gx[q, a]) <= 1e-2 * max(1.0, abs(fd)), (q, a, fd, gx[q, a])
    fds = (loss(x64, 0.9 + h) - loss(x64, 0.9 - h)) / (2 * h)
    assert abs(fds - gsv) <= 1e-2 * max(1.0, abs(fds)), (fds, gsv)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_laplace_off_centre_object_large_xi(api, precision):
    """An object far from the centre of a 256 x 256 frame at |xi| = 4: every exponent -s<xi,x> of its
    points lies hundreds of units below the frame's extreme vertex, so the shift must follow the
    list's own maximum.  With a log-scale output every query is checked in shifted form; without one,
    queries whose HT is finite are returned unshifted and exactly those that overflow raise the flag.
    Shared and ragged query sets."""
    from paper_2405_02256_amd import _native as N
    rng = np.random.default_rng(1301)
    img = np.zeros((256, 256), np.uint8)
    img[216:256, 0:40] = W.binary_field(rng, (40, 40), 3.0)   # the corner of largest axis 1, smallest axis 0
    img[236:256, 0:20] = 1                  # a solid block at the frame's corner: some HT overflow FP64
    ang = rng.uniform(0, 2 * np.pi, 96)
    xi = 4.0 * np.stack([np.cos(ang), np.sin(ang)], -1)
    xi[:5] = [[4.0, 0.0], [0.0, 4.0], [-4.0, 0.0], [0.0, -4.0], [2.8284271247461903, -2.8284271247461903]]
    plan = api.Plan(T(img))
    ref, m, S2 = laplace_shifted(img, xi, 1.0)
    S1, _ = term_scales(img, xi, "laplace", 1.0, shift=m)
    offs = np.array([0, len(xi)], np.int64)
    for ragged in (False, True):
        kw = dict(offsets=T(offs)) if ragged else {}
        out, ls = plan.hybrid(T(xi), "laplace", 1.0, precision, log_scale=True, **kw)
        out, ls = out.cpu().numpy(), ls.cpu().numpy()
        assert np.isfinite(out).all() and np.isfinite(ls).all()
        # the shift follows the list: the shifted output is O(1), not 0
        assert (np.abs(out) > 0).all() or (np.abs(ref) == 0).any()
        y = out * np.exp(ls - m)
        if precision == "fp32":
            ok, ratio, norm, strict = fp32_gate(y, ref, S2)
            assert ok, (ragged, ratio, norm, strict)
        else:
            ok, ratio = fp64_gate(y, ref, S1)
            assert ok, (ragged, ratio)
        assert plan.check() == 0
        # without a log-scale output
        full = plan.hybrid(T(xi), "laplace", 1.0, precision, **kw).cpu().numpy()
        flags = plan.check()
        loght = np.log(np.abs(ref) + 1e-300) + m           # log |HT|
        finite, over = loght < 705.0, loght > 712.0        # (the few in between may round either way)
        assert finite.sum() > 80 and over.sum() >= 3
        yf = full[finite] * np.exp(-m[finite])
        if precision == "fp32":
            ok, ratio, _, _ = fp32_gate(yf, ref[finite], S2[finite])
        else:
            ok, ratio = fp64_gate(yf, ref[finite], S1[finite])
        assert ok, (ragged, ratio)
        assert not np.isfinite(full[over]).any()
        assert flags & N.DEVERR_OVERFLOW


@pytest.mark.parametrize("construction", [O.PRIMAL, O.DUAL])
def test_hybrid_zero_scale_limit(api, construction):
    """s = 0: every kernel gives the constant-kernel limit sum D <xi, x> (Fourier: real part, imaginary
    0), alone and in the fused pass, on shared and ragged sets; the backward refuses s = 0."""
    from paper_2405_02256_amd import _native as N
    rng = np.random.default_rng(1201)
    imgs = [W.random_image(rng, (23, 19), 4), W.random_image(rng, (7, 9, 6), 3)]
    for img in imgs:
        n = img.ndim
        xi = rng.standard_normal((70, n))
        plan = api.Plan(T(img), construction=construction)
        ref = O.hybrid(img, xi, "laplace", 0.0, construction)
        _, od = O.critical_values(img, construction)
        x = _vertex_coords_np(img, construction)
        S1 = np.array([np.abs(od[:, _sidx(q)] * (x @ q)).sum() for q in xi])
        for kernel in ("fourier", "laplace", "bessel"):
            for precision in ("fp32", "fp64"):
                y = plan.hybrid(T(xi), kernel, 0.0, precision).cpu().numpy()
                if kernel == "fourier":
                    assert (y[:, 1] == 0).all()
                    y = y[:, 0]
                assert (np.abs(y - ref) <= 1e-11 * np.maximum(S1, 1.0)).all(), (kernel, precision)
        outs = plan.hybrid_multi(T(xi), ("fourier", "laplace", "bessel"), 0.0, "fp32")
        assert np.array_equal(outs["fourier"].cpu().numpy()[:, 0], outs["laplace"].cpu().numpy())
        assert np.array_equal(outs["bessel"].cpu().numpy(), outs["laplace"].cpu().numpy())
        y = plan.hybrid(T(xi), "laplace", 0.0, "fp64")
        with pytest.raises(N.EctError):
            plan.hybrid_backward(T(xi), y, T(np.ones(70)), "laplace", 0.0, "fp64")


def _vertex_coords_np(img, construction):
    V = list(reversed(O.vertex_shape(img, construction)))
    o = O.default_origin(img, construction)
    ks = np.array(list(np.ndindex(*reversed(V))))[:, ::-1]
    return ks + o[None, :]


def _sidx(xi):
    return sum(1 << a for a in range(len(xi)) if not (xi[a] >= 0))


@pytest.mark.parametrize("kernel", ["fourier", "bessel"])
def test_hybrid_rows_do_not_depend_on_their_tile(api, kernel):
    """Queries are reordered inside their buckets (sub-bins of |xi| and angle, LDS atomics): a permuted
    query set gives the permuted outputs bit for bit, in both precisions and for the backward."""
    rng = np.random.default_rng(1202)
    img = W.binary_field(rng, (96, 80), 3.0)
    plan = api.Plan(T(img))
    xi = W.polar_vectors(rng, 700, 0.01, 1.0, axis_gap=0.02)
    perm = rng.permutation(len(xi))
    for precision in ("fp32", "fp64"):
        y = plan.hybrid(T(xi), kernel, 1.0, precision).cpu().numpy()
        yp = plan.hybrid(T(xi[perm]), kernel, 1.0, precision).cpu().numpy()
        assert np.array_equal(yp, y[perm]), precision
    y = plan.hybrid(T(xi), kernel, 1.0, "fp32")
    g = rng.standard_normal(tuple(y.shape))
    gx, _ = plan.hybrid_backward(T(xi), y, T(g), kernel, 1.0, "fp32")
    yp = plan.hybrid(T(xi[perm]), kernel, 1.0, "fp32")
    gxp, _ = plan.hybrid_backward(T(xi[perm]), yp, T(g[perm]), kernel, 1.0, "fp32")
    assert np.array_equal(gxp.cpu().numpy(), gx.cpu().numpy()[perm])
