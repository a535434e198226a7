"""The combined call ect_hybrid_eval_multi: the ECT at thresholds and the
fused hybrid transforms from one call, the ECT workgroups inside the hybrid
launch where the call allows it.  Every output must equal the separate calls
(ect_eval, hybrid_eval_multi) bit for bit, in the one-launch cases (shared
direction sets, one or two directions per workgroup, one or several list
chunks, several images, two to four axes, both precisions) and in the cases
that fall back to two launches (ragged sets, more directions per workgroup,
long threshold arrays, s = 0); the ECT rows are also checked against the
oracle, and a backward call reusing the combined call's buckets against one
after the separate forward.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_02256_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KERNELS = ("fourier", "laplace", "bessel")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_02256_amd import api as A
    return A


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))


def compare(plan, dirs, thr, xi, kernels, s=1.0, precision="fp32", dir_offsets=None, xi_offsets=None):
    e_sep = plan.ect(dirs, thr, offsets=dir_offsets).cpu().numpy()
    h_sep = {k: v.cpu().numpy() for k, v in plan.hybrid_multi(xi, kernels, s, precision, offsets=xi_offsets).items()}
    e_one, h_one = plan.ect_hybrid_multi(dirs, thr, xi, kernels, s, precision, dir_offsets=dir_offsets,
                                         xi_offsets=xi_offsets)
    assert np.array_equal(e_one.cpu().numpy(), e_sep)
    for k in kernels:
        assert np.array_equal(h_one[k].cpu().numpy(), h_sep[k]), k
    assert plan.check() == 0
    return e_sep


@pytest.mark.parametrize("td,chunks", [(1, 1), (1, 3), (2, 0), (2, 5)])
def test_one_launch_2d_matches_separate_calls_and_oracle(api, td, chunks):
    rng = np.random.default_rng(1101)
    img = W.binary_field(rng, (96, 80), 3.0).astype(np.int32)
    plan = api.Plan(T(img))
    plan.set_tuning(ect_dirs_per_group=td, ect_chunks=chunks)
    dirs = np.concatenate([W.circle_dirs(37), np.eye(2), [[np.nan, 1.0]]])
    thr = np.linspace(-70, 70, 150)
    xi = rng.standard_normal((300, 2)) * 0.5
    dt = T(dirs)
    e_sep = plan.ect(dt, T(thr)).cpu().numpy()
    # the non-finite direction raises its flag in both calls
    assert plan.check() & 0x4
    e_one, h_one = plan.ect_hybrid_multi(dt, T(thr), T(xi), KERNELS)
    assert plan.check() & 0x4
    h_sep = plan.hybrid_multi(T(xi), KERNELS)
    assert np.array_equal(e_one.cpu().numpy(), e_sep)
    for k in KERNELS:
        assert np.array_equal(h_one[k].cpu().numpy(), h_sep[k].cpu().numpy()), k
    fin = dirs[:-1]
    assert np.array_equal(e_sep[:-1], O.ect(img, fin, thr))
    assert (e_sep[-1] == 0).all()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_one_launch_batch_three_axes(api, precision):
    rng = np.random.default_rng(1102)
    imgs = [W.random_image(rng, (14, 11, 9), 4), W.random_image(rng, (6, 7, 5), 3), W.random_image(rng, (1, 1, 1), 2)]
    plan = api.Plan([T(im) for im in imgs])
    plan.set_tuning(ect_dirs_per_group=1, ect_chunks=2)
    dirs = rng.standard_normal((21, 3))
    dirs[3] = [0.0, 0.0, -1.0]
    thr = np.sort(rng.uniform(-25, 25, 90))
    xi = rng.standard_normal((130, 3)) * 0.3
    for kernels in (KERNELS, ("laplace",), ("fourier", "bessel")):
        e = compare(plan, T(dirs), T(thr), T(xi), kernels, 0.8, precision)
    for i, im in enumerate(imgs):
        assert np.array_equal(e[i * 21:(i + 1) * 21], O.ect(im, dirs, thr))


def test_one_launch_four_axes_per_image_thresholds(api):
    rng = np.random.default_rng(1103)
    imgs = [W.random_image(rng, (5, 4, 6, 3), 3), W.random_image(rng, (4, 4, 4, 4), 3)]
    plan = api.Plan([T(im) for im in imgs])
    plan.set_tuning(ect_dirs_per_group=2)
    dirs = rng.standard_normal((9, 4))
    thr = np.stack([np.linspace(-12, 12, 64), np.linspace(-9, 9, 64)])
    xi = rng.standard_normal((70, 4)) * 0.3
    e = compare(plan, T(dirs), T(thr), T(xi), KERNELS)
    for i, im in enumerate(imgs):
        assert np.array_equal(e[i * 9:(i + 1) * 9], O.ect(im, dirs, thr[i]))


def test_two_launch_cases_match_separate_calls(api):
    rng = np.random.default_rng(1104)
    imgs = [W.random_image(rng, (30, 25), 4), W.random_image(rng, (12, 40), 3)]
    plan = api.Plan([T(im) for im in imgs])
    xi = T(rng.standard_normal((80, 2)) * 0.4)
    dirs = T(rng.standard_normal((15, 2)))
    # default directions per workgroup (eight) on a shared set
    compare(plan, dirs, T(np.linspace(-30, 30, 40)), xi, KERNELS)
    plan.set_tuning(ect_dirs_per_group=1)
    # ragged direction and query sets
    compare(plan, T(rng.standard_normal((11, 2))), T(np.linspace(-30, 30, 40)), T(rng.standard_normal((23, 2))),
            KERNELS, dir_offsets=T(np.array([0, 4, 11], np.int64)), xi_offsets=T(np.array([0, 20, 23], np.int64)))
    # thresholds beyond the one-launch LDS bound
    compare(plan, dirs, T(np.linspace(-30, 30, 1000)), xi, KERNELS)
    # the constant-kernel limit s = 0
    compare(plan, dirs, T(np.linspace(-30, 30, 40)), xi, KERNELS, s=0.0)
    # an empty query set on either side (a view of zero rows keeps a valid pointer)
    empty = T(np.zeros((1, 2)))[:0]
    compare(plan, empty, T(np.linspace(-30, 30, 40)), xi, KERNELS)
    compare(plan, dirs, T(np.linspace(-30, 30, 40)), empty, KERNELS)
    # the backward pass over no rows writes d/ds = 0
    z = torch.zeros((0, 2), dtype=torch.float64, device="cuda:0")
    gs = torch.full((), 7.0, dtype=torch.float64, device="cuda:0")
    plan.hybrid_backward(empty, z, z, "fourier", 1.0, "fp32", grad_s=gs)
    assert float(gs.cpu()) == 0.0


def test_backward_reuses_the_combined_buckets(api):
    rng = np.random.default_rng(1105)
    img = W.random_image(rng, (40, 33), 5)
    plan = api.Plan(T(img))
    plan.set_tuning(ect_dirs_per_group=1)
    dirs = T(W.circle_dirs(24))
    thr = T(np.linspace(-40, 40, 100))
    xi = api.QuerySet(T(rng.standard_normal((90, 2)) * 0.5))
    g = T(rng.standard_normal((90, 2)))
    out = plan.hybrid_multi(xi, KERNELS)["fourier"]
    ref = [t.cpu().numpy() for t in plan.hybrid_backward(xi, out, g, "fourier", 1.0, "fp32")]
    _, h = plan.ect_hybrid_multi(dirs, thr, xi, KERNELS)
    assert np.array_equal(h["fourier"].cpu().numpy(), out.cpu().numpy())
    got = [t.cpu().numpy() for t in plan.hybrid_backward(xi, h["fourier"], g, "fourier", 1.0, "fp32",
                                                         reuse_prepared=True)]
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


def test_step_combined_graph_matches_separate_step(api):
    from paper_2405_02256_amd import pipeline
    rng = np.random.default_rng(1106)
    img = W.binary_field(rng, (128, 128), 4.0).astype(np.int32)
    plan = api.Plan(T(img))
    plan.set_tuning(ect_dirs_per_group=1)
    dirs, thr = T(W.circle_dirs(60)), T(np.linspace(-100, 100, 128))
    xi = T(rng.standard_normal((256, 2)) * 0.5)
    g = T(rng.standard_normal((256, 2)))
    a = pipeline.Step(plan, dirs, thr, xi, kernels=KERNELS, backward_kernel="fourier", grad_out=g, combined=False)
    a.run()
    ref = [a.ect_out.cpu().numpy()] + [a.hy_out[k].cpu().numpy() for k in KERNELS] + [a.grad_xi.cpu().numpy()]
    b = pipeline.Step(plan, dirs, thr, xi, kernels=KERNELS, backward_kernel="fourier", grad_out=g)
    assert b.combined
    b.capture()
    for _ in range(3):
        b.ect_out.zero_()
        b.replay()
        torch.cuda.synchronize()
        got = [b.ect_out.cpu().numpy()] + [b.hy_out[k].cpu().numpy() for k in KERNELS] + [b.grad_xi.cpu().numpy()]
        for x, y in zip(got, ref):
            assert np.array_equal(x, y)


def test_one_launch_with_laplace_log_scale(api):
    """The Laplace output split into a shifted value and its log scale, through the combined call."""
    rng = np.random.default_rng(1107)
    img = W.random_image(rng, (50, 41), 6)
    plan = api.Plan(T(img))
    plan.set_tuning(ect_dirs_per_group=1)
    dirs, thr = T(W.circle_dirs(20)), T(np.linspace(-40, 40, 80))
    xi = T(rng.standard_normal((120, 2)) * 3.0)
    ls_sep = torch.empty(120, dtype=torch.float64, device="cuda:0")
    ls_one = torch.empty(120, dtype=torch.float64, device="cuda:0")
    sep = plan.hybrid_multi(xi, ("laplace", "bessel"), 2.0, "fp32", log_scale_out=ls_sep)
    e_one, one = plan.ect_hybrid_multi(dirs, thr, xi, ("laplace", "bessel"), 2.0, "fp32", log_scale_out=ls_one)
    for k in ("laplace", "bessel"):
        assert torch.equal(one[k], sep[k]), k
    assert torch.equal(ls_one, ls_sep)
    assert np.array_equal(e_one.cpu().numpy(), O.ect(img, W.circle_dirs(20), np.linspace(-40, 40, 80)))
    assert plan.check() == 0



def test_rerun_prepare_buckets_the_queries_in_the_compaction_launch(api):
    """ect_plan_rerun_prepare: the next forward call skips its bucketing and gives the same outputs as
    after a plain re-run, also when the image changed in place (new list sizes: the work list is built
    from this launch's totals); calls in between that write the workspace or re-run cancel the skip."""
    rng = np.random.default_rng(1108)
    a = W.binary_field(rng, (150, 170), 3.0).astype(np.uint8)
    b = W.binary_field(rng, (150, 170), 6.0).astype(np.uint8)
    buf = T(a)
    plan = api.Plan(buf)
    plan.set_tuning(ect_dirs_per_group=1)
    dirs, thr = T(W.circle_dirs(30)), T(np.linspace(-120, 120, 96))
    xi = api.QuerySet(T(rng.standard_normal((700, 2)) * 0.5))
    for img in (a, b, a):
        buf.copy_(T(img))
        plan.rerun()
        e_ref, h_ref = plan.ect_hybrid_multi(dirs, thr, xi, KERNELS)
        e_ref, h_ref = e_ref.cpu().numpy(), {k: v.cpu().numpy() for k, v in h_ref.items()}
        plan.rerun_prepare(xi)
        e, h = plan.ect_hybrid_multi(dirs, thr, xi, KERNELS)
        assert np.array_equal(e.cpu().numpy(), e_ref)
        for k in KERNELS:
            assert np.array_equal(h[k].cpu().numpy(), h_ref[k]), k
        assert np.array_equal(e_ref, O.ect(img, W.circle_dirs(30), np.linspace(-120, 120, 96)))
        # the separate forward call consumes the buckets as well
        plan.rerun_prepare(xi)
        hm = plan.hybrid_multi(xi, KERNELS)
        for k in KERNELS:
            assert np.array_equal(hm[k].cpu().numpy(), h_ref[k]), k
        # an ECT call on the same workspace in between: the evaluation buckets again
        plan.rerun_prepare(xi)
        plan.ect(dirs, thr)
        hm = plan.hybrid_multi(xi, KERNELS)
        for k in KERNELS:
            assert np.array_equal(hm[k].cpu().numpy(), h_ref[k]), k
    # the backward pass reuses what the skipped forward call found in the workspace
    plan.rerun_prepare(xi)
    y = plan.hybrid_multi(xi, KERNELS)["fourier"]
    g = T(rng.standard_normal((700, 2)))
    got = [t.cpu().numpy() for t in plan.hybrid_backward(xi, y, g, "fourier", 1.0, "fp32", reuse_prepared=True)]
    ref = [t.cpu().numpy() for t in plan.hybrid_backward(xi, y, g, "fourier", 1.0, "fp32")]
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    assert plan.check() == 0


def test_rerun_prepare_on_plans_it_does_not_apply_to(api):
    """Three axes and batches of several images: a plain re-run, the evaluation buckets the set itself."""
    rng = np.random.default_rng(1109)
    vol = W.random_image(rng, (12, 10, 9), 4)
    p3 = api.Plan(T(vol))
    xi3 = api.QuerySet(T(rng.standard_normal((90, 3)) * 0.4))
    ref = {k: v.cpu().numpy() for k, v in p3.hybrid_multi(xi3, KERNELS).items()}
    p3.rerun_prepare(xi3)
    for k, v in p3.hybrid_multi(xi3, KERNELS).items():
        assert np.array_equal(v.cpu().numpy(), ref[k]), k
    imgs = [W.random_image(rng, (30, 20), 4), W.random_image(rng, (25, 25), 3)]
    p2 = api.Plan([T(im) for im in imgs])
    xi2 = api.QuerySet(T(rng.standard_normal((80, 2)) * 0.4))
    ref = {k: v.cpu().numpy() for k, v in p2.hybrid_multi(xi2, KERNELS).items()}
    p2.rerun_prepare(xi2)
    for k, v in p2.hybrid_multi(xi2, KERNELS).items():
        assert np.array_equal(v.cpu().numpy(), ref[k]), k
    with pytest.raises(ValueError):
        p2.rerun_prepare(api.QuerySet(T(rng.standard_normal((4, 2))), T(np.array([0, 2, 4], np.int64))))
    assert p3.check() == 0 and p2.check() == 0
