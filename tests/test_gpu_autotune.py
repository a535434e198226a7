"""Schedule knobs and the autotuner on the GPU: any setting keeps the ECT
bit-exact and the hybrid transforms within the FP32 gate of the oracle;
identical settings give bitwise identical outputs; a tuned, captured step
replays to its eager result; the cache answers a repeated workload without
timing anything."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_02256_amd import workloads as W

from oracle.gates import fp32_gate, grad_gate, grad_scales, term_scales

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


def _cplx(y):
    return y[:, 0] + 1j * y[:, 1]


@pytest.fixture(scope="module")
def small():
    rng = np.random.default_rng(77)
    img = W.binary_field(rng, (96, 80), 3.0)
    xi = W.polar_vectors(rng, 200, 0.01, 1.0)
    # shuffled: neighbouring directions in a group fall in different orthants
    dirs = W.circle_dirs(40)[rng.permutation(40)]
    thr = W.even_thresholds(70.0, 96)
    return img, xi, dirs, thr


# chunk 16 splits every list into many chunks (more than the reduce kernel's
# batch of 16 per pass); large chunks leave every tile in one chunk
@pytest.mark.parametrize("chunk,items,td,ech", [(16, 2048, 1, 1), (48, 2048, 3, 0), (0, 1, 8, 7), (0, 1 << 24, 0, 64),
                                                (1 << 20, 2048, 5, 4096)])
def test_any_tuning_keeps_parity(api, small, chunk, items, td, ech):
    img, xi, dirs, thr = small
    plan = api.Plan(T(img))
    plan.set_tuning(chunk, items, td, ech)
    assert np.array_equal(plan.ect(T(dirs), T(thr)).cpu().numpy(), O.ect(img, dirs, thr))
    # the Radon transform splits its lists the same way (chunk histograms and point values)
    assert np.array_equal(plan.radon(T(dirs), T(thr)).cpu().numpy(), O.radon(img, dirs, thr))
    outs = plan.hybrid_multi(T(xi), ("fourier", "laplace", "bessel"), 1.0, "fp32")
    for k in ("fourier", "laplace", "bessel"):
        y = outs[k].cpu().numpy()
        y = _cplx(y) if k == "fourier" else y
        ref = O.hybrid(img, xi, k, 1.0)
        _, S2 = term_scales(img, xi, k, 1.0)
        ok, ratio, norm, _ = fp32_gate(y, ref, S2)
        assert ok, (k, ratio, norm)
    # the backward reduces per-query partials over the same chunks
    y = plan.hybrid(T(xi), "fourier", 1.0, "fp32")
    g = np.random.default_rng(8).standard_normal((len(xi), 2))
    gxi, gs = plan.hybrid_backward(T(xi), y, T(g), "fourier", 1.0, "fp32")
    ref_xi, ref_s = O.hybrid_grad(img, xi, "fourier", 1.0, g[:, 0] + 1j * g[:, 1])
    S2x, _, S2s, _ = grad_scales(img, xi, "fourier", 1.0, g)
    ok, ratio, norm, _ = grad_gate(gxi.cpu().numpy(), ref_xi, S2x)
    assert ok, (ratio, norm)
    ok, ratio, _, _ = fp32_gate([float(gs.cpu())], [ref_s], [np.sqrt((S2s ** 2).sum())], normwise=False)
    assert ok, ratio
    assert plan.check() == 0


def test_same_tuning_bitwise_identical(api, small):
    img, xi, dirs, thr = small
    plan = api.Plan(T(img))
    plan.set_tuning(32, 2048, 2)
    a = plan.hybrid_multi(T(xi), ("fourier", "laplace"), 1.0, "fp32")
    plan.set_tuning(0, 64, 0)
    plan.hybrid_multi(T(xi), ("fourier", "laplace"), 1.0, "fp32")
    plan.set_tuning(32, 2048, 2)
    b = plan.hybrid_multi(T(xi), ("fourier", "laplace"), 1.0, "fp32")
    for k in a:
        assert torch.equal(a[k], b[k]), k


def test_rejects_out_of_range(api, small):
    plan = api.Plan(T(small[0]))
    for args in [(8, 2048, 0), (-1, 2048, 0), (0, 0, 0), (0, 2048, 9), (0, 2048, -1), (0, 2048, 0, -1),
                 (0, 2048, 0, 4097)]:
        with pytest.raises(RuntimeError):
            plan.set_tuning(*args)


def test_autotuned_step_replays_and_caches(api, small, tmp_path):
    from paper_2405_02256_amd import autotune as AT
    from paper_2405_02256_amd.pipeline import Step
    img, xi, dirs, thr = small
    cache = AT.Cache(str(tmp_path / "tuning.json"))
    plan = api.Plan(T(img))
    g = T(np.random.default_rng(9).standard_normal((len(xi), 2)))
    step = Step(plan, T(dirs), T(thr), T(xi), ("fourier", "laplace", "bessel"), backward_kernel="fourier",
                grad_out=g)
    t = step.autotune(cache=cache, reps=3)
    assert (t.ect_dirs_per_group, t.ect_chunks) in AT.ECT_CANDIDATES
    assert t.hybrid_target_items in AT.HYBRID_ITEM_CANDIDATES
    # the step runs the ECT inside the hybrid launch, so its knobs are swept again on that call
    assert set(t.timings) == {"ect", "hybrid", "ect_hybrid"}
    assert min(t.timings["ect_hybrid"], key=t.timings["ect_hybrid"].get) == f"{t.ect_dirs_per_group}/{t.ect_chunks}"
    assert plan.tuning == t.as_args()
    step.run()
    torch.cuda.synchronize()
    eager = {k: v.clone() for k, v in step.hy_out.items()}
    eager_ect, eager_gxi = step.ect_out.clone(), step.grad_xi.clone()
    assert np.array_equal(eager_ect.cpu().numpy(), O.ect(img, dirs, thr))
    step.capture()
    for _ in range(3):
        for v in step.hy_out.values():
            v.fill_(float("nan"))
        step.ect_out.fill_(-1)
        step.replay()
        torch.cuda.synchronize()
        for k in eager:
            assert torch.equal(step.hy_out[k], eager[k]), k
        assert torch.equal(step.ect_out, eager_ect)
        assert torch.equal(step.grad_xi, eager_gxi)

    def no_timing(fn, reps):
        raise AssertionError("cache hit expected")
    plan2 = api.Plan(T(img))
    t2 = AT.tune(plan2, T(dirs), T(thr), T(xi), ("fourier", "laplace", "bessel"), backward_kernel="fourier",
                 grad_out=g, cache=cache, timer=no_timing, combined=True)
    assert t2.as_args() == t.as_args() and plan2.tuning == t.as_args()


def test_concurrent_ect_branch_matches_serial_step(api, small):
    """The ECT branch on its own stream (and graph branch) gives the serial step's outputs bitwise."""
    from paper_2405_02256_amd.pipeline import Step
    img, xi, dirs, thr = small
    g = T(np.random.default_rng(10).standard_normal((len(xi), 2)))
    outs = []
    for concurrent in (False, True):
        plan = api.Plan(T(img))
        st = Step(plan, T(dirs), T(thr), T(xi), ("fourier", "laplace"), backward_kernel="fourier", grad_out=g,
                  concurrent=concurrent)
        st.run()
        torch.cuda.synchronize()
        eager = (st.ect_out.clone(), {k: v.clone() for k, v in st.hy_out.items()}, st.grad_xi.clone())
        st.capture()
        for _ in range(2):
            st.ect_out.fill_(-7)
            st.replay()
            torch.cuda.synchronize()
            assert torch.equal(st.ect_out, eager[0])
            assert all(torch.equal(st.hy_out[k], eager[1][k]) for k in eager[1])
            assert torch.equal(st.grad_xi, eager[2])
        outs.append(eager)
    assert torch.equal(outs[0][0], outs[1][0])
    assert all(torch.equal(outs[0][1][k], outs[1][1][k]) for k in outs[0][1])
    assert torch.equal(outs[0][2], outs[1][2])


def test_concurrent_batched_ect_beside_ragged_laplace(api):
    """The step of many images (per-image thresholds, so the batched ECT
    kernel, and a ragged Laplace set) with the ECT on its own stream and
    graph branch equals the serial step bitwise, over graph replays."""
    from paper_2405_02256_amd.pipeline import Step
    rng = np.random.default_rng(12)
    sides = rng.choice([12, 24, 40], size=160)
    imgs = [W.binary_field(rng, (int(s), int(s)), 2.0) for s in sides]
    dirs = W.circle_dirs(24) + 1e-3
    thr = np.stack([W.even_thresholds(float(s), 32) for s in sides])
    nq = 40
    xi = np.concatenate([W.polar_vectors(rng, nq, 0.01, 1.0) for _ in imgs])
    offs = T(np.arange(len(imgs) + 1, dtype=np.int64) * nq)
    outs = []
    for concurrent in (False, True):
        plan = api.Plan([T(im) for im in imgs])
        st = Step(plan, T(dirs), T(thr), T(xi), ("laplace",), precision="fp32", hybrid_offsets=offs,
                  concurrent=concurrent)
        assert st.concurrent == concurrent
        st.run()
        torch.cuda.synchronize()
        eager = (st.ect_out.clone(), st.hy_out["laplace"].clone())
        st.capture()
        for _ in range(3):
            st.ect_out.fill_(-7)
            st.hy_out["laplace"].fill_(0.5)
            st.replay()
            torch.cuda.synchronize()
            assert torch.equal(st.ect_out, eager[0])
            assert torch.equal(st.hy_out["laplace"], eager[1])
        assert plan.check() == 0
        outs.append(eager)
    assert torch.equal(outs[0][0], outs[1][0])
    assert torch.equal(outs[0][1], outs[1][1])
    for i in (0, 77, 159):
        assert np.array_equal(outs[1][0].cpu().numpy().reshape(len(imgs), len(dirs), -1)[i],
                              O.ect(imgs[i], dirs, thr[i])), i


def test_backward_reuses_forward_buckets(api, small):
    """The backward call with the reuse flag gives the same gradients as a
    backward call that buckets again, and is refused when the last
    preparation does not match (other query set, re-run, retuning)."""
    from paper_2405_02256_amd import _native as N
    img, xi, dirs, thr = small
    plan = api.Plan(T(img))
    q = api.QuerySet(T(xi))
    g = T(np.random.default_rng(11).standard_normal((len(xi), 2)))
    y = plan.hybrid_multi(q, ("fourier", "bessel"), 1.0, "fp32")["fourier"]
    a = plan.hybrid_backward(q, y, g, "fourier", 1.0, "fp32", reuse_prepared=True)
    b = plan.hybrid_backward(q, y, g, "fourier", 1.0, "fp32")
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    # the plain backward call above prepared again, so reuse still matches
    c = plan.hybrid_backward(q, y, g, "fourier", 1.0, "fp32", reuse_prepared=True)
    assert torch.equal(a[0], c[0])
    other = api.QuerySet(T(xi[:50]))
    plan.hybrid(other, "laplace", 1.0, "fp32")
    with pytest.raises(N.EctError):
        plan.hybrid_backward(q, y, g, "fourier", 1.0, "fp32", reuse_prepared=True)
    plan.hybrid(q, "fourier", 1.0, "fp32")
    plan.rerun()
    with pytest.raises(N.EctError):
        plan.hybrid_backward(q, y, g, "fourier", 1.0, "fp32", reuse_prepared=True)
    plan.hybrid(q, "fourier", 1.0, "fp32")
    plan.set_tuning(64, 2048, 0)
    with pytest.raises(N.EctError):
        plan.hybrid_backward(q, y, g, "fourier", 1.0, "fp32", reuse_prepared=True)
    plan.hybrid(q, "fourier", 1.0, "fp32", slot="other")
    with pytest.raises(N.EctError):
        plan.hybrid_backward(q, y, g, "fourier", 1.0, "fp32", reuse_prepared=True)
    # any other call that writes the same workspace ends the reuse
    for other_call in (lambda: plan.ect(T(dirs), T(thr)), lambda: plan.exact(T(dirs), "ect"),
                       lambda: plan.exact(T(dirs), "radon")):
        plan.hybrid(q, "fourier", 1.0, "fp32")
        plan.hybrid_backward(q, y, g, "fourier", 1.0, "fp32", reuse_prepared=True)
        other_call()
        with pytest.raises(N.EctError):
            plan.hybrid_backward(q, y, g, "fourier", 1.0, "fp32", reuse_prepared=True)
    torch.cuda.synchronize()
