"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark uses; the oracle checks sampled outputs (all lists are compared in
full for the volume)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_02256_amd import workloads as W

from gates import fp32_gate, term_scales

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


def test_volume_128_full(api):
    w = W.volume_128(3)
    vol = w.images[0]
    org = np.zeros(3)
    plan = api.Plan(T(vol), origin=org)
    # every list, entry by entry
    lw, od = O.critical_values(vol, O.PRIMAL)
    V = 129
    for e in range(8):
        coords, vals = plan.export(0, 0, e)
        nz = np.nonzero(lw[:, e])[0]
        lin = coords[:, 0] + V * (coords[:, 1] + V * coords[:, 2])
        assert np.array_equal(lin, nz) and np.array_equal(vals, lw[nz, e]), e
    for e in range(4):
        coords, vals = plan.export(0, 1, e)
        nz = np.nonzero(od[:, e])[0]
        lin = coords[:, 0] + V * (coords[:, 1] + V * coords[:, 2])
        assert np.array_equal(lin, nz) and np.array_equal(vals, od[nz, e]), e
    # ECT: all 2048 directions on the GPU, 8 of them checked
    ect = plan.ect(T(w.ect_dirs), T(w.ect_thresholds)).cpu().numpy()
    sel = np.linspace(0, 2047, 8).astype(int)
    assert np.array_equal(ect[sel], O.ect(vol, w.ect_dirs[sel], w.ect_thresholds, origin=org))
    # hybrid: all 16384 xi, Fourier and Laplace (log-scale) in one fused pass
    ls = torch.empty(len(w.hybrid_xi), dtype=torch.float64, device="cuda:0")
    outs = plan.hybrid_multi(T(w.hybrid_xi), ("fourier", "laplace"), 1.0, "fp32", log_scale_out=ls)
    f = _cplx(outs["fourier"].cpu().numpy())
    lo, lsv = outs["laplace"].cpu().numpy(), ls.cpu().numpy()
    qs = np.random.default_rng(3).choice(len(w.hybrid_xi), 10, replace=False)
    ref_f = O.hybrid(vol, w.hybrid_xi[qs], "fourier", 1.0, origin=org)
    _, S2 = term_scales(vol, w.hybrid_xi[qs], "fourier", 1.0, origin=org)
    ok, ratio, norm, strict = fp32_gate(f[qs], ref_f, S2)
    assert ok, ("fourier", ratio, norm)
    ref_l, m = O.hybrid(vol, w.hybrid_xi[qs], "laplace", 1.0, origin=org, with_shift=True)
    _, S2 = term_scales(vol, w.hybrid_xi[qs], "laplace", 1.0, origin=org, shift=m)
    ok, ratio, norm, strict = fp32_gate(lo[qs] * np.exp(lsv[qs] - m), ref_l, S2)
    assert ok, ("laplace", ratio, norm)
    assert plan.check() == 0


def test_batch_4096_full(api):
    w = W.batch_4096(4)
    imgs = w.images
    plan = api.Plan([T(im) for im in imgs])
    c, o = plan.counts()
    rng = np.random.default_rng(4)
    sample = rng.choice(len(imgs), 12, replace=False)
    for i in sample:
        lw, od = O.critical_values(imgs[i], O.PRIMAL)
        assert c[i].tolist() == [int(np.count_nonzero(lw[:, e])) for e in range(4)]
        assert o[i].tolist() == [int(np.count_nonzero(od[:, e])) for e in range(2)]
    thr = w.ect_thresholds
    ect = plan.ect(T(w.ect_dirs), T(thr)).cpu().numpy().reshape(len(imgs), len(w.ect_dirs), -1)
    for i in sample:
        assert np.array_equal(ect[i], O.ect(imgs[i], w.ect_dirs, thr[i])), i
    nq = 512
    offs = np.arange(len(imgs) + 1, dtype=np.int64) * nq
    y = plan.hybrid(T(w.hybrid_xi), "laplace", 1.0, "fp32", offsets=T(offs)).cpu().numpy()
    y64 = plan.hybrid(T(w.hybrid_xi), "laplace", 1.0, "fp64", offsets=T(offs)).cpu().numpy()
    for i in sample[:6]:
        rows = offs[i] + rng.choice(nq, 16, replace=False)
        ref = O.hybrid(imgs[i], w.hybrid_xi[rows], "laplace", 1.0)
        _, S2 = term_scales(imgs[i], w.hybrid_xi[rows], "laplace", 1.0)
        ok, ratio, norm, strict = fp32_gate(y[rows], ref, S2)
        assert ok, (i, ratio, norm)
        ok64, ratio64, _, _ = fp32_gate(y64[rows], ref, S2)
        assert ok64 and ratio64 < ratio + 1e-3
    assert plan.check() == 0


def test_diff_256_forward_backward(api):
    w = W.diff_256(5)
    imgs = w.images
    plan = api.Plan([T(im) for im in imgs])
    xi = T(w.hybrid_xi)
    nq = len(w.hybrid_xi)
    rng = np.random.default_rng(5)
    for kernel in ("fourier", "laplace"):
        y = plan.hybrid(xi, kernel, 1.0, "fp32").cpu().numpy()
        y = _cplx(y) if kernel == "fourier" else y
        y = y.reshape(len(imgs), nq)
        for i in rng.choice(len(imgs), 3, replace=False):
            qs = rng.choice(nq, 12, replace=False)
            ref = O.hybrid(imgs[i], w.hybrid_xi[qs], kernel, 1.0)
            _, S2 = term_scales(imgs[i], w.hybrid_xi[qs], kernel, 1.0)
            ok, ratio, norm, strict = fp32_gate(y[i, qs], ref, S2)
            assert ok, (kernel, i, ratio, norm)
        # backward of the seeded loss sum(W * outputs) at the shared xi, summed over the 256 images
        wts = w.meta["loss_weights"] if kernel == "fourier" else w.meta["loss_weights"][..., 0]
        g = T(wts.reshape(len(imgs) * nq, -1) if kernel == "fourier" else wts.reshape(-1))
        yd = plan.hybrid(xi, kernel, 1.0, "fp32")
        gxi, gs = plan.hybrid_backward(xi, yd, g, kernel, 1.0, "fp32")
        gxi = gxi.cpu().numpy()
        qs = rng.choice(nq, 6, replace=False)
        ref = np.zeros((len(qs), 2))
        for i, im in enumerate(imgs):
            gi = wts[i, qs] if kernel == "fourier" else wts[i, qs]
            a, _ = O.hybrid_grad(im, w.hybrid_xi[qs], kernel, 1.0, gi)
            ref += a
        err = np.abs(gxi[qs] - ref).max() / np.abs(ref).max()
        assert err < 1e-5, (kernel, err)


def test_diff_256_finite_differences_fp64(api):
    """Central differences (h = 1e-3) of the FP64 forward against the backward kernel."""
    w = W.diff_256(5, count=32)
    imgs = w.images
    plan = api.Plan([T(im) for im in imgs])
    nq = len(w.hybrid_xi)
    wts = w.meta["loss_weights"]
    xi0 = w.hybrid_xi.copy()
    for kernel in ("fourier", "laplace"):
        wk = wts if kernel == "fourier" else wts[..., 0]
        g = T(wk.reshape(len(imgs) * nq, -1) if kernel == "fourier" else wk.reshape(-1))

        def loss(xv, s, q=None):
            # dL/dxi_q involves only the outputs at query q (Laplace rows reach 1e19, which would
            # swamp a perturbation of one row in the full sum)
            y = plan.hybrid(T(xv), kernel, s, "fp64").cpu().numpy().reshape(wk.shape)
            if q is not None:
                return float((y[:, q] * wk[:, q]).sum())
            return float((y * wk).sum())

        y = plan.hybrid(T(xi0), kernel, 1.0, "fp64")
        gxi, gs = plan.hybrid_backward(T(xi0), y, g, kernel, 1.0, "fp64")
        gxi, gs = gxi.cpu().numpy(), float(gs.cpu())
        h = 1e-3
        far = [q for q in range(nq) if np.abs(xi0[q]).min() > 10 * h][:3]   # stay inside the orthant
        for q in far:
            for a in range(2):
                xp, xm = xi0.copy(), xi0.copy()
                xp[q, a] += h
                xm[q, a] -= h
                fd = (loss(xp, 1.0, q) - loss(xm, 1.0, q)) / (2 * h)
                assert abs(fd - gxi[q, a]) <= 1e-2 * max(1.0, abs(fd)), (kernel, q, a, fd, gxi[q, a])
        fds = (loss(xi0, 1.0 + h) - loss(xi0, 1.0 - h)) / (2 * h)
        assert abs(fds - gs) <= 1e-2 * max(1.0, abs(fds)), (kernel, fds, gs)
