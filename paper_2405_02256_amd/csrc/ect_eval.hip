// Exact Euler characteristic transform at explicit thresholds (gfx950).
//
// By Lemma 3.1, ECT(xi, t) = sum over classical points x of eps(xi) of
// Delta^-(eps, x) [<xi, x> <= t].  For a group of directions sharing one sign
// vector, a workgroup streams that list once (one point per lane), projects
// each point on every direction of the group with the canonical FP64
// expression, finds the first threshold at or above the projection and adds
// the critical value into an LDS histogram (integer atomics, so the result
// does not depend on their order).  An inclusive prefix sum of each histogram
// is the ECT row (the vectorization of Sec. 4.3 and Appendix A, at arbitrary
// non-decreasing thresholds).
//
// The bin search starts from the arithmetic guess for evenly spaced thresholds
// and corrects it against the stored thresholds, so any non-decreasing array
// gives the exact answer and an evenly spaced one needs at most a step or two.
#include "eval_internal.h"

namespace ect {

namespace {

template <int N>
__global__ void __launch_bounds__(kEctThreads) ect_kernel(EctArgs a) {
    extern __shared__ __align__(16) char smem[];
    constexpr int TD = kEctMaxDirs;
    constexpr int B = 1 << N;
    constexpr int W = kEctThreads / 64;
    const int M = a.M;
    double* s_thr = (double*)smem;
    int32_t* s_hist = (int32_t*)(smem + sizeof(double) * M);
    __shared__ double s_xi[TD][3];
    __shared__ int64_t s_row[TD];
    __shared__ int s_valid[TD];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t item = blockIdx.x;
    const int64_t E = (int64_t)a.num_images * B;
    if (item >= a.item_off[E]) return;
    int64_t lo = 0, hi = E - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (a.item_off[mid] <= item) lo = mid; else hi = mid - 1;
    }
    const int64_t e = lo;
    const int64_t img = e / B;
    const int b = (int)(e % B);
    const int64_t t = item - a.item_off[e];
    const bool shared_q = a.offsets == nullptr;
    const int64_t bidx = shared_q ? b : e;
    const int64_t qn = a.bcnt[bidx];
    const int TDg = a.dirs_per_group;
    const int64_t q0 = t * TDg;
    const int nd = (int)min<int64_t>(TDg, qn - q0);
    const int64_t row_base = shared_q ? img * a.count : a.offsets[img];

    if (tid < TD) {
        int ok = 0;
        int64_t row = -1;
        if (tid < nd) {
            const QRec r = a.recs[bucket_start(a.offsets, a.count, img, B, b) + q0 + tid];
            row = row_base + (r.code >> 1);               // output row
            ok = 1;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double v = r.v[c];
                s_xi[tid][c] = v;
                ok &= isfinite(v) ? 1 : 0;
            }
        }
        s_row[tid] = row;
        s_valid[tid] = ok;
    }
    const double* thr = a.thresholds + (a.thr_per_image ? img * M : 0);
    int bad = 0;
    for (int j = tid; j < M; j += kEctThreads) {
        double v = thr[j];
        s_thr[j] = v;
        if (j > 0 && !(v >= thr[j - 1])) bad = 1;
        if (!isfinite(v)) bad = 1;
    }
    for (int j = tid; j < a.dirs_per_group * M; j += kEctThreads) s_hist[j] = 0;
    bad = __syncthreads_or(bad);
    if (bad) {
        if (tid == 0) raise_error(a.err, ECT_DEVERR_THRESHOLDS);
        for (int dd = 0; dd < nd; ++dd)
            for (int j = tid; j < M; j += kEctThreads) a.out[s_row[dd] * M + j] = 0;
        return;
    }

    const double t0 = s_thr[0], t1 = s_thr[M - 1];
    const double inv = (M > 1 && t1 > t0) ? (double)(M - 1) / (t1 - t0) : 0.0;
    double xi[TD][N];
    bool use[TD];
#pragma unroll
    for (int dd = 0; dd < TD; ++dd) {
        use[dd] = dd < nd && s_valid[dd];
#pragma unroll
        for (int c = 0; c < N; ++c) xi[dd][c] = s_xi[dd][c];
    }

    const Point* __restrict__ pts = a.points + (int64_t)b * a.capacity;
    const int64_t p0 = a.list_off[img * a.NL + b], p1 = a.list_off[(img + 1) * a.NL + b];
    // U points per thread are loaded before any is processed, so that their
    // memory latencies overlap
    constexpr int U = 4;
    for (int64_t p = p0 + tid; p < p1; p += (int64_t)kEctThreads * U) {
        Point pt[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t pp = p + (int64_t)u * kEctThreads;
            if (pp < p1) pt[u] = pts[pp];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (p + (int64_t)u * kEctThreads >= p1) break;
            const int32_t val = (int32_t)pt[u].val;
#pragma unroll
            for (int dd = 0; dd < TD; ++dd) {
                if (!use[dd]) continue;
                const double uu = project<N>(xi[dd], pt[u].x);
                double g = ceil((uu - t0) * inv);
                g = fmin(fmax(g, 0.0), (double)M);
                int j = (int)g;
                while (j > 0 && s_thr[j - 1] >= uu) --j;
                while (j < M && s_thr[j] < uu) ++j;
                if (j < M) atomicAdd(&s_hist[dd * M + j], val);
            }
        }
    }
    __syncthreads();

    for (int dd = wave; dd < nd; dd += W) {
        int32_t* out = a.out + s_row[dd] * M;
        if (!s_valid[dd]) {
            for (int j = lane; j < M; j += 64) out[j] = 0;
            continue;
        }
        int32_t carry = 0;
        for (int jb = 0; jb < M; jb += 64) {
            const int j = jb + lane;
            int32_t v = j < M ? s_hist[dd * M + j] : 0;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                int32_t o = __shfl_up(v, off, 64);
                if (lane >= off) v += o;
            }
            if (j < M) out[j] = carry + v;
            carry += __shfl(v, 63, 64);
        }
    }
}

}  // namespace

hipError_t launch_ect(int ndim, const EctArgs& a, int64_t grid, hipStream_t stream) {
    if (grid <= 0) return hipSuccess;
    size_t shmem = sizeof(double) * a.M + sizeof(int32_t) * a.dirs_per_group * a.M;
    hipError_t e = stage_mark(ECT_STAGE_ECT, false, stream);
    if (e != hipSuccess) return e;
    if (ndim == 2)
        hipLaunchKernelGGL(ect_kernel<2>, dim3((unsigned)grid), dim3(kEctThreads), shmem, stream, a);
    else
        hipLaunchKernelGGL(ect_kernel<3>, dim3((unsigned)grid), dim3(kEctThreads), shmem, stream, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return stage_mark(ECT_STAGE_ECT, true, stream);
}

}  // namespace ect
