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
// The Radon transform at thresholds uses the same kernels (RADON = true): by
// Lemma 3.1 with the sign the definition gives, R(xi, t) = sum over classical
// points of Delta^-(eps, x) [<xi,x> = t] - sum over ordinary points of
// D(eps, x) [<xi,x> < t], so the classical list feeds a per-threshold point
// array (no prefix sum) and the ordinary list of the orthant pair (negated for
// the mirrored half) a histogram binned at the first threshold above the
// projection, whose prefix sum is added.
//
// Shared query sets (one direction set for every image) are evaluated without
// a bucketing pass (ect_direct_kernel); ragged sets are bucketed by sign vector
// first (ect_kernel).
//
// The bin search starts from the arithmetic guess for evenly spaced thresholds
// and corrects it against the stored thresholds, so any non-decreasing array
// gives the exact answer and an evenly spaced one needs at most a step or two.
#include "ect_body.h"

namespace ect {

namespace {

// Bucketed sets (ragged query sets): one workgroup per group of up to
// dirs_per_group directions of one (image, sign vector) bucket.
template <int N, bool RADON>
__global__ void __launch_bounds__(kEctThreads) ect_kernel(EctArgs a) {
    extern __shared__ __align__(16) char smem[];
    constexpr int TD = kEctMaxDirs;
    constexpr int B = 1 << N;
    const int M = a.M;
    double* s_thr = (double*)smem;
    int32_t* s_hist = (int32_t*)(smem + sizeof(double) * M);
    __shared__ double s_xi[TD][kMaxDim];
    __shared__ int64_t s_row[TD];
    __shared__ int s_valid[TD];

    const int tid = threadIdx.x;
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
            const QRecT<N> r = ((const QRecT<N>*)a.recs)[bucket_start(a.offsets, a.count, img, B, b) + q0 + tid];
            row = row_base + (r.code >> 1);               // output row
            ok = 1;
#pragma unroll
            for (int c = 0; c < N; ++c) {
                const double v = r.v[c];
                s_xi[tid][c] = v;
                ok &= isfinite(v) ? 1 : 0;
            }
        }
        s_row[tid] = row;
        s_valid[tid] = ok;
    }
    int32_t* s_point = s_hist + (int64_t)a.dirs_per_group * M;   // Radon point values
    if (stage_thresholds(a, img, s_thr, s_hist, RADON ? 2 : 1)) {
        if (tid == 0) raise_error(a.err, ECT_DEVERR_THRESHOLDS);
        zero_rows(a, nd, s_row);
        return;
    }
    double xi[TD][N];
    bool use[TD];
#pragma unroll
    for (int dd = 0; dd < TD; ++dd) {
        use[dd] = dd < nd && s_valid[dd];
#pragma unroll
        for (int c = 0; c < N; ++c) xi[dd][c] = s_xi[dd][c];
    }
    if constexpr (RADON) {
        accumulate_radon<N>(a, img, b, 0, 1, xi, use, s_thr, s_hist, s_point);
    } else {
        const int64_t p0 = a.list_off[img * a.NL + b], p1 = a.list_off[(img + 1) * a.NL + b];
        accumulate_list<N, kBinClosed>(list_entries(a.points, a.capacity, b), a.desc[img], p0, p1, xi, use, s_thr, M,
                                       s_hist);
    }
    __syncthreads();
    write_rows(a, nd, s_row, s_valid, s_hist, RADON ? s_point : nullptr);
}

// Shared query sets: one workgroup per (image, group of directions, part of
// the list); see ect_direct_block.
template <int N, bool RADON>
__global__ void __launch_bounds__(kEctWideThreads) ect_direct_kernel(EctArgs a, int64_t groups) {
    ect_direct_block<N, RADON>(a, groups, blockIdx.x);
}

// Shared direction sets over many images with short lists: one workgroup per
// (image, sign vector b).  The set was bucketed by sign vector once (records
// in input order within a bucket); the workgroup takes its bucket's
// directions kBatchDirs at a time and gives each of them 256 / D lanes (D the
// pass's directions rounded up to a power of two), which split the list
// between them.  So every lane works even when a list holds a few dozen
// points, where streaming the list across the lanes for a few directions
// leaves most of them idle.
//
// The list is staged in LDS a stage of 256 points at a time (one coalesced
// load per thread, the next stage's loads in flight while this one is
// binned).  A lane bins the canonical projection of each of its points on its
// direction: the arithmetic guess for evenly spaced thresholds is checked
// against the two thresholds around it with one LDS read (the thresholds sit
// between -inf and +inf sentinels), and only a wrong guess searches; the
// critical value is added into the direction's LDS histogram (integer
// atomics; rows at an odd stride, so that neighbouring directions' bins fall
// in different banks).  The histograms are then prefix-summed in place by
// eight threads per row (a sequential scan of a segment, then a scan of the
// eight segment totals), and written out row by row with consecutive threads
// on consecutive thresholds.  Same bins as the other threshold kernels, so the
// rows are the same integers.
template <int N>
__global__ void __launch_bounds__(kBatchThreads) ect_batch_kernel(EctArgs a) {
    extern __shared__ __align__(16) char smem[];
    constexpr int B = 1 << N;
    constexpr int kSeg = kBatchThreads / kBatchDirs;   // threads per histogram row in the scan
    const int M = a.M;
    const int MS = M | 1;
    double* s_tp = (double*)smem;                                          // [M + 2]
    int32_t* s_hist = (int32_t*)(smem + batch_hist_offset(M));             // [kBatchDirs][MS]
    __shared__ double s_px[kBatchThreads * N];
    __shared__ int32_t s_pv[kBatchThreads];
    __shared__ double s_xi[kBatchDirs][kMaxDim];
    __shared__ int64_t s_row[kBatchDirs];
    __shared__ int s_valid[kBatchDirs];

    const int tid = threadIdx.x;
    const int64_t img = blockIdx.x / B;
    const int b = (int)(blockIdx.x % B);
    const int64_t qn = a.bcnt[b];
    if (qn == 0) return;
    const QRecT<N>* recs = (const QRecT<N>*)a.recs + (int64_t)b * a.count;
    const int64_t p0 = a.list_off[img * a.NL + b], p1 = a.list_off[(img + 1) * a.NL + b];
    const ListEntry* __restrict__ pts = list_entries(a.points, a.capacity, b);
    const ImageDesc& dsc = a.desc[img];

    // the list's first stage of points is requested with the thresholds
    ListEntry nxt{0u, 0};
    if (p0 + tid < p1) nxt = pts[p0 + tid];
    const double* thr = a.thresholds + (a.thr_per_image ? img * M : 0);
    int bad = 0;
    for (int j = tid; j < M; j += kBatchThreads) {
        const double v = thr[j];
        s_tp[j + 1] = v;
        if (j > 0 && !(v >= thr[j - 1])) bad = 1;
        if (!isfinite(v)) bad = 1;
    }
    if (tid == 0) {
        s_tp[0] = -INFINITY;
        s_tp[M + 1] = INFINITY;
    }
    bad = __syncthreads_or(bad);
    if (bad && tid == 0 && b == 0) raise_error(a.err, ECT_DEVERR_THRESHOLDS);
    const double t0 = s_tp[1], t1 = s_tp[M];
    const double inv = (M > 1 && t1 > t0) ? (double)(M - 1) / (t1 - t0) : 0.0;
    const int seg = (M + kSeg - 1) / kSeg;
    const int rows_per_pass = M <= kBatchThreads ? kBatchThreads / M : 1;
    const int wrow = M <= kBatchThreads ? tid / M : 0;
    const int wj = M <= kBatchThreads ? tid - wrow * M : tid;

    for (int64_t q0 = 0; q0 < qn; q0 += kBatchDirs) {
        const int nd = (int)min<int64_t>(kBatchDirs, qn - q0);
        if (tid < kBatchDirs) {
            int ok = 0;
            int64_t row = -1;
            if (tid < nd) {
                const QRecT<N> r = recs[q0 + tid];
                row = img * a.count + (r.code >> 1);
                ok = 1;
#pragma unroll
                for (int c = 0; c < N; ++c) {
                    s_xi[tid][c] = r.v[c];
                    ok &= isfinite(r.v[c]) ? 1 : 0;
                }
                if (!ok && img == 0) raise_error(a.err, ECT_DEVERR_NONFINITE);
            }
            s_row[tid] = row;
            s_valid[tid] = ok && !bad;
        }
        {
            int4* h4 = (int4*)s_hist;
            const int n4 = kBatchDirs * MS / 4;   // kBatchDirs is a multiple of 4
            for (int j = tid; j < n4; j += kBatchThreads) h4[j] = make_int4(0, 0, 0, 0);
        }
        // lanes per direction: D = nd rounded up to a power of two
        int D = 1;
        while (D < nd) D <<= 1;
        const int d = tid & (D - 1);
        const int lanes = kBatchThreads / D;
        const int slice = tid / D;
        __syncthreads();
        const bool active = d < nd && s_valid[d];
        double xi[N];
#pragma unroll
        for (int c = 0; c < N; ++c) xi[c] = s_xi[d][c];
        int32_t* hist = s_hist + d * MS;
        for (int64_t base = p0; base < p1; base += kBatchThreads) {
            const int cnt = (int)min<int64_t>(kBatchThreads, p1 - base);
            if (tid < cnt) {
                const PointT<N> pt = decode_entry<N>(nxt, dsc);
#pragma unroll
                for (int c = 0; c < N; ++c) s_px[tid * N + c] = pt.x[c];
                s_pv[tid] = nxt.val;
            }
            __syncthreads();
            // next stage, or after the last one the list's start for the next pass
            const int64_t nb = base + kBatchThreads;
            const int64_t src = nb < p1 ? nb + tid : (q0 + kBatchDirs < qn ? p0 + tid : p1);
            if (src < p1) nxt = pts[src];
            if (active) {
                for (int k = slice; k < cnt; k += lanes) {
                    double x[N];
#pragma unroll
                    for (int c = 0; c < N; ++c) x[c] = s_px[k * N + c];
                    const double u = project<N>(xi, x);
                    double g = ceil((u - t0) * inv);
                    g = fmin(fmax(g, 0.0), (double)M);
                    int j = (int)g;                         // candidate: t_{j-1} < u <= t_j
                    const double lo = s_tp[j], hi = s_tp[j + 1];
                    if (!((lo < u) & (u <= hi))) {          // a guess off by a threshold or more (rare)
                        while (j > 0 && s_tp[j] >= u) --j;
                        while (j < M && s_tp[j + 1] < u) ++j;
                    }
                    if (j < M) atomicAdd(&hist[j], s_pv[k]);
                }
            }
            __syncthreads();
        }
        // inclusive prefix sums in place: kSeg threads per row, a segment each
        {
            const int dd = tid / kSeg, part = tid % kSeg;
            const int j0 = min(M, part * seg), j1 = min(M, j0 + seg);
            int32_t* h = s_hist + dd * MS;
            int32_t run = 0;
            if (dd < nd)
                for (int j = j0; j < j1; ++j) {
                    run += h[j];
                    h[j] = run;
                }
            int32_t off = run;   // inclusive scan of the segment totals within the row's kSeg lanes
#pragma unroll
            for (int o = 1; o < kSeg; o <<= 1) {
                const int32_t v = __shfl_up(off, o, kSeg);
                if (part >= o) off += v;
            }
            off -= run;
            if (dd < nd && off != 0)
                for (int j = j0; j < j1; ++j) h[j] += off;
        }
        __syncthreads();
        // rows out: consecutive threads on consecutive thresholds
        if (wj < M && wrow < rows_per_pass)
            for (int dd = wrow; dd < nd; dd += rows_per_pass) {
                int32_t* out = a.out + s_row[dd] * M;
                const bool ok = s_valid[dd];
                for (int j = wj; j < M; j += (M <= kBatchThreads ? M : kBatchThreads))
                    out[j] = ok ? s_hist[dd * MS + j] : 0;
            }
        __syncthreads();
    }
}

// Sum of the chunk histograms of one direction (one wave per output row) and
// the inclusive prefix over thresholds; for the Radon transform (arrays = 2)
// plus the sum of the chunks' point values.
__global__ void __launch_bounds__(64) ect_chunk_sum_kernel(EctArgs a, int64_t groups, int arrays) {
    const int lane = threadIdx.x;
    const int TDg = a.dirs_per_group;
    const int M = a.M;
    const int64_t chunks = a.chunks;
    const int64_t dd = blockIdx.x % TDg;
    const int64_t rest = blockIdx.x / TDg;   // image * groups + g
    const int64_t q = (rest % groups) * TDg + dd;
    if (q >= a.count) return;
    const int64_t img = rest / groups;
    int32_t* out = a.out + (img * a.count + q) * M;
    const int64_t stride = (int64_t)arrays * TDg * M;   // one chunk's arrays
    const int32_t* part = a.part + rest * chunks * stride + dd * M;
    int32_t carry = 0;
    for (int jb = 0; jb < M; jb += 64) {
        const int j = jb + lane;
        int32_t v = 0, pv = 0;
        if (j < M)
            for (int64_t c = 0; c < chunks; ++c) {
                v += part[c * stride + j];
                if (arrays == 2) pv += part[c * stride + (int64_t)TDg * M + j];
            }
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t o = __shfl_up(v, off, 64);
            if (lane >= off) v += o;
        }
        if (j < M) out[j] = carry + v + pv;
        carry += __shfl(v, 63, 64);
    }
}

template <int N, bool RADON>
hipError_t launch_ect_typed(const EctArgs& a, int64_t grid, int64_t direct_groups, size_t shmem, hipStream_t stream) {
    if (direct_groups > 0) {
        hipLaunchKernelGGL((ect_direct_kernel<N, RADON>), dim3((unsigned)grid), dim3(a.threads), shmem, stream, a,
                           direct_groups);
        if (a.chunks > 1) {
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            const int64_t rows = (grid / a.chunks) * a.dirs_per_group;
            hipLaunchKernelGGL(ect_chunk_sum_kernel, dim3((unsigned)rows), dim3(64), 0, stream, a, direct_groups,
                               RADON ? 2 : 1);
        }
    } else {
        hipLaunchKernelGGL((ect_kernel<N, RADON>), dim3((unsigned)grid), dim3(a.threads), shmem, stream, a);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_ect_chunk_sum(const EctArgs& a, int64_t grid, int64_t groups, hipStream_t stream) {
    if (a.chunks <= 1 || grid <= 0) return hipSuccess;
    const int64_t rows = (grid / a.chunks) * a.dirs_per_group;
    hipLaunchKernelGGL(ect_chunk_sum_kernel, dim3((unsigned)rows), dim3(64), 0, stream, a, groups, 1);
    return hipGetLastError();
}

hipError_t launch_ect_batch(int ndim, const EctArgs& a, hipStream_t stream) {
    const int64_t grid = (int64_t)a.num_images << ndim;
    if (grid <= 0) return hipSuccess;
    const size_t shmem = batch_ect_lds(a.M);
    hipError_t e = stage_mark(ECT_STAGE_ECT, false, stream);
    if (e != hipSuccess) return e;
    if (ndim == 2)
        hipLaunchKernelGGL(ect_batch_kernel<2>, dim3((unsigned)grid), dim3(kBatchThreads), shmem, stream, a);
    else if (ndim == 3)
        hipLaunchKernelGGL(ect_batch_kernel<3>, dim3((unsigned)grid), dim3(kBatchThreads), shmem, stream, a);
    else
        hipLaunchKernelGGL(ect_batch_kernel<4>, dim3((unsigned)grid), dim3(kBatchThreads), shmem, stream, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return stage_mark(ECT_STAGE_ECT, true, stream);
}

hipError_t launch_ect(int ndim, const EctArgs& a, int64_t grid, int64_t direct_groups, bool radon,
                      hipStream_t stream) {
    if (grid <= 0) return hipSuccess;
    if (a.threads != 64 && a.threads != kEctThreads && !(a.threads == kEctWideThreads && direct_groups > 0))
        return hipErrorInvalidValue;
    const size_t shmem = sizeof(double) * a.M + (radon ? 2 : 1) * sizeof(int32_t) * a.dirs_per_group * a.M;
    hipError_t e = stage_mark(ECT_STAGE_ECT, false, stream);
    if (e != hipSuccess) return e;
    if (ndim == 2)
        e = radon ? launch_ect_typed<2, true>(a, grid, direct_groups, shmem, stream)
                  : launch_ect_typed<2, false>(a, grid, direct_groups, shmem, stream);
    else if (ndim == 3)
        e = radon ? launch_ect_typed<3, true>(a, grid, direct_groups, shmem, stream)
                  : launch_ect_typed<3, false>(a, grid, direct_groups, shmem, stream);
    else
        e = radon ? launch_ect_typed<4, true>(a, grid, direct_groups, shmem, stream)
                  : launch_ect_typed<4, false>(a, grid, direct_groups, shmem, stream);
    if (e != hipSuccess) return e;
    return stage_mark(ECT_STAGE_ECT, true, stream);
}

}  // namespace ect
