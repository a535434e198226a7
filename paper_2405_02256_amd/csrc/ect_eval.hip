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
// directions kBatchDirs at a time.  The list is streamed a stage of 256
// points at a time, one point per thread (decoded once, the next stage's
// entries in flight), and each thread bins its point on every direction of
// the pass in turn (the point stays in registers, the directions come from
// LDS).
//
// Binning: the first j with t_j >= u.  The workgroup measures, once, how far
// its thresholds stray from evenly spaced ones, in bins (tol, plus a margin
// for the rounding of the position p = (u - t_0)(M - 1)/(t_{M-1} - t_0)).
// With p clamped to [-1/2, M - 1/2], when p is farther than tol from every
// integer the bin is ceil(p) exactly (0 below t_0, M above t_{M-1});
// otherwise (a projection within rounding of a threshold, or uneven
// thresholds) it is searched among the thresholds in LDS, which sit between
// -inf and +inf sentinels.  The critical value is added into the direction's
// LDS histogram (integer atomics; rows of M + 1 bins at an odd stride, bin M
// unused); a non-finite direction bins as the zero vector (its row is not
// written).  Thread t takes the pass's directions starting at t mod nd, so
// the lanes of one atomic spread over the rows.  The histograms are then
// prefix-summed in place by kSeg threads per row (a sequential scan of a
// segment, then a scan of the segment totals), and written out row by row
// with consecutive threads on consecutive thresholds.  Same bins as the other
// threshold kernels, so the rows are the same integers.
template <int N>
__global__ void __launch_bounds__(kBatchThreads) ect_batch_kernel(EctArgs a) {
    extern __shared__ __align__(16) char smem[];
    constexpr int B = 1 << N;
    constexpr int kSeg = kBatchThreads / kBatchDirs;   // threads per histogram row in the scan
    constexpr int W = kBatchThreads / 64;
    const int M = a.M;
    const int MS = batch_row_stride(M);
    double* s_tp = (double*)smem;                                          // [M + 2]
    int32_t* s_hist = (int32_t*)(smem + batch_hist_offset(M));             // [kBatchDirs][MS]
    __shared__ double s_xi[kBatchDirs][N];
    __shared__ int64_t s_row[kBatchDirs];
    __shared__ int s_valid[kBatchDirs];
    __shared__ double s_dev[W];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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
    const double t0i = t0 * inv;
    // largest distance of a threshold's position from its index, in bins
    double dv = 0.0;
    for (int j = tid; j < M; j += kBatchThreads) dv = fmax(dv, fabs(fma(s_tp[j + 1], inv, -t0i) - (double)j));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) dv = fmax(dv, __shfl_xor(dv, off, 64));
    if (lane == 0) s_dev[wave] = dv;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < W; ++w) dv = fmax(dv, s_dev[w]);
    // the position's rounding (fma of |u inv| and |t0 inv|, both below M + |t0 inv| + 1 where it matters)
    // and the measurement's own; tol >= 0.5 never certifies
    const double tol = (inv > 0.0 && !bad) ? dv + ((double)M + 4.0 + fabs(t0i)) * 0x1p-48 : 1.0;
    const double p_hi = (double)M - 0.5;
    const int seg = (M + kSeg - 1) / kSeg;
    const int rows_per_pass = M <= kBatchThreads ? kBatchThreads / M : 1;
    const int wrow = M <= kBatchThreads ? tid / M : 0;
    const int wj = M <= kBatchThreads ? tid - wrow * M : tid;

    for (int64_t q0 = 0; q0 < qn; q0 += kBatchDirs) {
        const int nd = (int)min<int64_t>(kBatchDirs, qn - q0);
        if (tid < kBatchDirs) {
            // a non-finite direction bins as the zero vector (its row is not written)
            int ok = 0;
            int64_t row = -1;
            double v[N];
#pragma unroll
            for (int c = 0; c < N; ++c) v[c] = 0.0;
            if (tid < nd) {
                const QRecT<N> r = recs[q0 + tid];
                row = img * a.count + (r.code >> 1);
                ok = 1;
#pragma unroll
                for (int c = 0; c < N; ++c) ok &= isfinite(r.v[c]) ? 1 : 0;
                if (ok) {
#pragma unroll
                    for (int c = 0; c < N; ++c) v[c] = r.v[c];
                } else if (img == 0) {
                    raise_error(a.err, ECT_DEVERR_NONFINITE);
                }
            }
#pragma unroll
            for (int c = 0; c < N; ++c) s_xi[tid][c] = v[c];
            s_row[tid] = row;
            s_valid[tid] = ok && !bad;
        }
        {
            int4* h4 = (int4*)s_hist;
            const int n4 = kBatchDirs * MS / 4;   // kBatchDirs is a multiple of 4
            for (int j = tid; j < n4; j += kBatchThreads) h4[j] = make_int4(0, 0, 0, 0);
        }
        __syncthreads();
        const int dd0 = tid % nd;
        for (int64_t base = p0; base < p1; base += kBatchThreads) {
            const bool has = base + tid < p1;
            const PointT<N> pt = decode_entry<N>(nxt, dsc);
            const int32_t val = nxt.val;
            // next stage, or after the last one the list's start for the next pass
            const int64_t nb = base + kBatchThreads;
            const int64_t src = nb < p1 ? nb + tid : (q0 + kBatchDirs < qn ? p0 + tid : p1);
            if (src < p1) nxt = pts[src];
            if (has) {
                // thread t starts at direction t mod nd and walks through all nd of
                // them, so one instruction's atomics spread over the directions'
                // rows instead of piling onto the few bins of one direction
                int dd = dd0;
                for (int step = 0; step < nd; ++step, dd = (dd + 1 == nd) ? 0 : dd + 1) {
                    const double u = project<N>(s_xi[dd], pt.x);
                    // position clamped to [-1/2, M - 1/2]: below t_0 or above
                    // t_{M-1} (by more than tol) the bin is 0 or M and certain
                    const double p = fmin(fmax(fma(u, inv, -t0i), -0.5), p_hi);
                    const double g = ceil(p);
                    const double rr = g - p;
                    int j = (int)g;
                    if (!(fmin(rr, 1.0 - rr) > tol)) {
                        // within rounding of a threshold: search (t_{j-1} < u <= t_j)
                        while (j > 0 && s_tp[j] >= u) --j;
                        while (j < M && s_tp[j + 1] < u) ++j;
                    }
                    atomicAdd(&s_hist[dd * MS + j], val);   // bin M: above every threshold, not written
                }
            }
        }
        __syncthreads();
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
            // inclusive scan of the segment totals within the row's kSeg = 16
            // lanes: DPP row shifts (a DPP row is 16 lanes; lanes shifted in
            // from outside the row read 0)
            static_assert(kSeg == 16, "one DPP row per histogram row");
            int32_t off = run;
            off += __builtin_amdgcn_update_dpp(0, off, 0x111, 0xf, 0xf, false);   // row_shr:1
            off += __builtin_amdgcn_update_dpp(0, off, 0x112, 0xf, 0xf, false);   // row_shr:2
            off += __builtin_amdgcn_update_dpp(0, off, 0x114, 0xf, 0xf, false);   // row_shr:4
            off += __builtin_amdgcn_update_dpp(0, off, 0x118, 0xf, 0xf, false);   // row_shr:8
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
