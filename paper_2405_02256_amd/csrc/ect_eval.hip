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
#include "eval_internal.h"

namespace ect {

namespace {

// Stage the thresholds of image img in LDS and clear the histograms; returns
// nonzero (in every thread) when they are not non-decreasing or not finite.
__device__ __forceinline__ int stage_thresholds(const EctArgs& a, int64_t img, double* s_thr, int32_t* s_hist,
                                                int hist_arrays = 1) {
    const int M = a.M;
    const double* thr = a.thresholds + (a.thr_per_image ? img * M : 0);
    int bad = 0;
    for (int j = threadIdx.x; j < M; j += kEctThreads) {
        const double v = thr[j];
        s_thr[j] = v;
        if (j > 0 && !(v >= thr[j - 1])) bad = 1;
        if (!isfinite(v)) bad = 1;
    }
    for (int j = threadIdx.x; j < hist_arrays * a.dirs_per_group * M; j += kEctThreads) s_hist[j] = 0;
    return __syncthreads_or(bad);
}

// Binning of a projection u against the non-decreasing thresholds:
//   kBinClosed  the first j with t_j >= u ({xi <= t} contains the point);
//   kBinOpen    the first j with t_j > u (the open ray (u, inf));
//   kBinPoint   every j with t_j == u (the point u itself).
constexpr int kBinClosed = 0, kBinOpen = 1, kBinPoint = 2;

// Stream points [p0, p1) of one list and add sign * (critical value) into the
// histogram of every direction dd with use[dd].
template <int N, int MODE>
__device__ __forceinline__ void accumulate_list(const PointT<N>* __restrict__ pts, int64_t p0, int64_t p1,
                                                const double (&xi)[kEctMaxDirs][N], const bool (&use)[kEctMaxDirs],
                                                const double* s_thr, int M, int32_t* s_hist, int32_t sign = 1) {
    const double t0 = s_thr[0], t1 = s_thr[M - 1];
    const double inv = (M > 1 && t1 > t0) ? (double)(M - 1) / (t1 - t0) : 0.0;
    // U points per thread are loaded before any is processed, so that their
    // memory latencies overlap
    constexpr int U = 4;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += (int64_t)kEctThreads * U) {
        PointT<N> pt[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t pp = p + (int64_t)u * kEctThreads;
            if (pp < p1) pt[u] = pts[pp];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (p + (int64_t)u * kEctThreads >= p1) break;
            const int32_t val = sign * (int32_t)pt[u].val;
#pragma unroll
            for (int dd = 0; dd < kEctMaxDirs; ++dd) {
                if (!use[dd]) continue;
                const double uu = project<N>(xi[dd], pt[u].x);
                double g = ceil((uu - t0) * inv);
                g = fmin(fmax(g, 0.0), (double)M);
                int j = (int)g;
                // first j with t_j >= u
                while (j > 0 && s_thr[j - 1] >= uu) --j;
                while (j < M && s_thr[j] < uu) ++j;
                if constexpr (MODE == kBinClosed) {
                    if (j < M) atomicAdd(&s_hist[dd * M + j], val);
                } else if constexpr (MODE == kBinOpen) {
                    while (j < M && s_thr[j] == uu) ++j;
                    if (j < M) atomicAdd(&s_hist[dd * M + j], val);
                } else {
                    for (; j < M && s_thr[j] == uu; ++j) atomicAdd(&s_hist[dd * M + j], val);
                }
            }
        }
    }
}

// Inclusive prefix sum of each histogram into its output row (zeros for an
// invalid direction); one wave per direction.
__device__ __forceinline__ void write_rows(const EctArgs& a, int nd, const int64_t* s_row, const int* s_valid,
                                           const int32_t* s_hist, const int32_t* s_point = nullptr) {
    const int M = a.M;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int W = kEctThreads / 64;
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
            if (j < M) out[j] = carry + v + (s_point ? s_point[dd * M + j] : 0);
            carry += __shfl(v, 63, 64);
        }
    }
}

// Radon transform: the classical list of eps at the thresholds it hits, the
// ordinary list of eps's orthant pair (negated when eps is the mirrored half)
// on the open rays.
template <int N>
__device__ __forceinline__ void accumulate_radon(const EctArgs& a, int64_t img, int e, int64_t chunk, int64_t chunks,
                                                 const double (&xi)[kEctMaxDirs][N], const bool (&use)[kEctMaxDirs],
                                                 const double* s_thr, int32_t* s_hist, int32_t* s_point) {
    constexpr int full = (1 << N) - 1;
    const int M = a.M;
    const int64_t c0 = a.list_off[img * a.NL + e], c1 = a.list_off[(img + 1) * a.NL + e];
    const int64_t cl = c1 - c0;
    accumulate_list<N, kBinPoint>(list_points<N>(a.points, a.capacity, e), c0 + cl * chunk / chunks,
                                  c0 + cl * (chunk + 1) / chunks, xi, use, s_thr, M, s_point);
    const bool mirrored = (e >> (N - 1)) & 1;
    const int l = (1 << N) + (mirrored ? (e ^ full) : e);
    const int64_t o0 = a.list_off[img * a.NL + l], o1 = a.list_off[(img + 1) * a.NL + l];
    const int64_t ol = o1 - o0;
    accumulate_list<N, kBinOpen>(list_points<N>(a.points, a.capacity, l), o0 + ol * chunk / chunks,
                                 o0 + ol * (chunk + 1) / chunks, xi, use, s_thr, M, s_hist, mirrored ? 1 : -1);
}

__device__ __forceinline__ void zero_rows(const EctArgs& a, int nd, const int64_t* s_row) {
    for (int dd = 0; dd < nd; ++dd)
        for (int j = threadIdx.x; j < a.M; j += kEctThreads) a.out[s_row[dd] * a.M + j] = 0;
}

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
        accumulate_list<N, kBinClosed>(list_points<N>(a.points, a.capacity, b), p0, p1, xi, use, s_thr, M, s_hist);
    }
    __syncthreads();
    write_rows(a, nd, s_row, s_valid, s_hist, RADON ? s_point : nullptr);
}

// Shared query sets: no bucketing pass.  Workgroup (image, g, c) takes rows
// [g * dirs_per_group, ...) of the set in input order and, for each distinct
// sign vector among them (one pass when neighbouring directions share an
// orthant, as in angle-ordered sets), streams the c-th of `chunks` equal parts
// of that list once for the directions that have it.  Splitting the lists
// lets many workgroups share one group of directions, so each streamed point
// serves up to eight directions while the chip stays full.  One chunk writes
// the ECT rows itself; several write their histograms, which
// ect_chunk_sum_kernel adds (integers, so the order cannot matter) before the
// prefix sum.  A non-finite direction gets a zero row and raises
// ECT_DEVERR_NONFINITE, as in the bucketed path.
template <int N, bool RADON>
__global__ void __launch_bounds__(kEctThreads) ect_direct_kernel(EctArgs a, int64_t groups) {
    extern __shared__ __align__(16) char smem[];
    constexpr int TD = kEctMaxDirs;
    const int M = a.M;
    double* s_thr = (double*)smem;
    int32_t* s_hist = (int32_t*)(smem + sizeof(double) * M);
    __shared__ double s_xi[TD][kMaxDim];
    __shared__ int64_t s_row[TD];
    __shared__ int s_valid[TD];
    __shared__ int s_sign[TD];
    __shared__ int64_t s_loff[2][1 << N];

    const int tid = threadIdx.x;
    const int64_t chunks = a.chunks;
    const int64_t c = blockIdx.x % chunks;
    const int64_t rest = blockIdx.x / chunks;
    const int64_t img = rest / groups;
    const int64_t g = rest % groups;
    const int TDg = a.dirs_per_group;
    const int64_t q0 = g * TDg;
    const int nd = (int)min<int64_t>(TDg, a.count - q0);
    if (tid < TD) {
        int ok = 0, sg = 0;
        int64_t row = -1;
        if (tid < nd) {
            const int64_t q = q0 + tid;
            row = img * a.count + q;
            double v[kMaxDim] = {};
            ok = 1;
#pragma unroll
            for (int cc = 0; cc < N; ++cc) {
                v[cc] = a.vecs[q * N + cc];
                ok &= isfinite(v[cc]) ? 1 : 0;
            }
#pragma unroll
            for (int cc = 0; cc < kMaxDim; ++cc) s_xi[tid][cc] = v[cc];
            sg = sign_index<N>(v);
            if (!ok && c == 0) raise_error(a.err, ECT_DEVERR_NONFINITE);
        }
        s_row[tid] = row;
        s_valid[tid] = ok;
        s_sign[tid] = sg;
    }
    // every classical list's bounds are requested now, with the directions and
    // thresholds, instead of after the barrier
    if (tid >= 64 && tid < 64 + (2 << N)) {
        const int k = tid - 64, b = k & ((1 << N) - 1), hi = k >> N;
        s_loff[hi][b] = a.list_off[(img + hi) * a.NL + b];
    }
    int32_t* s_point = s_hist + (int64_t)a.dirs_per_group * M;   // Radon point values
    const int bad = stage_thresholds(a, img, s_thr, s_hist, RADON ? 2 : 1);
    if (bad) {
        if (tid == 0 && c == 0) raise_error(a.err, ECT_DEVERR_THRESHOLDS);
    } else {
        double xi[TD][N];
        int sgn[TD];
        bool pending[TD];
#pragma unroll
        for (int dd = 0; dd < TD; ++dd) {
            pending[dd] = dd < nd && s_valid[dd];
            sgn[dd] = s_sign[dd];
#pragma unroll
            for (int cc = 0; cc < N; ++cc) xi[dd][cc] = s_xi[dd][cc];
        }
        // one pass per distinct sign vector, in order of first appearance
        for (int pass = 0; pass < TD; ++pass) {
            int b = -1;
#pragma unroll
            for (int dd = TD - 1; dd >= 0; --dd)
                if (pending[dd]) b = sgn[dd];
            if (b < 0) break;
            bool use[TD];
#pragma unroll
            for (int dd = 0; dd < TD; ++dd) {
                use[dd] = pending[dd] && sgn[dd] == b;
                if (use[dd]) pending[dd] = false;
            }
            if constexpr (RADON) {
                accumulate_radon<N>(a, img, b, c, chunks, xi, use, s_thr, s_hist, s_point);
            } else {
                const int64_t p0 = s_loff[0][b], p1 = s_loff[1][b];
                const int64_t len = p1 - p0;
                accumulate_list<N, kBinClosed>(list_points<N>(a.points, a.capacity, b), p0 + len * c / chunks,
                                               p0 + len * (c + 1) / chunks, xi, use, s_thr, M, s_hist);
            }
        }
    }
    __syncthreads();
    if (chunks == 1) {
        if (bad) zero_rows(a, nd, s_row);
        else write_rows(a, nd, s_row, s_valid, s_hist, RADON ? s_point : nullptr);
        return;
    }
    // chunk histograms (zeros for invalid directions or bad thresholds)
    int32_t* part = a.part + (rest * chunks + c) * (int64_t)TDg * M;
    for (int j = tid; j < nd * M; j += kEctThreads) part[j] = s_hist[j];
}

// Sum of the chunk histograms of one direction (one wave per output row) and
// the inclusive prefix over thresholds.
__global__ void __launch_bounds__(64) ect_chunk_sum_kernel(EctArgs a, int64_t groups) {
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
    const int32_t* part = a.part + rest * chunks * (int64_t)TDg * M + dd * M;
    int32_t carry = 0;
    for (int jb = 0; jb < M; jb += 64) {
        const int j = jb + lane;
        int32_t v = 0;
        if (j < M)
            for (int64_t c = 0; c < chunks; ++c) v += part[c * TDg * M + j];
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t o = __shfl_up(v, off, 64);
            if (lane >= off) v += o;
        }
        if (j < M) out[j] = carry + v;
        carry += __shfl(v, 63, 64);
    }
}

template <int N, bool RADON>
hipError_t launch_ect_typed(const EctArgs& a, int64_t grid, int64_t direct_groups, size_t shmem, hipStream_t stream) {
    if (direct_groups > 0) {
        hipLaunchKernelGGL((ect_direct_kernel<N, RADON>), dim3((unsigned)grid), dim3(kEctThreads), shmem, stream, a,
                           direct_groups);
        if (a.chunks > 1) {
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            const int64_t rows = (grid / a.chunks) * a.dirs_per_group;
            hipLaunchKernelGGL(ect_chunk_sum_kernel, dim3((unsigned)rows), dim3(64), 0, stream, a, direct_groups);
        }
    } else {
        hipLaunchKernelGGL((ect_kernel<N, RADON>), dim3((unsigned)grid), dim3(kEctThreads), shmem, stream, a);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_ect(int ndim, const EctArgs& a, int64_t grid, int64_t direct_groups, bool radon,
                      hipStream_t stream) {
    if (grid <= 0) return hipSuccess;
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
