// Device code of the ECT and the Radon transform at thresholds that the
// threshold kernels (ect_eval.hip) and the combined ECT + hybrid launch
// (hybrid.hip) share: threshold staging, list streaming into LDS histograms,
// the prefix-sum write-out, and the shared-set direct evaluation of one
// workgroup's block.  Everything strides by the launch's workgroup size, a
// multiple of 64 up to kEctThreads: short lists are evaluated by one-wave
// workgroups, so that four times as many (image, directions) blocks are in
// flight to cover their memory latency.
#pragma once

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
    const int nt = (int)blockDim.x;
    for (int j = threadIdx.x; j < M; j += nt) {
        const double v = thr[j];
        s_thr[j] = v;
        if (j > 0 && !(v >= thr[j - 1])) bad = 1;
        if (!isfinite(v)) bad = 1;
    }
    for (int j = threadIdx.x; j < hist_arrays * a.dirs_per_group * M; j += nt) s_hist[j] = 0;
    return __syncthreads_or(bad);
}

// Binning of a projection u against the non-decreasing thresholds:
//   kBinClosed  the first j with t_j >= u ({xi <= t} contains the point);
//   kBinOpen    the first j with t_j > u (the open ray (u, inf));
//   kBinPoint   every j with t_j == u (the point u itself).
constexpr int kBinClosed = 0, kBinOpen = 1, kBinPoint = 2;

// First j with t_j >= u among the M non-decreasing thresholds in LDS (M if
// none): an arithmetic guess for evenly spaced thresholds (inv = (M - 1) /
// (t_{M-1} - t_0), or 0), corrected against the stored values, so any
// non-decreasing array gives the exact bin.
__device__ __forceinline__ int bin_closed(double uu, const double* s_thr, int M, double t0, double inv) {
    double g = ceil((uu - t0) * inv);
    g = fmin(fmax(g, 0.0), (double)M);
    int j = (int)g;
    while (j > 0 && s_thr[j - 1] >= uu) --j;
    while (j < M && s_thr[j] < uu) ++j;
    return j;
}

// Stream points [p0, p1) of one list and add sign * (critical value) into the
// histogram of every direction dd with use[dd].
template <int N, int MODE, int TD>
__device__ __forceinline__ void accumulate_list(const ListEntry* __restrict__ pts, const ImageDesc& d, int64_t p0,
                                                int64_t p1, const double (&xi)[TD][N], const bool (&use)[TD],
                                                const double* s_thr, int M, int32_t* s_hist, int32_t sign = 1) {
    const double t0 = s_thr[0], t1 = s_thr[M - 1];
    const double inv = (M > 1 && t1 > t0) ? (double)(M - 1) / (t1 - t0) : 0.0;
    // U points per thread are loaded before any is processed, so that their
    // memory latencies overlap
    constexpr int U = 4;
    const int64_t nt = blockDim.x;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += nt * U) {
        ListEntry en[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t pp = p + (int64_t)u * nt;
            if (pp < p1) en[u] = pts[pp];
        }
        PointT<N> pt[U];
#pragma unroll
        for (int u = 0; u < U; ++u) pt[u] = decode_entry<N>(en[u], d);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (p + (int64_t)u * nt >= p1) break;
            const int32_t val = sign * (int32_t)pt[u].val;
#pragma unroll
            for (int dd = 0; dd < TD; ++dd) {
                if (!use[dd]) continue;
                const double uu = project<N>(xi[dd], pt[u].x);
                int j = bin_closed(uu, s_thr, M, t0, inv);
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
    const int W = (int)blockDim.x / 64;
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
template <int N, int TD>
__device__ __forceinline__ void accumulate_radon(const EctArgs& a, int64_t img, int e, int64_t chunk, int64_t chunks,
                                                 const double (&xi)[TD][N], const bool (&use)[TD],
                                                 const double* s_thr, int32_t* s_hist, int32_t* s_point) {
    constexpr int full = (1 << N) - 1;
    const int M = a.M;
    const int64_t c0 = a.list_off[img * a.NL + e], c1 = a.list_off[(img + 1) * a.NL + e];
    const int64_t cl = c1 - c0;
    accumulate_list<N, kBinPoint>(list_entries(a.points, a.capacity, e), a.desc[img], c0 + cl * chunk / chunks,
                                  c0 + cl * (chunk + 1) / chunks, xi, use, s_thr, M, s_point);
    const bool mirrored = (e >> (N - 1)) & 1;
    const int l = (1 << N) + (mirrored ? (e ^ full) : e);
    const int64_t o0 = a.list_off[img * a.NL + l], o1 = a.list_off[(img + 1) * a.NL + l];
    const int64_t ol = o1 - o0;
    accumulate_list<N, kBinOpen>(list_entries(a.points, a.capacity, l), a.desc[img], o0 + ol * chunk / chunks,
                                 o0 + ol * (chunk + 1) / chunks, xi, use, s_thr, M, s_hist, mirrored ? 1 : -1);
}

__device__ __forceinline__ void zero_rows(const EctArgs& a, int nd, const int64_t* s_row) {
    for (int dd = 0; dd < nd; ++dd)
        for (int j = threadIdx.x; j < a.M; j += (int)blockDim.x) a.out[s_row[dd] * a.M + j] = 0;
}

// Shared query sets: no bucketing pass.  Workgroup (image, g, c) takes rows
// [g * dirs_per_group, ...) of the set in input order and, for each distinct
// sign vector among them (one pass when neighbouring directions share an
// orthant, as in angle-ordered sets), streams the c-th of `chunks` equal parts
// of that list once for the directions that have it.  Splitting the lists
// lets many workgroups share one group of directions, so each streamed point
// serves up to eight directions while the chip stays full.  One chunk writes
// the rows itself; several write their histograms (and, for the Radon
// transform, their point values), which ect_chunk_sum_kernel adds (integers,
// so the order cannot matter) before the prefix sum.  A non-finite direction gets a zero row and raises
// ECT_DEVERR_NONFINITE, as in the bucketed path.  TD bounds dirs_per_group
// (the caller checks it); a smaller bound keeps fewer directions in registers.
template <int N, bool RADON, int TD = kEctMaxDirs>
__device__ __forceinline__ void ect_direct_block(const EctArgs& a, int64_t groups, int64_t block) {
    extern __shared__ __align__(16) char smem[];
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
    const int64_t c = block % chunks;
    const int64_t rest = block / chunks;
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
    // thresholds, instead of after the barrier (by the second wave, or by the
    // only one)
    const int kl = blockDim.x > 64 ? tid - 64 : tid;
    if (kl >= 0 && kl < (2 << N)) {
        const int k = kl, b = k & ((1 << N) - 1), hi = k >> N;
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
                accumulate_list<N, kBinClosed>(list_entries(a.points, a.capacity, b), a.desc[img], p0 + len * c / chunks,
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
    // chunk histograms, and for the Radon transform the chunk's point values
    // after them (zeros for invalid directions or bad thresholds)
    constexpr int arrays = RADON ? 2 : 1;
    int32_t* part = a.part + (rest * chunks + c) * (int64_t)arrays * TDg * M;
    for (int j = tid; j < arrays * TDg * M; j += (int)blockDim.x) part[j] = s_hist[j];
}

}  // namespace

}  // namespace ect
