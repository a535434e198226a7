// Device code of the query bucketing that the bucketing kernels
// (queries.hip) and the compaction launch (precompute.hip, which can bucket a
// shared hybrid query set in a workgroup of its own) share: the record and
// bucket of one query, the sub-bin of a hybrid query, the counting sort of a
// shared set by one workgroup, and the one-wave work list.
#pragma once

#include "eval_internal.h"

namespace ect {

namespace {

// Bucket key and record of query row r with vector v in image img (rows
// [r0, r0 + q) of the set belong to it): returns the (image, bucket) entry.
template <int N>
__device__ __forceinline__ int64_t classify_vec(const double (&v)[N], int64_t r, int img, int64_t r0, int64_t q,
                                                int mode_hybrid, uint32_t* __restrict__ err, QRecT<N>* rec,
                                                int64_t* slot_base) {
    const int B = mode_hybrid ? (1 << (N - 1)) : (1 << N);
    const int full = (1 << N) - 1;
    constexpr int NV = sizeof(QRecT<N>::v) / sizeof(double);
    bool fin = true;
#pragma unroll
    for (int a = 0; a < NV; ++a) {
        rec->v[a] = a < N ? v[a < N ? a : 0] : 0.0;
        fin = fin && isfinite(rec->v[a]);
    }
    if (!fin && err) raise_error(err, ECT_DEVERR_NONFINITE);
    int e = sign_index<N>(rec->v);
    int neg = 0;
    if (mode_hybrid && ((e >> (N - 1)) & 1)) { e ^= full; neg = 1; }
    rec->code = 2 * (r - r0) + neg;
    *slot_base = B * r0 + e * q;
    return (int64_t)img * B + e;
}

constexpr int kSubBands = 16, kSubAngles = 32, kSubBins = kSubBands * kSubAngles;

template <int N>
__device__ __forceinline__ int sub_bin(const double* v) {
    double r2 = 0.0;
#pragma unroll
    for (int a = 0; a < N; ++a) r2 = fma(v[a], v[a], r2);
    // floor(log2 |xi|^2) from the exponent field; octaves of |xi| from 2^-12
    const int ex = (int)((__double_as_longlong(r2) >> 52) & 0x7ff) - 1023;
    const int lb = ex + 24 < 0 ? 0 : (ex + 24) >> 1;
    const int band = !(r2 > 0.0) ? 0 : (lb >= kSubBands ? kSubBands - 1 : lb);
    // angle of (xi_0, xi_1) modulo pi as a monotone "diamond" angle in [0, 2)
    float x = (float)v[0], y = (float)v[1];
    if (y < 0.0f || (y == 0.0f && x < 0.0f)) {
        x = -x;
        y = -y;
    }
    // (the hardware reciprocal: any bin is a valid order, the same query always
    // gets the same one)
    const float d = fabsf(x) + y;
    const float q = y * __builtin_amdgcn_rcpf(d);
    const float t = d > 0.0f ? (x >= 0.0f ? q : 2.0f - q) : 0.0f;
    const float f = t * (0.5f * kSubAngles);
    const int ab = f >= 0.0f && f < (float)kSubAngles ? (int)f : (f >= (float)kSubAngles ? kSubAngles - 1 : 0);
    return band * kSubAngles + ab;
}

// Counting sort of a shared hybrid query set of `rows` rows by (orthant
// pair, sub-bin) in one workgroup of any multiple of 64 threads: counts in
// LDS, their exclusive scan, then each record to its bin's next slot.  Writes
// the records and bcnt[pair]; leaves the pair counts in s_tot.  Every thread
// takes kSortRows rows per round, all loads of a round in flight together.
// s_bin holds 2^(N-1) * kSubBins counters, s_w one word per wave.
constexpr int kSortRows = 8;

constexpr int kKeepRows = 16;   // rows per thread kept in registers between the two phases

template <int N>
__device__ void sort_shared_queries(const double* __restrict__ vecs, int64_t rows, uint32_t* __restrict__ err,
                                    QRecT<N>* __restrict__ recs, int32_t* __restrict__ bcnt, int32_t* s_bin,
                                    int32_t* s_w, int32_t* s_tot, int32_t* s_start) {
    constexpr int B = 1 << (N - 1);
    const int nt = (int)blockDim.x, tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6, W = nt / 64;
    const int nbins = B * kSubBins;
    for (int i = tid; i < nbins; i += nt) s_bin[i] = 0;
    // up to kKeepRows rows per thread: every load of a phase in flight at
    // once, and only each row's bin kept in registers between the phases (the
    // second phase loads the rows again, from L2, to build the records)
    const bool keep = rows <= (int64_t)nt * kKeepRows;
    int kbin[kKeepRows];
    auto load_kept = [&](double (&v)[kKeepRows][N]) {
#pragma unroll
        for (int u = 0; u < kKeepRows; ++u)
#pragma unroll
            for (int a = 0; a < N; ++a) {
                const int64_t r = tid + (int64_t)u * nt;
                v[u][a] = r < rows ? vecs[r * N + a] : 0.0;
            }
    };
    if (keep) {
        double v[kKeepRows][N];
        load_kept(v);
#pragma unroll
        for (int u = 0; u < kKeepRows; ++u) {
            const int64_t r = tid + (int64_t)u * nt;
            kbin[u] = -1;
            if (r < rows) {
                QRecT<N> rec;
                int64_t sb;
                const int key = (int)classify_vec<N>(v[u], r, 0, 0, rows, 1, err, &rec, &sb);
                kbin[u] = key * kSubBins + sub_bin<N>(rec.v);
            }
        }
    }
    __syncthreads();
    if (keep) {
#pragma unroll
        for (int u = 0; u < kKeepRows; ++u)
            if (kbin[u] >= 0) atomicAdd(&s_bin[kbin[u]], 1);
    }
    for (int pass = 0; pass < 2; ++pass) {
        if (keep && pass == 1) {
            double v[kKeepRows][N];
            load_kept(v);
#pragma unroll
            for (int u = 0; u < kKeepRows; ++u) {
                if (kbin[u] < 0) continue;
                QRecT<N> rec;
                int64_t sb = 0;
                classify_vec<N>(v[u], tid + (int64_t)u * nt, 0, 0, rows, 1, nullptr, &rec, &sb);
                const int pos = atomicAdd(&s_bin[kbin[u]], 1) - s_start[kbin[u] / kSubBins];
                recs[sb + pos] = rec;
            }
            break;
        }
        // (kept rows were counted above)
        for (int64_t rb = tid; !keep && rb < rows; rb += (int64_t)nt * kSortRows) {
            double v[kSortRows][N];
#pragma unroll
            for (int u = 0; u < kSortRows; ++u)
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    const int64_t r = rb + (int64_t)u * nt;
                    v[u][a] = r < rows ? vecs[r * N + a] : 0.0;
                }
#pragma unroll
            for (int u = 0; u < kSortRows; ++u) {
                const int64_t r = rb + (int64_t)u * nt;
                if (r >= rows) break;
                QRecT<N> rec;
                int64_t sb = 0;
                const int key = (int)classify_vec<N>(v[u], r, 0, 0, rows, 1, pass == 0 ? err : nullptr, &rec, &sb);
                const int bin = key * kSubBins + sub_bin<N>(rec.v);
                if (pass == 0) {
                    atomicAdd(&s_bin[bin], 1);
                } else {
                    const int pos = atomicAdd(&s_bin[bin], 1) - s_start[key];
                    recs[sb + pos] = rec;
                }
            }
        }
        if (pass == 1) break;
        __syncthreads();
        // exclusive scan of the bins: a contiguous run of bins per thread
        const int bpt = (nbins + nt - 1) / nt;
        int32_t loc = 0;
        for (int j = 0; j < bpt; ++j) {
            const int i = tid * bpt + j;
            if (i < nbins) loc += s_bin[i];
        }
        int32_t inc = loc;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t o = __shfl_up(inc, off, 64);
            if (lane >= off) inc += o;
        }
        if (lane == 63) s_w[wave] = inc;
        __syncthreads();
        int32_t run = inc - loc, total = 0;
        for (int w = 0; w < W; ++w) {
            if (w < wave) run += s_w[w];
            total += s_w[w];
        }
        for (int j = 0; j < bpt; ++j) {
            const int i = tid * bpt + j;
            if (i < nbins) {
                const int32_t c = s_bin[i];
                s_bin[i] = run;
                run += c;
            }
        }
        __syncthreads();
        if (tid < B) {
            const int32_t start = s_bin[tid * kSubBins];
            const int32_t end = tid + 1 < B ? s_bin[(tid + 1) * kSubBins] : total;
            s_start[tid] = start;
            s_tot[tid] = end - start;
            bcnt[tid] = end - start;
        }
        __syncthreads();
    }
}

// Work list of at most 64 entries by one wave, lane = entry (no barrier):
// q = the entry's query count, np = its list size.  Same items, prefixes,
// chunk doubling and outputs as build_worklist.
__device__ void worklist_wave(int64_t E, int64_t q, int64_t np, int qtile, int64_t chunk0, int64_t capacity,
                              uint32_t* __restrict__ err, int64_t* __restrict__ item_off,
                              int64_t* __restrict__ tile_off, int64_t* __restrict__ params) {
    const int lane = threadIdx.x & 63;
    const bool valid = lane < E;
    const int64_t t = valid ? (q + qtile - 1) / qtile : 0;
    auto items_for = [&](int64_t chunk) {
        int64_t ch = chunk > 0 ? (np + chunk - 1) / chunk : 1;
        if (ch < 1) ch = 1;  // an empty list still gets one item per tile, which writes zeros
        return t * ch;
    };
    int64_t chunk = chunk0;
    if (chunk > 0 && capacity > 0) {
        for (int attempt = 0;; ++attempt) {
            int64_t total = items_for(chunk);
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) total += __shfl_xor(total, off, 64);
            if (total <= capacity) break;
            chunk *= 2;
            if (attempt == 39) {
                if (lane == 0) {
                    raise_error(err, ECT_DEVERR_CAPACITY);
                    params[0] = 0;
                    params[1] = 0;
                    params[2] = chunk;
                    item_off[E] = 0;
                    tile_off[E] = 0;
                }
                return;
            }
        }
    }
    int64_t it = items_for(chunk), tl = t, ii = it, ti = tl;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t a = __shfl_up(ii, off, 64), b = __shfl_up(ti, off, 64);
        if (lane >= off) { ii += a; ti += b; }
    }
    if (valid) {
        item_off[lane] = ii - it;
        tile_off[lane] = ti - tl;
    }
    const int64_t tot_i = __shfl(ii, 63, 64), tot_t = __shfl(ti, 63, 64);
    if (lane == 0) {
        item_off[E] = tot_i;
        tile_off[E] = tot_t;
        params[0] = tot_i;
        params[1] = tot_t;
        params[2] = chunk;
    }
}

}  // namespace

}  // namespace ect
