// Exact representations of the ECT and of the Radon transform along each
// query direction (Sec. 4.3), built from the critical-point lists.
//
// ECT: the classical points of eps(xi) sorted by projection, equal
// projections merged, and the running sum of their critical values:
// T = [-inf, t_1 < ... < t_k], E[i] = ECT(xi, t) for t in [T[i], T[i+1]).
//
// Radon (with the sign the definition gives, see ect_eval.hip): the ordinary
// points of the orthant pair, sorted and merged the same way with the values
// -D (the mirrored half of the pair carries +stored value), give
// (T, E'): R(xi, t) = E'[i] for the largest T[i] < t away from classical
// projections; the distinct classical projections Tc carry
// Ec = E'[largest T[i] < Tc] + the classical values at Tc.
//
// One workgroup builds one row in one launch: it reads the row's list (or
// lists), turns each canonical FP64 projection into an order-preserving
// 64-bit key and sorts (key, value) pairs in LDS.  The sort is a bucket sort:
// the projection range [lo, hi] of the tile is cut into about as many buckets
// as the tile has points (a monotone map, so bucket order is key order), an
// LDS histogram and a block scan place every point in its bucket, and a
// point's place inside its bucket is the number of bucket members with
// smaller keys.  Tiles whose largest bucket holds more than kBucketMax points
// (projections clustered far below the range's resolution) are sorted by a
// bitonic network instead, whose cost does not depend on the data.  A block
// scan of head flags and values then merges equal keys and writes the
// distinct entries.  A list longer than one LDS tile is sorted tile by tile
// into the workspace and the sorted tiles are merged pairwise there by the
// same workgroup (merge path), before the same merge of equal keys.  For
// Radon, each classical entry then takes E' from a binary search in the
// row's T.  Global memory written by the workgroup is read back by it only
// after a workgroup barrier.
#include <rocprim/device/device_scan.hpp>

#include "exact_internal.h"

namespace ect {

namespace {

constexpr int kRowThreads = 256;
constexpr int kFinThreads = 512;         // the row-building workgroup
constexpr int kFinWaves = kFinThreads / 64;
constexpr int kFinItems = 4;            // consecutive sorted entries per thread per step (long lists)
constexpr int kFinStep = kFinThreads * kFinItems;
constexpr int kMergeItems = 8;          // outputs per thread per step of a pairwise merge
constexpr int kBucketMax = 64;          // largest bucket ranked by comparisons
constexpr int kEvalThreads = 256;
constexpr int kFixThreads = 256;
constexpr int kFixSamples = 4096;       // entries of T a Radon fix-up workgroup stages
constexpr uint64_t kTopBit = 0x8000000000000000ull;

// Order-preserving key of a finite or infinite FP64 value (-0 taken as +0):
// non-negative values get the top bit set, negative values are inverted.
__device__ __forceinline__ uint64_t order_key(double u) {
    const uint64_t b = (uint64_t)__double_as_longlong(u + 0.0);
    return (b & kTopBit) ? ~b : (b | kTopBit);
}

__device__ __forceinline__ double key_value(uint64_t k) {
    const uint64_t b = (k & kTopBit) ? (k & ~kTopBit) : ~k;
    return __longlong_as_double((long long)b);
}

// Image of query row r: r / count for a shared set, else the image i with
// offsets[i] <= r < offsets[i+1].
__device__ __forceinline__ int64_t row_image(const ExactArgs& a, int64_t r) {
    if (!a.offsets) return r / a.count;
    int64_t lo = 0, hi = a.num_images - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (a.offsets[mid] <= r) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Everything the later steps need about row r, and the entries it needs in
// the output (ECT: classical points + 1; Radon: ordinary points + 1 +
// classical points; a non-finite direction: 1).
template <int N>
__device__ __forceinline__ int64_t row_info(const ExactArgs& a, int64_t r, ExactRow& ri) {
    constexpr int B = 1 << N, full = B - 1;
    const int64_t img = row_image(a, r);
    ri.img = img;
    const double* v = a.vecs + (a.offsets ? r : r % a.count) * N;
    int ok = 1;
#pragma unroll
    for (int c = 0; c < kMaxDim; ++c) {
        const double x = c < N ? v[c] : 0.0;
        ri.xi[c] = x;
        ok &= isfinite(x) ? 1 : 0;
    }
    ri.valid = ok;
    ri.nc = ri.no = 0;
    ri.pc = ri.po = 0;
    ri.sign_o = -1;
    if (!ok) return 1;
    const int e = sign_index<N>(ri.xi);
    const int64_t* lo = a.list_off + img * a.NL;
    const int64_t* hi = lo + a.NL;
    ri.pc = (int64_t)e * a.list_capacity + lo[e];
    ri.nc = hi[e] - lo[e];
    if (a.kind == ECT_EXACT_ECT) return ri.nc + 1;
    const bool mirrored = (e >> (N - 1)) & 1;
    const int l = B + (mirrored ? (e ^ full) : e);
    ri.po = (int64_t)l * a.list_capacity + lo[l];
    ri.no = hi[l] - lo[l];
    ri.sign_o = mirrored ? 1 : -1;
    return ri.no + 1 + ri.nc;
}

template <int N>
__global__ void __launch_bounds__(kRowThreads) exact_need_kernel(ExactArgs a, int64_t* need) {
    const int64_t r = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (r > a.rows) return;
    if (r == a.rows) {
        need[r] = 0;
        return;
    }
    ExactRow ri;
    need[r] = row_info<N>(a, r, ri);
}

// Exclusive block scan of (count, sum) pairs over kFinThreads threads; also
// returns the block totals.
__device__ __forceinline__ void block_scan2(int32_t c, int32_t v, int32_t& c_ex, int32_t& v_ex, int32_t& c_tot,
                                            int32_t& v_tot, int32_t (*s_wave)[2]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int W = kFinThreads / 64;
    int32_t ci = c, vi = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t oc = __shfl_up(ci, off, 64), ov = __shfl_up(vi, off, 64);
        if (lane >= off) {
            ci += oc;
            vi += ov;
        }
    }
    if (lane == 63) {
        s_wave[wave][0] = ci;
        s_wave[wave][1] = vi;
    }
    __syncthreads();
    int32_t pc = 0, pv = 0, tc = 0, tv = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        if (w < wave) {
            pc += s_wave[w][0];
            pv += s_wave[w][1];
        }
        tc += s_wave[w][0];
        tv += s_wave[w][1];
    }
    __syncthreads();   // s_wave is reused by the next call
    c_ex = pc + ci - c;
    v_ex = pv + vi - v;
    c_tot = tc;
    v_tot = tv;
}

// Merge equal keys of the sorted segment [sb, se) into distinct entries
// out_T[j], out_E[j] (j = 0, 1, ...): the value written at entry j is the
// running sum of every value up to the last entry with that key.  Returns the
// number of distinct keys (in every thread).
__device__ int64_t merge_segment(const uint64_t* __restrict__ keys, const int32_t* __restrict__ vals, int64_t sb,
                                 int64_t se, double* out_T, int32_t* out_E, int32_t (*s_wave)[2]) {
    int64_t distinct = 0;
    int32_t run = 0;
    for (int64_t g0 = sb; g0 < se; g0 += kFinStep) {
        const int64_t i0 = g0 + (int64_t)threadIdx.x * kFinItems;
        uint64_t k[kFinItems + 1];
        int32_t v[kFinItems];
        // k[0] is the key before this thread's first entry (none at sb)
        k[0] = (i0 > sb && i0 <= se) ? keys[i0 - 1] : 0;
#pragma unroll
        for (int u = 0; u < kFinItems; ++u) {
            const int64_t i = i0 + u;
            k[u + 1] = i < se ? keys[i] : 0;
            v[u] = i < se ? vals[i] : 0;
        }
        int32_t heads = 0, sum = 0;
#pragma unroll
        for (int u = 0; u < kFinItems; ++u) {
            const int64_t i = i0 + u;
            if (i < se) {
                heads += (i == sb || k[u + 1] != k[u]) ? 1 : 0;
                sum += v[u];
            }
        }
        int32_t h_ex, s_ex, h_tot, s_tot;
        block_scan2(heads, sum, h_ex, s_ex, h_tot, s_tot, s_wave);
        int64_t h = distinct + h_ex;   // heads before this entry
        int32_t c = run + s_ex;        // values before this entry
#pragma unroll
        for (int u = 0; u < kFinItems; ++u) {
            const int64_t i = i0 + u;
            if (i >= se) break;
            h += (i == sb || k[u + 1] != k[u]) ? 1 : 0;
            c += v[u];
            const bool tail = (i + 1 == se) || (u + 1 < kFinItems ? k[u + 2] != k[u + 1] : keys[i + 1] != k[u + 1]);
            if (tail) {
                out_T[h - 1] = key_value(k[u + 1]);
                out_E[h - 1] = c;
            }
        }
        distinct += h_tot;
        run += s_tot;
    }
    return distinct;
}


// A direction passed by value (kept in registers across calls).
template <int N>
struct Dir {
    double v[N];
};

// LDS of one tile of C points (C a power of two, a multiple of the workgroup
// size): keys and values in sorted order once a sort returns, and the bucket
// starts (start[b] = first slot of bucket b, start[nb] = points).
template <int C>
struct TileLds {
    uint64_t key[C];
    int32_t val[C];
    int32_t start[C + 1];
};

// Small per-workgroup LDS: the wave totals of the striped scans and the
// scratch of block_scan2.
constexpr int kScanSlots = 128;   // rounds x waves of the largest striped scan
constexpr int kMaxRuns = 64;     // runs of coarse buckets of one long list
struct RowSmall {
    int32_t tot[2][kScanSlots];
    int32_t wave[kFinWaves][2];
    int32_t run_b[kMaxRuns + 1];  // first coarse bucket and first point of each run
    int32_t run_s[kMaxRuns + 1];
};

// Inclusive scan over the 64 lanes of a wave with DPP moves (no LDS): shifts
// by 1, 2, 4 and 8 inside each row of 16 lanes (lanes shifted in from
// outside the row read 0), then the last lane of row 0 added to row 1 and of
// row 2 to row 3 (row_bcast:15), then the last lane of row 1 added to rows 2
// and 3 (row_bcast:31).
__device__ __forceinline__ int32_t wave_scan(int32_t x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);   // row_bcast:15 -> rows 1, 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);   // row_bcast:31 -> rows 2, 3
    return x;
}

// Exclusive scans of two sequences held striped over the workgroup: element
// u * kFinThreads + t of each is x[u], y[u] of thread t (u < rounds, every
// LDS access of the callers consecutive across lanes).  On return x[u], y[u]
// hold the sums of the elements before it and tx, ty the totals.  One
// barrier between the wave scans and the scan of the wave totals.
template <int R>
__device__ __forceinline__ void striped_scan2(int32_t (&x)[R], int32_t (&y)[R], int rounds, int32_t& tx, int32_t& ty,
                                              RowSmall& sm) {
    static_assert(R * kFinWaves <= kScanSlots, "scan slots");
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
    for (int u = 0; u < R; ++u) {
        if (u < rounds) {
            const int32_t ix = wave_scan(x[u]), iy = wave_scan(y[u]);
            if (lane == 63) {
                sm.tot[0][u * kFinWaves + wave] = ix;
                sm.tot[1][u * kFinWaves + wave] = iy;
            }
            x[u] = ix - x[u];
            y[u] = iy - y[u];
        }
    }
    __syncthreads();
    // exclusive prefix of the wave totals in (round, wave) order, 64 at a time
    const int slots = rounds * kFinWaves;
    int32_t cx = 0, cy = 0;
    for (int c0 = 0; c0 < slots; c0 += 64) {
        const int j = c0 + lane;
        const int32_t vx = j < slots ? sm.tot[0][j] : 0, vy = j < slots ? sm.tot[1][j] : 0;
        const int32_t sx = wave_scan(vx) - vx + cx, sy = wave_scan(vy) - vy + cy;
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int idx = u * kFinWaves + wave;   // wave-uniform
            if (u < rounds && idx >= c0 && idx < c0 + 64) {
                x[u] += __builtin_amdgcn_readlane(sx, idx - c0);
                y[u] += __builtin_amdgcn_readlane(sy, idx - c0);
            }
        }
        cx = __builtin_amdgcn_readlane(sx + vx, 63);
        cy = __builtin_amdgcn_readlane(sy + vy, 63);
    }
    tx = cx;
    ty = cy;
    __syncthreads();   // tot is reused by the next scan
}

// Sort the keys of a power-of-two range [0, P) of the tile ascending with a
// bitonic network (each merge of two sorted halves starts with the step that
// compares mirrored positions, so every comparator puts the smaller key at
// the lower index).
template <int C>
__device__ __forceinline__ void bitonic_sort(TileLds<C>& tl, int P) {
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int lj = __ffs(j) - 1;
            for (int q = threadIdx.x; q < (P >> 1); q += kFinThreads) {
                int lo, hi;
                if (j == (k >> 1)) {
                    const int base = (q >> lj) * k, off = q & (j - 1);
                    lo = base + off;
                    hi = base + k - 1 - off;
                } else {
                    lo = ((q >> lj) << (lj + 1)) + (q & (j - 1));
                    hi = lo + j;
                }
                const uint64_t kl = tl.key[lo], kh = tl.key[hi];
                if (kh < kl) {
                    const int32_t vl = tl.val[lo];
                    tl.key[lo] = kh;
                    tl.key[hi] = kl;
                    tl.val[lo] = tl.val[hi];
                    tl.val[hi] = vl;
                }
            }
            __syncthreads();
        }
    }
}

// Where a tile's points come from: a list (entry decoded, canonical FP64
// projection turned into its key, value times sign) ...
template <int N>
struct ListSource {
    const ListEntry* pts;
    const ImageDesc* dsc;
    int32_t sign;
    Dir<N> xi;
    __device__ __forceinline__ void get(int64_t j, uint64_t& k, int32_t& v) const {
        const PointT<N> pt = decode_entry<N>(pts[j], *dsc);
        k = order_key(project<N>(xi.v, pt.x));
        v = sign * (int32_t)pt.val;
    }
};

// ... or keys and values already in the workspace.
struct KeySource {
    const uint64_t* ka;
    const int32_t* va;
    __device__ __forceinline__ void get(int64_t j, uint64_t& k, int32_t& v) const {
        k = ka[j];
        v = va[j];
    }
};

// Bucket of a key among nb buckets over [lo, lo + nb / scale): floor((p -
// lo) * scale) clamped to [0, nb - 1], p the key's projection.  Subtraction,
// multiplication by a non-negative factor, the clamps and the truncation are
// monotone, so p <= q gives bucket(p) <= bucket(q) whatever lo and scale are
// (-0 comes back from its key as +0, which changes no bucket).
__device__ __forceinline__ int32_t bucket_of(uint64_t k, double lo, double scale, int nb) {
    const double x = (key_value(k) - lo) * scale;
    return x > 0.0 ? (x < (double)(nb - 1) ? (int32_t)x : nb - 1) : 0;
}

__device__ __forceinline__ double bucket_scale(double lo, double hi, int nb) {
    const double s = hi > lo ? (double)nb / (hi - lo) : 0.0;
    return isfinite(s) ? s : 0.0;
}

// Stage points [first, first + m) (1 <= m <= C) of a source and sort them:
// on return tl.key[0, m) holds their keys in ascending order (equal keys in
// some order) and tl.val the matching values.  [lo, hi]: a range that holds
// the projections up to rounding (it only balances the buckets).
template <int C, class Src>
__device__ __forceinline__ void sort_tile(const Src& src, int64_t first, int m, double lo, double hi, TileLds<C>& tl,
                                          RowSmall& sm) {
    constexpr int I = C / kFinThreads;
    const int t = threadIdx.x;
    // nb buckets (a power of two, at least one per thread, held striped)
    int nb = kFinThreads;
    while (nb < m) nb <<= 1;
    const int rounds_b = nb / kFinThreads;
    for (int c = 0; c < rounds_b; ++c) tl.start[c * kFinThreads + t] = 0;
    if (t == 0) tl.start[nb] = m;
    uint64_t k[I];
    int32_t v[I];
#pragma unroll
    for (int u = 0; u < I; ++u) {
        const int j = u * kFinThreads + t;
        k[u] = ~0ull;
        v[u] = 0;
        if (j < m) src.get(first + j, k[u], v[u]);
    }
    const double scale = bucket_scale(lo, hi, nb);
    __syncthreads();   // bins cleared
    int32_t bs[I];     // bucket | slot in the bucket << 16
#pragma unroll
    for (int u = 0; u < I; ++u) {
        bs[u] = -1;
        if (u * kFinThreads + t < m) {
            const int32_t b = bucket_of(k[u], lo, scale, nb);
            bs[u] = b | (atomicAdd(&tl.start[b], 1) << 16);
        }
    }
    __syncthreads();
    int32_t cnt[I], big[I];
#pragma unroll
    for (int c = 0; c < I; ++c) {
        cnt[c] = c < rounds_b ? tl.start[c * kFinThreads + t] : 0;
        big[c] = cnt[c] > kBucketMax ? 1 : 0;
    }
    int32_t total, nbig;
    striped_scan2<I>(cnt, big, rounds_b, total, nbig, sm);
    if (nbig > 0) {
        // clustered projections: the bitonic network on the padded tile
        int P = 1;
        while (P < m) P <<= 1;
#pragma unroll
        for (int u = 0; u < I; ++u) {
            const int j = u * kFinThreads + t;
            if (j < P) {
                tl.key[j] = k[u];   // ~0 (above every finite key) past m
                tl.val[j] = v[u];
            }
        }
        __syncthreads();
        bitonic_sort<C>(tl, P);
        return;
    }
#pragma unroll
    for (int c = 0; c < I; ++c)
        if (c < rounds_b) tl.start[c * kFinThreads + t] = cnt[c];
    __syncthreads();
    // pos: the slot in bucket order, then the place in key order
    int32_t pos[I];
#pragma unroll
    for (int u = 0; u < I; ++u) {
        pos[u] = -1;
        if (bs[u] >= 0) {
            pos[u] = tl.start[bs[u] & 0xFFFF] + (bs[u] >> 16);
            tl.key[pos[u]] = k[u];
        }
    }
    __syncthreads();
    // place inside the bucket: members with a smaller key, or an equal key
    // in an earlier slot.  Each step reads one member of every bucket of the
    // thread (the last one again once a bucket is exhausted, so the loads
    // carry no branch and go out together).
    int32_t span[I], r[I];   // first member | members << 16 (0 when alone)
    int32_t longest = 0;
#pragma unroll
    for (int u = 0; u < I; ++u) {
        span[u] = 0;
        r[u] = 0;
        if (bs[u] >= 0) {
            const int b = bs[u] & 0xFFFF;
            const int q0 = tl.start[b], q1 = tl.start[b + 1];
            span[u] = q0 | (q1 - q0 > 1 ? (q1 - q0) << 16 : 0);
            longest = max(longest, (q1 - q0 > 1 ? q1 - q0 : 0));
        }
    }
    for (int o = 0; o < longest; ++o) {
        uint64_t kq[I];
#pragma unroll
        for (int u = 0; u < I; ++u) {
            const int len = span[u] >> 16;
            kq[u] = tl.key[(span[u] & 0xFFFF) + (o < len ? o : (len > 0 ? len - 1 : 0))];
        }
#pragma unroll
        for (int u = 0; u < I; ++u) {
            const int q = (span[u] & 0xFFFF) + o;
            r[u] += (o < (span[u] >> 16) && (kq[u] < k[u] || (kq[u] == k[u] && q < pos[u]))) ? 1 : 0;
        }
    }
#pragma unroll
    for (int u = 0; u < I; ++u)
        if (bs[u] >= 0) pos[u] = (span[u] & 0xFFFF) + r[u];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < I; ++u) {
        if (pos[u] >= 0) {
            tl.key[pos[u]] = k[u];
            tl.val[pos[u]] = v[u];
        }
    }
    __syncthreads();
}

// Distinct entries of the sorted tile tl[0, m): out_T[j], out_E[j] for the
// j-th distinct key, with carry plus the running sum of the values up to its
// last occurrence; carry grows by the tile's sum.  Elements are taken
// striped (consecutive across lanes), so a wave's stores land on consecutive
// entries.
template <int C>
__device__ __forceinline__ int64_t merge_tile(TileLds<C>& tl, int m, double* out_T, int32_t* out_E, int32_t& carry,
                                              RowSmall& sm) {
    constexpr int I = C / kFinThreads;
    const int t = threadIdx.x;
    const int rounds = (m + kFinThreads - 1) / kFinThreads;
    uint64_t k[I];
    int32_t h[I], c[I], v[I];
    uint32_t tails = 0;
#pragma unroll
    for (int u = 0; u < I; ++u) {
        const int i = u * kFinThreads + t;
        k[u] = 0;
        h[u] = 0;
        v[u] = 0;
        if (i < m) {
            k[u] = tl.key[i];
            v[u] = tl.val[i];
            h[u] = (i == 0 || tl.key[i - 1] != k[u]) ? 1 : 0;
            if (i + 1 == m || tl.key[i + 1] != k[u]) tails |= 1u << u;
        }
        c[u] = v[u];
    }
    uint32_t heads = 0;
#pragma unroll
    for (int u = 0; u < I; ++u) heads |= (uint32_t)h[u] << u;
    int32_t th, tc;
    striped_scan2<I>(h, c, rounds, th, tc, sm);
#pragma unroll
    for (int u = 0; u < I; ++u) {
        if (tails & (1u << u)) {
            const int32_t j = h[u] + (int32_t)((heads >> u) & 1u) - 1;
            out_T[j] = key_value(k[u]);
            out_E[j] = carry + c[u] + v[u];
        }
    }
    carry += tc;
    return th;
}

// Merge sorted runs A [0, la) and B [0, lb) into D (ties: A first); every
// thread of the workgroup takes kMergeItems consecutive outputs per step,
// found by a merge-path search.
__device__ __forceinline__ void merge_runs(const uint64_t* __restrict__ ka, const int32_t* __restrict__ va, int64_t la,
                                           const uint64_t* __restrict__ kb, const int32_t* __restrict__ vb, int64_t lb,
                                           uint64_t* __restrict__ kd, int32_t* __restrict__ vd) {
    const int64_t L = la + lb;
    for (int64_t d0 = 0; d0 < L; d0 += (int64_t)kFinThreads * kMergeItems) {
        const int64_t d = d0 + (int64_t)threadIdx.x * kMergeItems;
        if (d >= L) continue;
        int64_t lo = d > lb ? d - lb : 0, hi = d < la ? d : la;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (ka[mid] <= kb[d - 1 - mid]) lo = mid + 1; else hi = mid;
        }
        int64_t i = lo, j = d - lo;
        const int64_t end = d + kMergeItems < L ? d + kMergeItems : L;
        for (int64_t o = d; o < end; ++o) {
            if (j >= lb || (i < la && ka[i] <= kb[j])) {
                kd[o] = ka[i];
                vd[o] = va[i];
                ++i;
            } else {
                kd[o] = kb[j];
                vd[o] = vb[j];
                ++j;
            }
        }
    }
}

// Distinct entries of one list (n points at pts, values times sign).  A list
// of at most C points is sorted and merged in LDS.  A longer one is first
// distributed over C coarse buckets: a histogram pass, a scan, and a pass
// that places every key and value at its bucket's slots in workspace A (ka,
// va).  With no coarse bucket above C/2 points, the first bucket reaching
// each multiple of C/2 points starts a run of whole buckets of fewer than C
// points (equal keys share a bucket, so no run splits them); the runs are
// sorted and merged in LDS one after the other.  Otherwise (projections
// crowded below the range's resolution, or more than kMaxRuns runs) the
// general path runs: sorted tiles into A, pairwise merges between A and B,
// then the merge of equal keys from memory.
template <int N, int C>
__device__ __forceinline__ int64_t build_segment(const ListEntry* pts, const ImageDesc* dsc, int64_t n, int32_t sign,
                                                 Dir<N> xi, uint64_t* ka, int32_t* va, uint64_t* kb, int32_t* vb,
                                                 double* out_T, int32_t* out_E, TileLds<C>& tl, RowSmall& sm) {
    constexpr int I = C / kFinThreads;
    constexpr int H = C / 2;
    const int t = threadIdx.x;
    if (n <= 0) return 0;
    const ListSource<N> src{pts, dsc, sign, xi};
    // projections of the image's vertex box
    double lo = 0.0, hi = 0.0;
#pragma unroll
    for (int a = 0; a < N; ++a) {
        const double e0 = xi.v[a] * dsc->lo[a], e1 = xi.v[a] * dsc->hi[a];
        lo += fmin(e0, e1);
        hi += fmax(e0, e1);
    }
    int32_t carry = 0;
    if (n <= C) {
        sort_tile<C>(src, 0, (int)n, lo, hi, tl, sm);
        return merge_tile<C>(tl, (int)n, out_T, out_E, carry, sm);
    }
    if (n / H < kMaxRuns) {
        // coarse buckets: counts in tl.start, then cursors in tl.val
        const double scale = bucket_scale(lo, hi, C);
#pragma unroll
        for (int c = 0; c < I; ++c) tl.start[c * kFinThreads + t] = 0;
        if (t == 0) tl.start[C] = (int32_t)n;
        __syncthreads();
        for (int64_t j0 = 0; j0 < n; j0 += C) {   // I loads in flight per thread
            uint64_t k[I];
            int32_t v[I];
#pragma unroll
            for (int u = 0; u < I; ++u)
                if (j0 + u * kFinThreads + t < n) src.get(j0 + u * kFinThreads + t, k[u], v[u]);
#pragma unroll
            for (int u = 0; u < I; ++u)
                if (j0 + u * kFinThreads + t < n) atomicAdd(&tl.start[bucket_of(k[u], lo, scale, C)], 1);
        }
        __syncthreads();
        int32_t cnt[I], big[I];
#pragma unroll
        for (int c = 0; c < I; ++c) {
            cnt[c] = tl.start[c * kFinThreads + t];
            big[c] = cnt[c] > H ? 1 : 0;
        }
        int32_t total, nbig;
        striped_scan2<I>(cnt, big, I, total, nbig, sm);
        if (nbig == 0) {
#pragma unroll
            for (int c = 0; c < I; ++c) {
                tl.start[c * kFinThreads + t] = cnt[c];
                tl.val[c * kFinThreads + t] = cnt[c];
            }
            if (t == 0) {
                sm.run_b[0] = 0;
                sm.run_s[0] = 0;
            }
            __syncthreads();
            // run starts: bucket b begins run k = floor(start[b] / H) when it
            // is the first to reach k * H points (steps of at most H points
            // cross each multiple once)
            for (int b = t + 1; b <= C; b += kFinThreads) {
                const int32_t sb = tl.start[b], sp = tl.start[b - 1];
                if (sb / H > sp / H) {
                    sm.run_b[sb / H] = b;
                    sm.run_s[sb / H] = sb;
                }
            }
            for (int64_t j0 = 0; j0 < n; j0 += C) {
                uint64_t k[I];
                int32_t v[I];
#pragma unroll
                for (int u = 0; u < I; ++u)
                    if (j0 + u * kFinThreads + t < n) src.get(j0 + u * kFinThreads + t, k[u], v[u]);
#pragma unroll
                for (int u = 0; u < I; ++u) {
                    if (j0 + u * kFinThreads + t < n) {
                        const int32_t q = atomicAdd(&tl.val[bucket_of(k[u], lo, scale, C)], 1);
                        ka[q] = k[u];
                        va[q] = v[u];
                    }
                }
            }
            __syncthreads();
            const int runs = (int)(n / H) + 1;
            int64_t d = 0;
            for (int w = 0; w < runs; ++w) {
                const int32_t b0 = sm.run_b[w], s0 = sm.run_s[w];
                const int32_t b1 = w + 1 < runs ? sm.run_b[w + 1] : C;
                const int32_t s1 = w + 1 < runs ? sm.run_s[w + 1] : (int32_t)n;
                const int m = s1 - s0;
                if (m > 0) {
                    sort_tile<C>(KeySource{ka, va}, s0, m, lo + (double)b0 / scale, lo + (double)b1 / scale, tl, sm);
                    d += merge_tile<C>(tl, m, out_T + d, out_E + d, carry, sm);
                }
            }
            return d;
        }
    }
    // crowded buckets: sorted tiles and pairwise merges
    for (int64_t c0 = 0; c0 < n; c0 += C) {
        const int m = (int)(n - c0 < C ? n - c0 : C);
        sort_tile<C>(src, c0, m, lo, hi, tl, sm);
        for (int j = t; j < m; j += kFinThreads) {
            ka[c0 + j] = tl.key[j];
            va[c0 + j] = tl.val[j];
        }
        __syncthreads();
    }
    for (int64_t width = C; width < n; width *= 2) {
        for (int64_t lo2 = 0; lo2 < n; lo2 += 2 * width) {
            const int64_t la = n - lo2 < width ? n - lo2 : width;
            const int64_t rest = n - lo2 - la;
            const int64_t lb = rest < width ? rest : width;
            merge_runs(ka + lo2, va + lo2, la, ka + lo2 + la, va + lo2 + la, lb, kb + lo2, vb + lo2);
        }
        __syncthreads();
        uint64_t* tk = ka; ka = kb; kb = tk;
        int32_t* tv = va; va = vb; vb = tv;
    }
    return merge_segment(ka, va, 0, n, out_T, out_E, sm.wave);
}

// Row record of row r (every thread reads the same words), with the check of
// the caller's offsets: a row that needs more room than its offsets give, or
// reaches past the capacity, is marked -1.
template <int N>
__device__ __forceinline__ ExactRow load_row(const ExactArgs& a, int64_t r, bool report) {
    ExactRow ri;
    const int64_t need = row_info<N>(a, r, ri);
    const int64_t b = a.row_off[r], e = a.row_off[r + 1];
    ri.base = b;
    if (!(b >= 0 && e <= a.capacity && e - b >= need)) {
        ri.valid = -1;
        if (report && threadIdx.x == 0) raise_error(a.err, ECT_DEVERR_LAYOUT);
    } else if (!ri.valid && report && threadIdx.x == 0) {
        raise_error(a.err, ECT_DEVERR_NONFINITE);
    }
    return ri;
}

// Workgroup (r, part): part 0 builds the ECT row from the classical list, or
// the (T, E') part of a Radon row from the ordinary list (values -D); part 1
// (Radon only) builds the distinct classical projections and their running
// sums into the workspace (ct, cum at the row's classical slots), which
// exact_radon_kernel moves behind (T, E') as Ec = E'[last T < Tc] + own
// values.  A row marked -1 gets length 0 and raises ECT_DEVERR_LAYOUT.
// C: points per LDS tile (12 B each plus a bucket word).
template <int N, int C>
__global__ void __launch_bounds__(kFinThreads, C >= 8192 ? 2 : 4) exact_kernel(ExactArgs a) {
    __shared__ TileLds<C> tl;
    __shared__ RowSmall sm;
    const bool radon = a.kind == ECT_EXACT_RADON;
    const int64_t r = radon ? blockIdx.x >> 1 : blockIdx.x;
    const int part = radon ? (int)(blockIdx.x & 1) : 0;
    const ExactRow ri = load_row<N>(a, r, part == 0);
    if (ri.valid < 0) {
        if (threadIdx.x == 0 && part == 0) {
            if (radon) {
                a.len[2 * r] = 0;
                a.len[2 * r + 1] = 0;
            } else {
                a.len[r] = 0;
            }
        }
        return;
    }
    const int64_t base = ri.base;
    Dir<N> xi;
#pragma unroll
    for (int c = 0; c < N; ++c) xi.v[c] = ri.xi[c];
    const ImageDesc* dsc = a.desc + ri.img;
    // the row's one list: part 0 writes T, E (the first entry -inf, 0) and
    // the row length; Radon's part 1 writes the classical part into ct, cum
    int64_t first, n, w0;
    int32_t sign;
    double* oT;
    int32_t* oE;
    if (part == 0) {
        if (threadIdx.x == 0) {
            a.T[base] = -HUGE_VAL;
            a.E[base] = 0;
        }
        first = radon ? ri.po : ri.pc;
        n = radon ? ri.no : ri.nc;
        sign = radon ? ri.sign_o : 1;
        w0 = base;
        oT = a.T + base + 1;
        oE = a.E + base + 1;
    } else {
        first = ri.pc;
        n = ri.nc;
        sign = 1;
        w0 = base + ri.no + 1;
        oT = a.ct + w0;
        oE = a.cum + w0;
    }
    int64_t d = 0;
    if (ri.valid == 1)
        d = build_segment<N, C>((const ListEntry*)a.points + first, dsc, n, sign, xi, a.keys_a + w0, a.vals_a + w0,
                                a.keys_b + w0, a.vals_b + w0, oT, oE, tl, sm);
    if (threadIdx.x == 0) {
        if (part == 0) a.len[radon ? 2 * r : r] = d + 1;
        else a.len[2 * r + 1] = d;
    }
}

// Radon rows: the distinct classical projections move right behind (T, E')
// with Ec[k] = E'[largest i with T[i] < Tc[k]] + the classical values at
// Tc[k] (difference of consecutive running sums).  The search runs on every
// st-th entry of T staged in LDS, then inside one stride of T.
template <int N>
__global__ void __launch_bounds__(kFixThreads) exact_radon_kernel(ExactArgs a) {
    __shared__ double s_t[kFixSamples];
    const int64_t r = blockIdx.x;
    ExactRow ri;
    const int64_t need = row_info<N>(a, r, ri);
    const int64_t b = a.row_off[r], e = a.row_off[r + 1];
    if (!(b >= 0 && e <= a.capacity && e - b >= need) || ri.valid != 1) return;
    const int64_t base = b;
    const int64_t lo_n = a.len[2 * r], nc = a.len[2 * r + 1];
    const int64_t w0 = base + ri.no + 1;
    const double* T = a.T + base;
    const int32_t* Ep = a.E + base;
    const int64_t cb = base + lo_n;
    int64_t st = 1;
    while (st * kFixSamples < lo_n) st <<= 1;
    const int ns = (int)((lo_n + st - 1) / st);
    for (int i = threadIdx.x; i < ns; i += kFixThreads) s_t[i] = T[(int64_t)i * st];
    __syncthreads();
    for (int64_t k = threadIdx.x; k < nc; k += kFixThreads) {
        const double tc = a.ct[w0 + k];
        const int32_t own = a.cum[w0 + k] - (k > 0 ? a.cum[w0 + k - 1] : 0);
        int lo = 0, hi = ns - 1;   // last sample below tc (T[0] = -inf)
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_t[mid] < tc) lo = mid; else hi = mid - 1;
        }
        int64_t glo = (int64_t)lo * st, ghi = glo + st < lo_n ? glo + st - 1 : lo_n - 1;
        while (glo < ghi) {        // last index with T[i] < tc inside the stride
            const int64_t mid = (glo + ghi + 1) >> 1;
            if (T[mid] < tc) glo = mid; else ghi = mid - 1;
        }
        a.T[cb + k] = tc;
        a.E[cb + k] = Ep[glo] + own;
    }
}

// out[r][j] from the representation of row r by binary search.
__global__ void __launch_bounds__(kEvalThreads) exact_eval_kernel(int32_t kind, int64_t rows, const int64_t* row_off,
                                                                  const double* T, const int32_t* E, const int64_t* len,
                                                                  int64_t capacity, const double* thr, int32_t M,
                                                                  int32_t per_row, int32_t* out, int64_t col_blocks) {
    const int64_t r = blockIdx.x / col_blocks;
    const int64_t j = (blockIdx.x % col_blocks) * kEvalThreads + threadIdx.x;
    if (r >= rows || j >= M) return;
    const double t = thr[per_row ? r * M + j : j];
    const int64_t base = row_off[r];
    int32_t res = 0;
    if (kind == ECT_EXACT_ECT) {
        const int64_t n = len[r];
        if (base >= 0 && n >= 1 && base + n <= capacity && T[base] <= t) {
            int64_t lo = 0, hi = n - 1;   // last i with T[i] <= t
            while (lo < hi) {
                const int64_t mid = (lo + hi + 1) >> 1;
                if (T[base + mid] <= t) lo = mid; else hi = mid - 1;
            }
            res = E[base + lo];
        }
    } else {
        const int64_t no = len[2 * r], nc = len[2 * r + 1];
        if (base >= 0 && no >= 1 && nc >= 0 && base + no + nc <= capacity && T[base] < t) {
            const int64_t cb = base + no;
            int64_t lo = 0, hi = nc;      // first k with Tc[k] >= t
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (T[cb + mid] < t) lo = mid + 1; else hi = mid;
            }
            if (lo < nc && T[cb + lo] == t) {
                res = E[cb + lo];
            } else {
                int64_t a0 = 0, a1 = no - 1;   // last i with T[i] < t
                while (a0 < a1) {
                    const int64_t mid = (a0 + a1 + 1) >> 1;
                    if (T[base + mid] < t) a0 = mid; else a1 = mid - 1;
                }
                res = E[base + a0];
            }
        }
    }
    out[r * M + j] = res;
}

// The size query and the launch go through this call, so that both
// instantiate the same rocPRIM template.
hipError_t scan_call(void* tmp, size_t& bytes, const int64_t* in, int64_t* out, int64_t rows, hipStream_t stream) {
    return rocprim::exclusive_scan(tmp, bytes, in, out, (int64_t)0, (size_t)(rows + 1), rocprim::plus<int64_t>(),
                                   stream);
}

template <int N>
hipError_t launch_need(const ExactArgs& a, int64_t* need, hipStream_t stream) {
    const int64_t blocks = (a.rows + 1 + kRowThreads - 1) / kRowThreads;
    hipLaunchKernelGGL((exact_need_kernel<N>), dim3((unsigned)blocks), dim3(kRowThreads), 0, stream, a, need);
    return hipGetLastError();
}

template <int N>
void launch_rows(const ExactArgs& a, int64_t max_len, unsigned grid, hipStream_t stream) {
    if (max_len <= 2048)
        hipLaunchKernelGGL((exact_kernel<N, 2048>), dim3(grid), dim3(kFinThreads), 0, stream, a);
    else if (max_len <= 4096)
        hipLaunchKernelGGL((exact_kernel<N, 4096>), dim3(grid), dim3(kFinThreads), 0, stream, a);
    else if (max_len <= 8192)
        hipLaunchKernelGGL((exact_kernel<N, 8192>), dim3(grid), dim3(kFinThreads), 0, stream, a);
    else   // runs of coarse buckets: two 4096-point workgroups per compute unit beat one of 8192
        hipLaunchKernelGGL((exact_kernel<N, 4096>), dim3(grid), dim3(kFinThreads), 0, stream, a);
}

}  // namespace

size_t exact_layout_scan_bytes(int64_t rows) {
    size_t bytes = 0;
    return scan_call(nullptr, bytes, nullptr, nullptr, rows, (hipStream_t)0) == hipSuccess ? bytes : 0;
}

hipError_t launch_exact_layout(int ndim, const ExactArgs& a, int64_t* need, void* scan_tmp, size_t scan_bytes,
                               hipStream_t stream) {
    hipError_t e = ndim == 2   ? launch_need<2>(a, need, stream)
                   : ndim == 3 ? launch_need<3>(a, need, stream)
                               : launch_need<4>(a, need, stream);
    if (e != hipSuccess) return e;
    size_t bytes = scan_bytes;
    return scan_call(scan_tmp, bytes, need, a.row_off_out, a.rows, stream);
}

hipError_t launch_exact(int ndim, const ExactArgs& a, int64_t max_len, hipStream_t stream) {
    if (a.rows == 0) return hipSuccess;
    const bool radon = a.kind == ECT_EXACT_RADON;
    const unsigned grid = (unsigned)(radon ? 2 * a.rows : a.rows);
    if (ndim == 2) launch_rows<2>(a, max_len, grid, stream);
    else if (ndim == 3) launch_rows<3>(a, max_len, grid, stream);
    else launch_rows<4>(a, max_len, grid, stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !radon) return e;
    if (ndim == 2)
        hipLaunchKernelGGL((exact_radon_kernel<2>), dim3((unsigned)a.rows), dim3(kFixThreads), 0, stream, a);
    else if (ndim == 3)
        hipLaunchKernelGGL((exact_radon_kernel<3>), dim3((unsigned)a.rows), dim3(kFixThreads), 0, stream, a);
    else
        hipLaunchKernelGGL((exact_radon_kernel<4>), dim3((unsigned)a.rows), dim3(kFixThreads), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_exact_eval(int32_t kind, int64_t rows, const int64_t* row_off, const double* T, const int32_t* E,
                             const int64_t* len, int64_t capacity, const double* thr, int32_t M, int32_t per_row,
                             int32_t* out, hipStream_t stream) {
    if (rows == 0) return hipSuccess;
    const int64_t cb = (M + kEvalThreads - 1) / kEvalThreads;
    hipLaunchKernelGGL(exact_eval_kernel, dim3((unsigned)(rows * cb)), dim3(kEvalThreads), 0, stream, kind, rows,
                       row_off, T, E, len, capacity, thr, M, per_row, out, cb);
    return hipGetLastError();
}

}  // namespace ect
