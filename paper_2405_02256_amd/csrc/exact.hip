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
// 64-bit key, sorts (key, value) pairs with a block radix sort in LDS, merges
// equal keys with a block scan of head flags and values and writes the
// distinct entries.  A list longer than one LDS tile (4096 points) is sorted
// tile by tile into the workspace and the sorted tiles are merged pairwise
// there by the same workgroup (merge path), before the same merge of equal
// keys.  For Radon, each classical entry then takes E' from a binary search
// in the row's T.  Global memory written by the workgroup is read back by it
// only after a workgroup barrier.
#include <rocprim/block/block_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "exact_internal.h"

namespace ect {

namespace {

constexpr int kRowThreads = 256;
constexpr int kFinThreads = 512;         // the row-building workgroup
constexpr int kFinItems = 4;            // consecutive sorted entries per thread per step (long lists)
constexpr int kFinStep = kFinThreads * kFinItems;
constexpr int kTileItems = 8;           // keys per thread of the largest LDS sort
constexpr int kTile = kFinThreads * kTileItems;
constexpr int kMergeItems = 8;          // outputs per thread per step of a pairwise merge
constexpr int kEvalThreads = 256;
constexpr int kFixThreads = 256;
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

// Tiles are sorted on 32-bit keys carrying the point's staging index: first
// on the FP32 rounding of the projection (monotone, so the result is ordered
// up to projections that round to the same float); only when that leaves two
// neighbours out of FP64 order is the tile sorted exactly, by the low then
// (stably) the high half of the 64-bit key.  The keys and values themselves
// stay in LDS and are read through the sorted indices.
template <int I>
using BlockSort = rocprim::block_radix_sort<uint32_t, kFinThreads, I, uint32_t>;

union SortStorage {
    typename BlockSort<1>::storage_type s1;
    typename BlockSort<2>::storage_type s2;
    typename BlockSort<4>::storage_type s4;
    typename BlockSort<6>::storage_type s6;
    typename BlockSort<kTileItems>::storage_type s8;
};

struct RowShared {
    SortStorage sort;
    uint64_t key[kTile];           // staged keys and values of the tile, by load index
    int32_t val[kTile];
    uint64_t first[kFinThreads];   // first / last key of each thread after a sort
    uint64_t last[kFinThreads];
    int32_t wave[kFinThreads / 64][2];
    ExactRow ri;
};

template <int I>
__device__ __forceinline__ typename BlockSort<I>::storage_type& sort_storage(RowShared& sh) {
    if constexpr (I == 1) return sh.sort.s1;
    else if constexpr (I == 2) return sh.sort.s2;
    else if constexpr (I == 4) return sh.sort.s4;
    else if constexpr (I == 6) return sh.sort.s6;
    else return sh.sort.s8;
}

// Order-preserving key of an FP32 value (-0 taken as +0).
__device__ __forceinline__ uint32_t order_key32(float f) {
    const uint32_t b = (uint32_t)__float_as_int(f + 0.0f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Stage points [0, n) (n <= I * threads) of one list and sort them: thread t
// receives the staging indices of ranks t*I .. t*I+I-1 (ranks past n:
// padding).
template <int N, int I>
__device__ __forceinline__ void sort_tile(const ListEntry* __restrict__ pts, const ImageDesc* dsc, int64_t n, int32_t sign, Dir<N> xi,
                                          uint32_t (&idx)[I], RowShared& sh) {
    uint32_t key32[I];
#pragma unroll
    for (int u = 0; u < I; ++u) {
        const int j = u * kFinThreads + threadIdx.x;
        key32[u] = 0xFFFFFFFFu;
        idx[u] = (uint32_t)j;
        if (j < n) {
            const PointT<N> pt = decode_entry<N>(pts[j], *dsc);
            const double p = project<N>(xi.v, pt.x);
            sh.key[j] = order_key(p);
            sh.val[j] = sign * (int32_t)pt.val;
            key32[u] = order_key32((float)p);
        }
    }
    BlockSort<I>().sort(key32, idx, sort_storage<I>(sh));
    __syncthreads();
    const int t = threadIdx.x;
    const int64_t i0 = (int64_t)t * I;
    int bad = 0;
    uint64_t prev = 0;
#pragma unroll
    for (int u = 0; u < I; ++u) {
        const uint64_t k = i0 + u < n ? sh.key[idx[u]] : ~0ull;
        if (u == 0) sh.first[t] = k;
        else if (k < prev) bad = 1;
        prev = k;
    }
    __syncthreads();
    if (t + 1 < kFinThreads && sh.first[t + 1] < prev) bad = 1;
    if (__syncthreads_or(bad)) {
        // exact order: low halves, then high halves (the sort is stable)
#pragma unroll
        for (int u = 0; u < I; ++u) key32[u] = i0 + u < n ? (uint32_t)sh.key[idx[u]] : 0xFFFFFFFFu;
        BlockSort<I>().sort(key32, idx, sort_storage<I>(sh));
        __syncthreads();
#pragma unroll
        for (int u = 0; u < I; ++u) key32[u] = i0 + u < n ? (uint32_t)(sh.key[idx[u]] >> 32) : 0xFFFFFFFFu;
        BlockSort<I>().sort(key32, idx, sort_storage<I>(sh));
        __syncthreads();
    }
}

// Distinct entries of a sorted tile (staging indices in registers, blocked),
// as merge_segment does for a sorted list in memory.
template <int I>
__device__ __forceinline__ int64_t merge_tile(const uint32_t (&idx)[I], int64_t n, double* out_T, int32_t* out_E,
                                              RowShared& sh) {
    const int t = threadIdx.x;
    const int64_t i0 = (int64_t)t * I;
    sh.first[t] = i0 < n ? sh.key[idx[0]] : ~0ull;
    sh.last[t] = i0 + I - 1 < n ? sh.key[idx[I - 1]] : ~0ull;
    __syncthreads();
    const uint64_t before = t > 0 ? sh.last[t - 1] : 0;
    const uint64_t after = t + 1 < kFinThreads ? sh.first[t + 1] : 0;
    int32_t heads = 0, sum = 0;
    uint64_t prev = before;
#pragma unroll
    for (int u = 0; u < I; ++u) {
        if (i0 + u < n) {
            const uint64_t k = sh.key[idx[u]];
            heads += (i0 + u == 0 || k != prev) ? 1 : 0;
            sum += sh.val[idx[u]];
            prev = k;
        }
    }
    int32_t h_ex, s_ex, h_tot, s_tot;
    block_scan2(heads, sum, h_ex, s_ex, h_tot, s_tot, sh.wave);
    int32_t h = h_ex, c = s_ex;
    prev = before;
#pragma unroll
    for (int u = 0; u < I; ++u) {
        const int64_t i = i0 + u;
        if (i >= n) break;
        const uint64_t k = sh.key[idx[u]];
        h += (i == 0 || k != prev) ? 1 : 0;
        c += sh.val[idx[u]];
        const uint64_t nk = u + 1 < I ? (i + 1 < n ? sh.key[idx[u + 1]] : ~0ull) : after;
        if (i + 1 == n || nk != k) {
            out_T[h - 1] = key_value(k);
            out_E[h - 1] = c;
        }
        prev = k;
    }
    __syncthreads();   // staging and first/last are reused by the next tile
    return h_tot;
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

// Sort one tile of a long list and store it, in order, at ka/va.
template <int N, int I>
__device__ __noinline__ void store_tile(const ListEntry* pts, const ImageDesc* dsc, int64_t m, int32_t sign, Dir<N> xi,
                                        uint64_t* ka, int32_t* va, RowShared& sh) {
    uint32_t idx[I];
    sort_tile<N, I>(pts, dsc, m, sign, xi, idx, sh);
#pragma unroll
    for (int u = 0; u < I; ++u) {
        const int64_t i = (int64_t)threadIdx.x * I + u;
        if (i < m) {
            ka[i] = sh.key[idx[u]];
            va[i] = sh.val[idx[u]];
        }
    }
    __syncthreads();
}

// A list longer than one tile: sorted tiles into workspace A, pairwise merges
// between A and B, then the merge of equal keys from memory.
template <int N>
__device__ __noinline__ int64_t build_long(const ListEntry* pts, const ImageDesc* dsc, int64_t n, int32_t sign, Dir<N> xi, uint64_t* ka,
                                           int32_t* va, uint64_t* kb, int32_t* vb, double* out_T, int32_t* out_E,
                                           RowShared& sh) {
    for (int64_t c0 = 0; c0 < n; c0 += kTile) {
        const int64_t m = n - c0 < kTile ? n - c0 : kTile;
        if (m <= kFinThreads) store_tile<N, 1>(pts + c0, dsc, m, sign, xi, ka + c0, va + c0, sh);
        else if (m <= 4 * kFinThreads) store_tile<N, 4>(pts + c0, dsc, m, sign, xi, ka + c0, va + c0, sh);
        else store_tile<N, kTileItems>(pts + c0, dsc, m, sign, xi, ka + c0, va + c0, sh);
    }
    for (int64_t width = kTile; width < n; width *= 2) {
        for (int64_t lo = 0; lo < n; lo += 2 * width) {
            const int64_t la = n - lo < width ? n - lo : width;
            const int64_t rest = n - lo - la;
            const int64_t lb = rest < width ? rest : width;
            merge_runs(ka + lo, va + lo, la, ka + lo + la, va + lo + la, lb, kb + lo, vb + lo);
        }
        __syncthreads();
        uint64_t* tk = ka; ka = kb; kb = tk;
        int32_t* tv = va; va = vb; vb = tv;
    }
    return merge_segment(ka, va, 0, n, out_T, out_E, sh.wave);
}

// Distinct entries of one list (n points at pts), values times sign.
template <int N, int I>
__device__ __noinline__ int64_t build_tile(const ListEntry* pts, const ImageDesc* dsc, int64_t n, int32_t sign, Dir<N> xi,
                                           double* out_T, int32_t* out_E, RowShared& sh) {
    uint32_t idx[I];
    sort_tile<N, I>(pts, dsc, n, sign, xi, idx, sh);
    return merge_tile<I>(idx, n, out_T, out_E, sh);
}

template <int N>
__device__ int64_t build_segment(const ExactArgs& a, const ListEntry* pts, const ImageDesc* dsc, int64_t n, int32_t sign, Dir<N> xi,
                                 int64_t w0, double* out_T, int32_t* out_E, RowShared& sh) {
    if (n <= 0) return 0;
    if (n <= kFinThreads) return build_tile<N, 1>(pts, dsc, n, sign, xi, out_T, out_E, sh);
    if (n <= 2 * kFinThreads) return build_tile<N, 2>(pts, dsc, n, sign, xi, out_T, out_E, sh);
    if (n <= 4 * kFinThreads) return build_tile<N, 4>(pts, dsc, n, sign, xi, out_T, out_E, sh);
    if (n <= 6 * kFinThreads) return build_tile<N, 6>(pts, dsc, n, sign, xi, out_T, out_E, sh);
    if (n <= kTile) return build_tile<N, kTileItems>(pts, dsc, n, sign, xi, out_T, out_E, sh);
    return build_long<N>(pts, dsc, n, sign, xi, a.keys_a + w0, a.vals_a + w0, a.keys_b + w0, a.vals_b + w0, out_T, out_E,
                         sh);
}

// Row record of row r (thread 0 of the workgroup), with the check of the
// caller's offsets: a row that needs more room than its offsets give, or
// reaches past the capacity, is marked -1.
template <int N>
__device__ __forceinline__ void load_row(const ExactArgs& a, int64_t r, bool report, RowShared& sh) {
    if (threadIdx.x == 0) {
        ExactRow ri;
        const int64_t need = row_info<N>(a, r, ri);
        const int64_t b = a.row_off[r], e = a.row_off[r + 1];
        ri.base = b;
        if (!(b >= 0 && e <= a.capacity && e - b >= need)) {
            ri.valid = -1;
            if (report) raise_error(a.err, ECT_DEVERR_LAYOUT);
        } else if (!ri.valid && report) {
            raise_error(a.err, ECT_DEVERR_NONFINITE);
        }
        sh.ri = ri;
    }
    __syncthreads();
}

// Workgroup (r, part): part 0 builds the ECT row from the classical list, or
// the (T, E') part of a Radon row from the ordinary list (values -D); part 1
// (Radon only) builds the distinct classical projections and their running
// sums into the workspace (ct, cum at the row's classical slots), which
// exact_radon_kernel moves behind (T, E') as Ec = E'[last T < Tc] + own
// values.  A row marked -1 gets length 0 and raises ECT_DEVERR_LAYOUT.
// Four waves per SIMD (two workgroups per compute unit) measured faster than
// the register allocation without the bound, despite a few spilled registers.
template <int N>
__global__ void __launch_bounds__(kFinThreads, 4) exact_kernel(ExactArgs a) {
    __shared__ RowShared sh;
    const bool radon = a.kind == ECT_EXACT_RADON;
    const int64_t r = radon ? blockIdx.x >> 1 : blockIdx.x;
    const int part = radon ? (int)(blockIdx.x & 1) : 0;
    load_row<N>(a, r, part == 0, sh);
    const ExactRow ri = sh.ri;
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
    const ListEntry* pts = (const ListEntry*)a.points;
    const ImageDesc* dsc = a.desc + ri.img;
    if (part == 0) {
        if (threadIdx.x == 0) {
            a.T[base] = -HUGE_VAL;
            a.E[base] = 0;
        }
        int64_t d = 0;
        if (ri.valid == 1) {
            if (radon) d = build_segment<N>(a, pts + ri.po, dsc, ri.no, ri.sign_o, xi, base, a.T + base + 1,
                                            a.E + base + 1, sh);
            else d = build_segment<N>(a, pts + ri.pc, dsc, ri.nc, 1, xi, base, a.T + base + 1, a.E + base + 1, sh);
        }
        if (threadIdx.x == 0) a.len[radon ? 2 * r : r] = d + 1;
    } else {
        const int64_t w0 = base + ri.no + 1;
        int64_t d = 0;
        if (ri.valid == 1) d = build_segment<N>(a, pts + ri.pc, dsc, ri.nc, 1, xi, w0, a.ct + w0, a.cum + w0, sh);
        if (threadIdx.x == 0) a.len[2 * r + 1] = d;
    }
}

// Radon rows: the distinct classical projections move right behind (T, E')
// with Ec[k] = E'[largest i with T[i] < Tc[k]] + the classical values at
// Tc[k] (difference of consecutive running sums).
template <int N>
__global__ void __launch_bounds__(kFixThreads) exact_radon_kernel(ExactArgs a) {
    __shared__ ExactRow s_ri;
    const int64_t r = blockIdx.x;
    if (threadIdx.x == 0) {
        ExactRow ri;
        const int64_t need = row_info<N>(a, r, ri);
        const int64_t b = a.row_off[r], e = a.row_off[r + 1];
        ri.base = b;
        if (!(b >= 0 && e <= a.capacity && e - b >= need)) ri.valid = -1;
        s_ri = ri;
    }
    __syncthreads();
    const ExactRow ri = s_ri;
    if (ri.valid != 1) return;
    const int64_t base = ri.base;
    const int64_t lo_n = a.len[2 * r], nc = a.len[2 * r + 1];
    const int64_t w0 = base + ri.no + 1;
    const double* T = a.T + base;
    const int32_t* Ep = a.E + base;
    const int64_t cb = base + lo_n;
    for (int64_t k = threadIdx.x; k < nc; k += kFixThreads) {
        const double tc = a.ct[w0 + k];
        const int32_t own = a.cum[w0 + k] - (k > 0 ? a.cum[w0 + k - 1] : 0);
        int64_t lo = 0, hi = lo_n - 1;   // last index with T[i] < tc (T[0] = -inf)
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (T[mid] < tc) lo = mid; else hi = mid - 1;
        }
        a.T[cb + k] = tc;
        a.E[cb + k] = Ep[lo] + own;
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

hipError_t launch_exact(int ndim, const ExactArgs& a, hipStream_t stream) {
    if (a.rows == 0) return hipSuccess;
    const bool radon = a.kind == ECT_EXACT_RADON;
    const unsigned grid = (unsigned)(radon ? 2 * a.rows : a.rows);
    if (ndim == 2)
        hipLaunchKernelGGL((exact_kernel<2>), dim3(grid), dim3(kFinThreads), 0, stream, a);
    else if (ndim == 3)
        hipLaunchKernelGGL((exact_kernel<3>), dim3(grid), dim3(kFinThreads), 0, stream, a);
    else
        hipLaunchKernelGGL((exact_kernel<4>), dim3(grid), dim3(kFinThreads), 0, stream, a);
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
