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
// Steps: rows (per query row: image, sign vector, list bounds, check of the
// caller's row offsets) -> project (one thread per slot: canonical FP64
// projection turned into an order-preserving 64-bit key) -> segmented radix
// sort of (key, value) per list segment -> finalize (one workgroup per row:
// merge equal keys with a block scan of head flags and values) -> for Radon,
// the classical values get E' from a binary search in the row's T.
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_segmented_radix_sort.hpp>

#include "exact_internal.h"

namespace ect {

namespace {

constexpr int kRowThreads = 256;
constexpr int kFinThreads = 256;
constexpr int kFinItems = 4;            // consecutive sorted entries per thread per step
constexpr int kFinStep = kFinThreads * kFinItems;
constexpr int kSlotThreads = 256;
constexpr int kEvalThreads = 256;
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
    const double* v = a.vecs + (a.offsets ? r : r % a.count) * N;
    int ok = 1;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
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

// Row records and sort segments; a row whose offsets do not leave room for
// its entries (or leave the output) is marked unusable and gets empty
// segments.
template <int N>
__global__ void __launch_bounds__(kRowThreads) exact_rows_kernel(ExactArgs a) {
    const int64_t r = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    if (r >= a.rows) return;
    ExactRow ri;
    const int64_t need = row_info<N>(a, r, ri);
    const int64_t b = a.row_off[r], e = a.row_off[r + 1];
    ri.base = b;
    if (!(b >= 0 && e <= a.capacity && e - b >= need)) {
        ri.valid = -1;
        raise_error(a.err, ECT_DEVERR_LAYOUT);
    } else if (!ri.valid) {
        raise_error(a.err, ECT_DEVERR_NONFINITE);
    }
    a.rowrec[r] = ri;
    const bool use = ri.valid == 1;
    const uint32_t ub = use ? (uint32_t)b : 0u;
    if (a.kind == ECT_EXACT_ECT) {
        a.seg_begin[r] = ub;
        a.seg_end[r] = use ? ub + (uint32_t)ri.nc : 0u;
    } else {
        a.seg_begin[2 * r] = ub;
        a.seg_end[2 * r] = use ? ub + (uint32_t)ri.no : 0u;
        const uint32_t cb = use ? ub + (uint32_t)ri.no + 1u : 0u;
        a.seg_begin[2 * r + 1] = cb;
        a.seg_end[2 * r + 1] = use ? cb + (uint32_t)ri.nc : 0u;
    }
}

// One thread per output slot: the row owning the slot (the last row whose
// offset is <= slot), then the list point the slot stands for.
template <int N>
__global__ void __launch_bounds__(kSlotThreads) exact_project_kernel(ExactArgs a) {
    const int64_t s = (int64_t)blockIdx.x * kSlotThreads + threadIdx.x;
    if (s >= a.capacity || a.rows == 0) return;
    int64_t lo = 0, hi = a.rows - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (a.row_off[mid] <= s) lo = mid; else hi = mid - 1;
    }
    const ExactRow& ri = a.rowrec[lo];
    if (ri.valid != 1) return;
    const int64_t k = s - ri.base;
    if (k < 0) return;
    int64_t p;
    int32_t sign = 1;
    if (a.kind == ECT_EXACT_ECT) {
        if (k >= ri.nc) return;
        p = ri.pc + k;
    } else if (k < ri.no) {
        p = ri.po + k;
        sign = ri.sign_o;
    } else if (k > ri.no && k - ri.no - 1 < ri.nc) {
        p = ri.pc + (k - ri.no - 1);
    } else {
        return;
    }
    const Point pt = a.points[p];
    double xi[N];
#pragma unroll
    for (int c = 0; c < N; ++c) xi[c] = ri.xi[c];
    a.keys_in[s] = order_key(project<N>(xi, pt.x));
    a.vals_in[s] = sign * (int32_t)pt.val;
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

// One workgroup per row.  ECT: T = [-inf, distinct classical projections],
// E = [0, running sums].  Radon: the same from the ordinary segment, then the
// distinct classical projections right after with their running classical
// sums in `cum` (turned into Ec by exact_radon_fix_kernel).
__global__ void __launch_bounds__(kFinThreads) exact_finalize_kernel(ExactArgs a) {
    __shared__ int32_t s_wave[kFinThreads / 64][2];
    const int64_t r = blockIdx.x;
    const ExactRow ri = a.rowrec[r];
    const bool radon = a.kind == ECT_EXACT_RADON;
    if (ri.valid < 0) {
        if (threadIdx.x == 0) {
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
    if (threadIdx.x == 0) {
        a.T[base] = -HUGE_VAL;
        a.E[base] = 0;
    }
    const int64_t n1 = radon ? ri.no : ri.nc;
    int64_t d1 = 0;
    if (ri.valid == 1) d1 = merge_segment(a.keys_out, a.vals_out, base, base + n1, a.T + base + 1, a.E + base + 1, s_wave);
    const int64_t len1 = d1 + 1;
    if (!radon) {
        if (threadIdx.x == 0) a.len[r] = len1;
        return;
    }
    int64_t d2 = 0;
    if (ri.valid == 1) {
        const int64_t cb = base + ri.no + 1;
        d2 = merge_segment(a.keys_out, a.vals_out, cb, cb + ri.nc, a.T + base + len1, a.cum + base + len1, s_wave);
    }
    if (threadIdx.x == 0) {
        a.len[2 * r] = len1;
        a.len[2 * r + 1] = d2;
    }
}

// Radon point values: Ec[k] = E'[largest i with T[i] < Tc[k]] + the classical
// values at Tc[k] (difference of consecutive running sums).
__global__ void __launch_bounds__(kFinThreads) exact_radon_fix_kernel(ExactArgs a) {
    const int64_t r = blockIdx.x;
    const ExactRow ri = a.rowrec[r];
    if (ri.valid != 1) return;
    const int64_t base = ri.base;
    const int64_t lo_n = a.len[2 * r], nc = a.len[2 * r + 1];
    const double* T = a.T + base;
    const int32_t* Ep = a.E + base;
    const int64_t cb = base + lo_n;
    for (int64_t k = threadIdx.x; k < nc; k += kFinThreads) {
        const double tc = a.T[cb + k];
        const int32_t own = a.cum[cb + k] - (k > 0 ? a.cum[cb + k - 1] : 0);
        // T[0] = -inf < tc: find the last index with T[i] < tc
        int64_t lo = 0, hi = lo_n - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (T[mid] < tc) lo = mid; else hi = mid - 1;
        }
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

// The size queries and the launches go through these two calls, so that both
// instantiate the same rocPRIM templates.
hipError_t scan_call(void* tmp, size_t& bytes, const int64_t* in, int64_t* out, int64_t rows, hipStream_t stream) {
    return rocprim::exclusive_scan(tmp, bytes, in, out, (int64_t)0, (size_t)(rows + 1), rocprim::plus<int64_t>(),
                                   stream);
}

hipError_t sort_call(void* tmp, size_t& bytes, const ExactArgs& a, int64_t capacity, int64_t segments,
                     hipStream_t stream) {
    return rocprim::segmented_radix_sort_pairs(tmp, bytes, (const uint64_t*)a.keys_in, a.keys_out,
                                               (const int32_t*)a.vals_in, a.vals_out, (unsigned)capacity,
                                               (unsigned)segments, (const uint32_t*)a.seg_begin,
                                               (const uint32_t*)a.seg_end, 0, 64, stream);
}

template <int N>
hipError_t launch_need(const ExactArgs& a, int64_t* need, hipStream_t stream) {
    const int64_t blocks = (a.rows + 1 + kRowThreads - 1) / kRowThreads;
    hipLaunchKernelGGL((exact_need_kernel<N>), dim3((unsigned)blocks), dim3(kRowThreads), 0, stream, a, need);
    return hipGetLastError();
}

template <int N>
hipError_t launch_exact_typed(const ExactArgs& a, void* sort_tmp, size_t sort_bytes, hipStream_t stream) {
    if (a.rows == 0) return hipSuccess;
    const int64_t rb = (a.rows + kRowThreads - 1) / kRowThreads;
    hipLaunchKernelGGL((exact_rows_kernel<N>), dim3((unsigned)rb), dim3(kRowThreads), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.capacity > 0) {
        const int64_t sb = (a.capacity + kSlotThreads - 1) / kSlotThreads;
        hipLaunchKernelGGL((exact_project_kernel<N>), dim3((unsigned)sb), dim3(kSlotThreads), 0, stream, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        size_t bytes = sort_bytes;
        e = sort_call(sort_tmp, bytes, a, a.capacity, exact_segments(a.kind, a.rows), stream);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(exact_finalize_kernel, dim3((unsigned)a.rows), dim3(kFinThreads), 0, stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (a.kind == ECT_EXACT_RADON) {
        hipLaunchKernelGGL(exact_radon_fix_kernel, dim3((unsigned)a.rows), dim3(kFinThreads), 0, stream, a);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace

size_t exact_layout_scan_bytes(int64_t rows) {
    size_t bytes = 0;
    return scan_call(nullptr, bytes, nullptr, nullptr, rows, (hipStream_t)0) == hipSuccess ? bytes : 0;
}

size_t exact_sort_bytes(int32_t kind, int64_t rows, int64_t capacity) {
    size_t bytes = 0;
    ExactArgs a{};
    return sort_call(nullptr, bytes, a, capacity, exact_segments(kind, rows), (hipStream_t)0) == hipSuccess ? bytes
                                                                                                           : 0;
}

hipError_t launch_exact_layout(int ndim, const ExactArgs& a, int64_t* need, void* scan_tmp, size_t scan_bytes,
                               hipStream_t stream) {
    hipError_t e = ndim == 2 ? launch_need<2>(a, need, stream) : launch_need<3>(a, need, stream);
    if (e != hipSuccess) return e;
    size_t bytes = scan_bytes;
    return scan_call(scan_tmp, bytes, need, a.row_off_out, a.rows, stream);
}

hipError_t launch_exact(int ndim, const ExactArgs& a, void* sort_tmp, size_t sort_bytes, hipStream_t stream) {
    return ndim == 2 ? launch_exact_typed<2>(a, sort_tmp, sort_bytes, stream)
                     : launch_exact_typed<3>(a, sort_tmp, sort_bytes, stream);
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
