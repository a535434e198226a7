// Query bucketing by sign vector and work-list construction (gfx950).
//
// All directions of one open orthant share their critical points and values
// (Lemma 3.2), so queries are grouped by sign vector before evaluation: a
// workgroup then holds several queries that read the same point list.  The
// sign of a zero coordinate is taken as +1.
//
// ECT mode: 2^n buckets, one per sign vector (classical lists).
// Hybrid mode: 2^(n-1) buckets, one per pair {eps, -eps}; a query whose
// eps_{n-1} = -1 is evaluated on the list of -eps with negated values, because
// Delta^ord(-eps, x) = -Delta^ord(eps, x).  The negation is carried as bit 0 of
// the permutation entry (entry = 2 * row + negated).
#include "eval_internal.h"

namespace ect {

namespace {

// One workgroup per image (ragged set) or a single workgroup (shared set).
// Stable: inside a bucket, queries keep their row order.
template <int N>
__global__ void __launch_bounds__(kBucketThreads)
bucket_kernel(const double* __restrict__ vecs, const int64_t* __restrict__ offsets, int64_t count,
              int mode_hybrid, uint32_t* __restrict__ err, int64_t* __restrict__ perm,
              int64_t* __restrict__ bstart, int32_t* __restrict__ bcnt) {
    const int B = mode_hybrid ? (1 << (N - 1)) : (1 << N);
    const int full = (1 << N) - 1;
    const int img = blockIdx.x;
    const int64_t r0 = offsets ? offsets[img] : 0;
    const int64_t r1 = offsets ? offsets[img + 1] : count;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int W = kBucketThreads / 64;

    __shared__ int32_t s_wc[W][8];
    __shared__ int64_t s_run[8];
    __shared__ int64_t s_start[8];

    auto key_of = [&](int64_t r, int* neg) -> int {
        double xi[N];
        bool fin = true;
#pragma unroll
        for (int a = 0; a < N; ++a) {
            xi[a] = vecs[r * N + a];
            fin = fin && isfinite(xi[a]);
        }
        if (!fin) raise_error(err, ECT_DEVERR_NONFINITE);
        int e = sign_index<N>(xi);
        *neg = 0;
        if (mode_hybrid && (e >> (N - 1)) & 1) { e ^= full; *neg = 1; }
        return e;
    };

    // pass 1: counts
    if (tid < 8) s_run[tid] = 0;
    __syncthreads();
    for (int64_t base = r0; base < r1; base += kBucketThreads) {
        int64_t r = base + tid;
        int key = -1, neg = 0;
        if (r < r1) key = key_of(r, &neg);
        for (int b = 0; b < B; ++b) {
            uint64_t m = __ballot(key == b);
            if (lane == 0) s_wc[wave][b] = __popcll(m);
        }
        __syncthreads();
        if (tid < B) {
            int64_t c = 0;
            for (int w = 0; w < W; ++w) c += s_wc[w][tid];
            s_run[tid] += c;
        }
        __syncthreads();
    }
    if (tid == 0) {
        int64_t acc = r0;
        for (int b = 0; b < B; ++b) {
            s_start[b] = acc;
            bstart[(int64_t)img * B + b] = acc;
            bcnt[(int64_t)img * B + b] = (int32_t)s_run[b];
            acc += s_run[b];
            s_run[b] = 0;
        }
    }
    __syncthreads();
    // pass 2: stable scatter
    for (int64_t base = r0; base < r1; base += kBucketThreads) {
        int64_t r = base + tid;
        int key = -1, neg = 0;
        if (r < r1) key = key_of(r, &neg);
        int rank = 0;
        for (int b = 0; b < B; ++b) {
            uint64_t m = __ballot(key == b);
            if (lane == 0) s_wc[wave][b] = __popcll(m);
            if (key == b) rank = __popcll(m & ((1ull << lane) - 1ull));
        }
        __syncthreads();
        if (key >= 0) {
            int64_t pos = s_start[key] + s_run[key] + rank;
            for (int w = 0; w < wave; ++w) pos += s_wc[w][key];
            perm[pos] = 2 * (r - r0) + neg;   // row relative to the image's first row
        }
        __syncthreads();
        if (tid < B) {
            int64_t c = 0;
            for (int w = 0; w < W; ++w) c += s_wc[w][tid];
            s_run[tid] += c;
        }
        __syncthreads();
    }
}

// Work list: items of entry (i, b) = ceil(bucket count / qtile) query tiles,
// each split into ceil(points / chunk) point chunks (chunk == 0: no split).
// Writes the item prefix over entries, the query-tile prefix (for the
// reduction counters) and the chunk size actually used.  If the item count
// exceeds `capacity`, the chunk size is doubled until it fits.
__global__ void __launch_bounds__(1024)
worklist_kernel(int num_images, int B, int list_base, int NL, int shared_queries,
                const int32_t* __restrict__ bcnt, const int64_t* __restrict__ list_off,
                int qtile, int64_t chunk0, int64_t capacity, uint32_t* __restrict__ err,
                int64_t* __restrict__ item_off, int64_t* __restrict__ tile_off,
                int64_t* __restrict__ params) {
    __shared__ int64_t s_part[1024];
    __shared__ int64_t s_tpart[1024];
    __shared__ int64_t s_total[2];
    const int tid = threadIdx.x;
    const int64_t E = (int64_t)num_images * B;
    int64_t chunk = chunk0;
    for (int attempt = 0; attempt < 40; ++attempt) {
        // per-thread contiguous range of entries
        const int64_t per = (E + 1023) / 1024;
        const int64_t e0 = tid * per, e1 = min(E, e0 + per);
        int64_t my = 0, myt = 0;
        for (int64_t e = e0; e < e1; ++e) {
            int64_t i = e / B, b = e % B;
            int64_t q = bcnt[shared_queries ? b : e];
            int64_t tiles = (q + qtile - 1) / qtile;
            int64_t np = list_off[(i + 1) * NL + list_base + b] - list_off[i * NL + list_base + b];
            int64_t ch = chunk > 0 ? (np + chunk - 1) / chunk : 1;
            if (ch < 1) ch = 1;  // an empty list still gets one item per tile, which writes zeros
            my += tiles * ch;
            myt += tiles;
        }
        s_part[tid] = my;
        s_tpart[tid] = myt;
        __syncthreads();
        if (tid == 0) {
            int64_t acc = 0, tacc = 0;
            for (int t = 0; t < 1024; ++t) {
                int64_t c = s_part[t], ct = s_tpart[t];
                s_part[t] = acc;
                s_tpart[t] = tacc;
                acc += c;
                tacc += ct;
            }
            s_total[0] = acc;
            s_total[1] = tacc;
        }
        __syncthreads();
        const int64_t total = s_total[0];
        if (capacity <= 0 || total <= capacity || chunk == 0) {
            int64_t run = s_part[tid], trun = s_tpart[tid];
            for (int64_t e = e0; e < e1; ++e) {
                int64_t i = e / B, b = e % B;
                int64_t q = bcnt[shared_queries ? b : e];
                int64_t tiles = (q + qtile - 1) / qtile;
                int64_t np = list_off[(i + 1) * NL + list_base + b] - list_off[i * NL + list_base + b];
                int64_t ch = chunk > 0 ? (np + chunk - 1) / chunk : 1;
                if (ch < 1) ch = 1;
                item_off[e] = run;
                tile_off[e] = trun;
                run += tiles * ch;
                trun += tiles;
            }
            if (tid == 0) {
                item_off[E] = total;
                tile_off[E] = s_total[1];
                params[0] = total;
                params[1] = s_total[1];
                params[2] = chunk;
            }
            return;
        }
        chunk *= 2;
        __syncthreads();
    }
    if (tid == 0) {
        raise_error(err, ECT_DEVERR_CAPACITY);
        params[0] = 0;
        params[1] = 0;
        params[2] = chunk;
        item_off[E] = 0;
        tile_off[E] = 0;
    }
}

}  // namespace

hipError_t launch_bucket(int ndim, const ect_query_set& qs, int num_images, bool hybrid, uint32_t* err,
                         int64_t* perm, int64_t* bstart, int32_t* bcnt, hipStream_t stream) {
    const int groups = qs.offsets ? num_images : 1;
    if (ndim == 2)
        hipLaunchKernelGGL(bucket_kernel<2>, dim3(groups), dim3(kBucketThreads), 0, stream, qs.vecs, qs.offsets,
                           qs.count, hybrid ? 1 : 0, err, perm, bstart, bcnt);
    else
        hipLaunchKernelGGL(bucket_kernel<3>, dim3(groups), dim3(kBucketThreads), 0, stream, qs.vecs, qs.offsets,
                           qs.count, hybrid ? 1 : 0, err, perm, bstart, bcnt);
    return hipGetLastError();
}

hipError_t launch_worklist(int num_images, int B, int list_base, int NL, bool shared_queries,
                           const int32_t* bcnt, const int64_t* list_off, int qtile, int64_t chunk,
                           int64_t capacity, uint32_t* err, int64_t* item_off, int64_t* tile_off,
                           int64_t* params, hipStream_t stream) {
    hipLaunchKernelGGL(worklist_kernel, dim3(1), dim3(1024), 0, stream, num_images, B, list_base, NL,
                       shared_queries ? 1 : 0, bcnt, list_off, qtile, chunk, capacity, err, item_off,
                       tile_off, params);
    return hipGetLastError();
}

}  // namespace ect
