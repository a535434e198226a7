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
// the record code (code = 2 * row + negated).
//
// Bucket b of image i owns the record slots [B*r0_i + b*Q_i, B*r0_i + (b+1)*Q_i)
// (r0_i = first query row of the image, Q_i = its number of queries).  Shared
// hybrid sets of up to 65536 rows are counting-sorted by one workgroup into
// sub-bins of |xi| and angle inside each bucket (see prepare_shared_kernel);
// other sets find their slots with one atomic increment per bucket and wave.
// No result depends on the order inside a bucket: every query is evaluated
// independently, with the same chunks, in a fixed order over the points.
// (Shared ECT sets are not bucketed at all: ect_direct_kernel reads them in
// place.)
#include "query_body.h"

namespace ect {

namespace {

// Slot of this lane in counters[key] (global or LDS), with one atomic per
// distinct key of the wave instead of one per lane.  Every lane of the wave
// must call it; lanes with !valid get 0.
template <typename Ctr>
__device__ __forceinline__ int aggregated_add(Ctr* counters, int key, bool valid) {
    const int lane = threadIdx.x & 63;
    uint64_t pending = __ballot(valid);
    int slot = 0;
    while (pending) {
        const int leader = (int)__ffsll((unsigned long long)pending) - 1;
        const int lkey = __shfl(key, leader, 64);
        const uint64_t m = __ballot(valid && key == lkey);
        int base = 0;
        if (lane == leader) base = atomicAdd(counters + lkey, (int)__popcll(m));
        base = __shfl(base, leader, 64);
        if (valid && key == lkey) slot = base + (int)__popcll(m & ((1ull << lane) - 1ull));
        pending &= ~m;
    }
    return slot;
}

// Image of row r: the last image whose first row is <= r (offsets in global
// memory or staged in LDS).
template <typename O>
__device__ __forceinline__ int image_of(const O* off, int num_images, int64_t r) {
    int lo = 0, hi = num_images - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int64_t)off[mid] <= r) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The same from global offsets, trying first the image that evenly sized
// images would give (two independent loads confirm it); the search runs
// only when the guess is wrong.
__device__ __forceinline__ int image_of_guess(const int64_t* __restrict__ off, int num_images, int64_t r,
                                              int64_t rows) {
    const int g = (int)min<int64_t>((int64_t)num_images - 1, rows > 0 ? r * num_images / rows : 0);
    if (off[g] <= r && off[g + 1] > r) return g;
    return image_of(off, num_images, r);
}

template <int N>
__device__ __forceinline__ int64_t classify_query(const double* __restrict__ vecs, const int64_t* __restrict__ offsets,
                                                  int64_t r, int64_t rows, int num_images, int mode_hybrid,
                                                  uint32_t* __restrict__ err, QRecT<N>* rec, int64_t* slot_base) {
    int img = 0;
    int64_t r0 = 0, q = rows;
    if (offsets) {
        img = image_of_guess(offsets, num_images, r, rows);
        r0 = offsets[img];
        q = offsets[img + 1] - r0;
    }
    double v[N];
#pragma unroll
    for (int a = 0; a < N; ++a) v[a] = vecs[r * N + a];
    return classify_vec<N>(v, r, img, r0, q, mode_hybrid, err, rec, slot_base);
}

template <int N>
__global__ void __launch_bounds__(kBucketThreads)
bucket_kernel(const double* __restrict__ vecs, const int64_t* __restrict__ offsets, int64_t rows,
              int num_images, int mode_hybrid, uint32_t* __restrict__ err, QRecT<N>* __restrict__ recs,
              int32_t* __restrict__ bcnt) {
    const int64_t r = (int64_t)blockIdx.x * kBucketThreads + threadIdx.x;
    const bool valid = r < rows;
    QRecT<N> rec;
    int64_t sbase = 0, ent = 0;
    if (valid) ent = classify_query<N>(vecs, offsets, r, rows, num_images, mode_hybrid, err, &rec, &sbase);
    const int slot = aggregated_add(bcnt, (int)ent, valid);
    if (valid) recs[sbase + slot] = rec;
}

// Exclusive scan of two int64 values per thread over a 1024-thread block.
__device__ __forceinline__ void block_exclusive_scan2(int64_t& a, int64_t& b, int64_t* tot_a, int64_t* tot_b,
                                                      int64_t* s_a, int64_t* s_b) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int64_t ia = a, ib = b;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int64_t ta = __shfl_up(ia, off, 64), tb = __shfl_up(ib, off, 64);
        if (lane >= off) { ia += ta; ib += tb; }
    }
    if (lane == 63) { s_a[wave] = ia; s_b[wave] = ib; }
    __syncthreads();
    if (tid == 0) {
        int64_t ra = 0, rb = 0;
        for (int w = 0; w < 16; ++w) {
            int64_t ca = s_a[w], cb = s_b[w];
            s_a[w] = ra;
            s_b[w] = rb;
            ra += ca;
            rb += cb;
        }
        s_a[16] = ra;
        s_b[16] = rb;
    }
    __syncthreads();
    a = s_a[wave] + ia - a;
    b = s_b[wave] + ib - b;
    *tot_a = s_a[16];
    *tot_b = s_b[16];
    __syncthreads();
}

// Work list: items of entry (i, b) = ceil(bucket count / qtile) query tiles,
// each split into ceil(points / chunk) point chunks (chunk == 0: no split).
// Writes the item prefix over entries, the query-tile prefix and the chunk
// size actually used.  If the item count exceeds `capacity`, the chunk size is
// doubled until it fits.  Runs on one 1024-thread workgroup.  Entry
// e = j * 1024 + tid is thread tid's j-th (coalesced loads); up to
// kWorklistRun entries per thread stay in registers, their loads in flight
// together, and the prefixes of all j come from one joint block scan.
constexpr int kWorklistRun = 8;

__device__ __forceinline__ void build_worklist(int num_images, int B, int list_base, int NL, int shared_queries,
                               const int32_t* bcnt, const int64_t* __restrict__ list_off,
                               const int32_t* np_lds, int qtile,
                               int64_t chunk0, int64_t capacity, uint32_t* __restrict__ err,
                               int64_t* __restrict__ item_off, int64_t* __restrict__ tile_off,
                               int64_t* __restrict__ params) {
    __shared__ int64_t s_a[17], s_b[17];
    __shared__ int64_t s_wi[16][kWorklistRun], s_wt[16][kWorklistRun];
    __shared__ int64_t s_ji[kWorklistRun + 1], s_jt[kWorklistRun + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t E = (int64_t)num_images * B;
    auto tiles_pts = [&](int64_t e, int64_t* t, int64_t* np) {
        const int64_t i = e / B, b = e % B;
        const int64_t q = bcnt[shared_queries ? b : e];
        *t = (q + qtile - 1) / qtile;
        *np = np_lds ? (int64_t)np_lds[e]
                     : list_off[(i + 1) * NL + list_base + b] - list_off[i * NL + list_base + b];
    };
    auto items_of = [](int64_t t, int64_t np, int64_t chunk) {
        int64_t ch = chunk > 0 ? (np + chunk - 1) / chunk : 1;
        if (ch < 1) ch = 1;  // an empty list still gets one item per tile, which writes zeros
        return t * ch;
    };
    const int64_t R = (E + 1023) / 1024;
    const bool in_regs = R <= kWorklistRun;
    // (tiles and points of an entry, and the item and tile counts of a wave,
    // fit 32 bits: the launch grid is below 2^32 items)
    uint32_t rt[kWorklistRun], rn[kWorklistRun];
    if (in_regs) {
#pragma unroll
        for (int j = 0; j < kWorklistRun; ++j) {
            int64_t t = 0, np = 0;
            const int64_t e = (int64_t)j * 1024 + tid;
            if (e < E) tiles_pts(e, &t, &np);
            rt[j] = (uint32_t)t;
            rn[j] = (uint32_t)np;
        }
    }
    int64_t chunk = chunk0;
    if (chunk > 0 && capacity > 0) {
        for (int attempt = 0;; ++attempt) {
            int64_t my = 0;
            if (in_regs) {
#pragma unroll
                for (int j = 0; j < kWorklistRun; ++j) my += items_of(rt[j], rn[j], chunk);
            } else {
                for (int64_t e = tid; e < E; e += 1024) {
                    int64_t t, np;
                    tiles_pts(e, &t, &np);
                    my += items_of(t, np, chunk);
                }
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) my += __shfl_xor(my, off, 64);
            if (lane == 0) s_a[wave] = my;
            __syncthreads();
            int64_t total = 0;
            for (int w = 0; w < 16; ++w) total += s_a[w];
            __syncthreads();
            if (total <= capacity) break;
            chunk *= 2;
            if (attempt == 39) {
                if (tid == 0) {
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
    int64_t carry_i = 0, carry_t = 0;
    if (in_regs) {
        // inclusive wave scans of every j, then the wave totals and the j
        // totals in LDS: one pass for all rows
        uint32_t vi[kWorklistRun], si[kWorklistRun], st[kWorklistRun];
#pragma unroll
        for (int j = 0; j < kWorklistRun; ++j) {
            vi[j] = (uint32_t)items_of(rt[j], rn[j], chunk);
            si[j] = vi[j];
            st[j] = rt[j];
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t a = __shfl_up(si[j], off, 64), b = __shfl_up(st[j], off, 64);
                if (lane >= off) {
                    si[j] += a;
                    st[j] += b;
                }
            }
            if (lane == 63) {
                s_wi[wave][j] = (int64_t)si[j];
                s_wt[wave][j] = (int64_t)st[j];
            }
        }
        __syncthreads();
        // thread j < R: exclusive prefix of the 16 wave totals of row j, and the row's total
        if (tid < kWorklistRun) {
            int64_t ri = 0, rtt = 0;
            for (int w = 0; w < 16; ++w) {
                const int64_t ci = s_wi[w][tid], ct = s_wt[w][tid];
                s_wi[w][tid] = ri;
                s_wt[w][tid] = rtt;
                ri += ci;
                rtt += ct;
            }
            s_ji[tid] = ri;
            s_jt[tid] = rtt;
        }
        __syncthreads();
        if (tid == 0) {
            int64_t ri = 0, rtt = 0;
            for (int j = 0; j < kWorklistRun; ++j) {
                const int64_t ci = s_ji[j], ct = s_jt[j];
                s_ji[j] = ri;
                s_jt[j] = rtt;
                ri += ci;
                rtt += ct;
            }
            s_ji[kWorklistRun] = ri;
            s_jt[kWorklistRun] = rtt;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kWorklistRun; ++j) {
            const int64_t e = (int64_t)j * 1024 + tid;
            if (e < E) {
                item_off[e] = s_ji[j] + s_wi[wave][j] + (int64_t)(si[j] - vi[j]);
                tile_off[e] = s_jt[j] + s_wt[wave][j] + (int64_t)(st[j] - rt[j]);
            }
        }
        carry_i = s_ji[kWorklistRun];
        carry_t = s_jt[kWorklistRun];
    } else {
        for (int64_t base = 0; base < E; base += 1024) {
            const int64_t e = base + tid;
            int64_t it = 0, tl = 0;
            if (e < E) {
                int64_t np;
                tiles_pts(e, &tl, &np);
                it = items_of(tl, np, chunk);
            }
            int64_t tot_i, tot_t;
            block_exclusive_scan2(it, tl, &tot_i, &tot_t, s_a, s_b);
            if (e < E) {
                item_off[e] = carry_i + it;
                tile_off[e] = carry_t + tl;
            }
            carry_i += tot_i;
            carry_t += tot_t;
        }
    }
    if (tid == 0) {
        item_off[E] = carry_i;
        tile_off[E] = carry_t;
        params[0] = carry_i;
        params[1] = carry_t;
        params[2] = chunk;
    }
}

__global__ void __launch_bounds__(1024)
worklist_kernel(int num_images, int B, int list_base, int NL, int shared_queries,
                const int32_t* __restrict__ bcnt, const int64_t* __restrict__ list_off,
                int qtile, int64_t chunk0, int64_t capacity, uint32_t* __restrict__ err,
                int64_t* __restrict__ item_off, int64_t* __restrict__ tile_off,
                int64_t* __restrict__ params) {
    build_worklist(num_images, B, list_base, NL, shared_queries, bcnt, list_off, nullptr, qtile, chunk0, capacity,
                   err, item_off, tile_off, params);
}

// Shared hybrid query sets of at most kSharedMaxRows rows: one 1024-thread
// workgroup.  Wave w takes a contiguous block of rows and walks it 64 rows at
// a time (lane l takes the l-th row of a batch, so loads coalesce).  Queries
// are counting-sorted by (orthant pair, sub-bin): LDS counters, an exclusive
// scan of them, then each record goes to its bin's next slot.  The sub-bin is
// the octave of |xi| (major), then the angle of (xi_0, xi_1) modulo pi in 32
// bins (of a monotone stand-in for the angle).  The 64 queries of a tile then
// project each point to nearby values, so the lanes of a wave mostly fall on
// the same side of the Bessel kernel's |z| < 8 branch (on a 512^2 field with
// 4096 random xi, waves that need both branches drop from 95% to about 23% of
// the (wave, point) pairs).  Every query's sum is independent of its tile and
// lane, so the order inside a sub-bin (LDS atomics) changes no output bit.  A
// work list of at most 64 entries is then built by one wave.
constexpr int kPrepRows = 8;   // query rows in flight per thread (ragged small sets)
constexpr int64_t kSharedMaxRows = 65536;
template <int N>
__global__ void __launch_bounds__(1024)
prepare_shared_kernel(const double* __restrict__ vecs, int64_t rows, int num_images,
                      uint32_t* __restrict__ err, QRecT<N>* __restrict__ recs, int32_t* __restrict__ bcnt,
                      const int64_t* __restrict__ list_off, int list_base, int NL, int qtile, int64_t chunk0,
                      int64_t capacity, int64_t* __restrict__ item_off, int64_t* __restrict__ tile_off,
                      int64_t* __restrict__ params) {
    constexpr int W = 16;
    constexpr int U = 4;   // batches whose loads are in flight together
    __shared__ int32_t s_wc[W];
    __shared__ int32_t s_tot[1 << kMaxDim];
    __shared__ int32_t s_start[1 << kMaxDim];
    __shared__ int32_t s_bin[(1 << (kMaxDim - 1)) * kSubBins];   // counts, then slots
    const int B = 1 << (N - 1);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t EW = (int64_t)num_images * B;
    // list sizes of a small work list, requested first
    int64_t np_lane = 0;
    if (EW <= 64 && wave == 0 && lane < EW) {
        const int i = lane / B, b = lane % B;
        np_lane = list_off[(int64_t)(i + 1) * NL + list_base + b] - list_off[(int64_t)i * NL + list_base + b];
    }
    const int64_t per = ((rows + W - 1) / W + 63) / 64 * 64;   // rows per wave, whole batches
    const int64_t w0 = min(rows, (int64_t)wave * per), w1 = min(rows, w0 + per);
    auto load = [&](int64_t rb, double (&v)[U][N]) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int a = 0; a < N; ++a) {
                const int64_t r = rb + 64 * u + lane;
                v[u][a] = r < w1 ? vecs[r * N + a] : 0.0;
            }
    };
    {
        // counting sort by (bucket, sub-bin): counts, exclusive scan, slots.
        // When every wave's block is one batch (up to 16 * 64 * U rows), the
        // records and bins stay in registers between the two phases.
        const int nbins = B * kSubBins;
        const bool one = per <= 64 * U;
        for (int i = tid; i < nbins; i += 1024) s_bin[i] = 0;
        QRecT<N> keep[U];
        int64_t keep_sb[U];
        int keep_bin[U];
        if (one) {
            double v[U][N];
            load(w0, v);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t r = w0 + 64 * u + lane;
                keep_bin[u] = -1;
                keep_sb[u] = 0;
                if (r < w1) {
                    const int key = (int)classify_vec<N>(v[u], r, 0, 0, rows, 1, err, &keep[u], &keep_sb[u]);
                    keep_bin[u] = key * kSubBins + sub_bin<N>(keep[u].v);
                }
            }
        }
        __syncthreads();
        if (one) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (keep_bin[u] >= 0) atomicAdd(&s_bin[keep_bin[u]], 1);
        } else {
            for (int64_t rb = w0; rb < w1; rb += 64 * U) {
                double v[U][N];
                load(rb, v);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t r = rb + 64 * u + lane;
                    if (r >= w1) continue;
                    QRecT<N> rec;
                    int64_t sb;
                    const int key = (int)classify_vec<N>(v[u], r, 0, 0, rows, 1, err, &rec, &sb);
                    atomicAdd(&s_bin[key * kSubBins + sub_bin<N>(rec.v)], 1);
                }
            }
        }
        __syncthreads();
        const int bpt = (nbins + 1023) / 1024;   // bins per thread
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
        if (lane == 63) s_wc[wave] = inc;
        __syncthreads();
        int32_t run = inc - loc, total = 0;
        for (int w = 0; w < W; ++w) {
            if (w < wave) run += s_wc[w];
            total += s_wc[w];
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
        if (one) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (keep_bin[u] < 0) continue;
                const int pos = atomicAdd(&s_bin[keep_bin[u]], 1) - s_start[keep_bin[u] / kSubBins];
                recs[keep_sb[u] + pos] = keep[u];
            }
        } else {
            for (int64_t rb = w0; rb < w1; rb += 64 * U) {
                double v[U][N];
                load(rb, v);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t r = rb + 64 * u + lane;
                    if (r >= w1) continue;
                    QRecT<N> rec;
                    int64_t sb = 0;
                    const int key = (int)classify_vec<N>(v[u], r, 0, 0, rows, 1, nullptr, &rec, &sb);
                    const int pos = atomicAdd(&s_bin[key * kSubBins + sub_bin<N>(rec.v)], 1) - s_start[key];
                    recs[sb + pos] = rec;
                }
            }
        }
        // the work list needs only the bucket totals: no barrier, so the
        // record stores drain while it is built
        if (EW <= 64) {
            if (wave == 0)
                worklist_wave(EW, lane < EW ? s_tot[lane % B] : 0, np_lane, qtile, chunk0, capacity, err, item_off,
                              tile_off, params);
        } else {
            build_worklist(num_images, B, list_base, NL, 1, s_tot, list_off, nullptr, qtile, chunk0, capacity, err,
                           item_off, tile_off, params);
        }
    }
}

// Small query sets: bucketing with LDS counters and the work list in one
// 1024-thread workgroup (one launch instead of three).  Everything the
// bucketing and the work list read is fetched up front with independent
// loads (list sizes and ragged offsets staged in LDS, kPrepRows query rows in
// flight per thread), so the kernel waits on memory a few times, not once per
// row and per entry.
constexpr int kSmallMaxOffsets = kSmallMaxEntries / 2 + 1;   // ragged: images <= entries / 2

template <int N>
__global__ void __launch_bounds__(1024)
prepare_small_kernel(const double* __restrict__ vecs, const int64_t* __restrict__ offsets, int64_t rows,
                     int num_images, int mode_hybrid, uint32_t* __restrict__ err, QRecT<N>* __restrict__ recs,
                     int32_t* __restrict__ bcnt, const int64_t* __restrict__ list_off, int list_base, int NL,
                     int qtile, int64_t chunk0, int64_t capacity, int64_t* __restrict__ item_off,
                     int64_t* __restrict__ tile_off, int64_t* __restrict__ params) {
    __shared__ int32_t s_cnt[kSmallMaxEntries];
    __shared__ int32_t s_np[kSmallMaxEntries];
    __shared__ int32_t s_off[kSmallMaxOffsets];
    const int B = mode_hybrid ? (1 << (N - 1)) : (1 << N);
    const int groups = offsets ? num_images : 1;
    const int E = groups * B;
    const int64_t EW = (int64_t)num_images * B;     // work-list entries
    const bool stage_np = EW <= kSmallMaxEntries && item_off != nullptr;
    const int tid = threadIdx.x;
    // the first batch of query rows is requested before anything else
    double v[kPrepRows][N];
    auto load_rows = [&](int64_t base) {
#pragma unroll
        for (int j = 0; j < kPrepRows; ++j) {
            const int64_t r = base + (int64_t)j * 1024 + tid;
#pragma unroll
            for (int a = 0; a < N; ++a) v[j][a] = r < rows ? vecs[r * N + a] : 0.0;
        }
    };
    load_rows(0);
    for (int i = tid; i < E; i += 1024) s_cnt[i] = 0;
    if (stage_np)
        for (int i = tid; i < (int)EW; i += 1024) {
            const int img = i / B, b = i % B;
            s_np[i] = (int32_t)(list_off[(int64_t)(img + 1) * NL + list_base + b] -
                                list_off[(int64_t)img * NL + list_base + b]);
        }
    if (offsets)
        for (int i = tid; i <= num_images; i += 1024) s_off[i] = (int32_t)offsets[i];
    __syncthreads();
    for (int64_t base = 0; base < rows; base += 1024 * kPrepRows) {
        if (base > 0) load_rows(base);
#pragma unroll
        for (int j = 0; j < kPrepRows; ++j) {
            const int64_t r = base + (int64_t)j * 1024 + tid;
            const bool valid = r < rows;
            QRecT<N> rec;
            int64_t sbase = 0, ent = 0;
            if (valid) {
                int img = 0;
                int64_t r0 = 0, q = rows;
                if (offsets) {
                    img = image_of(s_off, num_images, r);
                    r0 = s_off[img];
                    q = (int64_t)s_off[img + 1] - r0;
                }
                ent = classify_vec<N>(v[j], r, img, r0, q, mode_hybrid, err, &rec, &sbase);
            }
            const int slot = aggregated_add(s_cnt, (int)ent, valid);
            if (valid) recs[sbase + slot] = rec;
        }
    }
    __syncthreads();
    for (int i = tid; i < E; i += 1024) bcnt[i] = s_cnt[i];
    if (!item_off) return;   // buckets only (the batch ECT kernel needs no work list)
    build_worklist(num_images, B, list_base, NL, offsets == nullptr ? 1 : 0, s_cnt, list_off,
                   stage_np ? s_np : nullptr, qtile, chunk0, capacity, err, item_off, tile_off, params);
}

template <int N>
hipError_t launch_prepare_typed(const ect_query_set& qs, int num_images, bool hybrid, uint32_t* err, void* recs_v,
                                int32_t* bcnt, const int64_t* list_off, int list_base, int NL, int qtile,
                                int64_t chunk, int64_t capacity, int64_t* item_off, int64_t* tile_off,
                                int64_t* params, hipStream_t stream) {
    QRecT<N>* recs = (QRecT<N>*)recs_v;
    const int B = hybrid ? (1 << (N - 1)) : (1 << N);
    const int64_t rows = qs.count;  // shared: the set itself; ragged: all rows
    const int groups = qs.offsets ? num_images : 1;
    const bool shared = qs.offsets == nullptr;
    if (shared && hybrid && rows <= kSharedMaxRows) {
        hipLaunchKernelGGL(prepare_shared_kernel<N>, dim3(1), dim3(1024), 0, stream, qs.vecs, rows, num_images,
                           err, recs, bcnt, list_off, list_base, NL, qtile, chunk, capacity, item_off, tile_off,
                           params);
        return hipGetLastError();
    }
    if (rows <= kSmallMaxRows && (int64_t)groups * B <= kSmallMaxEntries) {
        hipLaunchKernelGGL(prepare_small_kernel<N>, dim3(1), dim3(1024), 0, stream, qs.vecs, qs.offsets, rows,
                           num_images, hybrid ? 1 : 0, err, recs, bcnt, list_off, list_base, NL, qtile, chunk,
                           capacity, item_off, tile_off, params);
        return hipGetLastError();
    }
    hipError_t e = launch_fill_u32((uint32_t*)bcnt, (int64_t)groups * B, 0u, stream);
    if (e != hipSuccess) return e;
    if (rows > 0) {
        const unsigned blocks = (unsigned)((rows + kBucketThreads - 1) / kBucketThreads);
        const int ni = qs.offsets ? num_images : 1;
        hipLaunchKernelGGL(bucket_kernel<N>, dim3(blocks), dim3(kBucketThreads), 0, stream, qs.vecs, qs.offsets,
                           rows, ni, hybrid ? 1 : 0, err, recs, bcnt);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (!item_off) return hipSuccess;   // buckets only
    hipLaunchKernelGGL(worklist_kernel, dim3(1), dim3(1024), 0, stream, num_images, B, list_base, NL,
                       shared ? 1 : 0, bcnt, list_off, qtile, chunk, capacity, err, item_off, tile_off, params);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_prepare(int ndim, const ect_query_set& qs, int num_images, bool hybrid, uint32_t* err,
                          void* recs, int32_t* bcnt, const int64_t* list_off, int list_base, int NL, int qtile,
                          int64_t chunk, int64_t capacity, int64_t* item_off, int64_t* tile_off, int64_t* params,
                          hipStream_t stream) {
    if (ndim == 2)
        return launch_prepare_typed<2>(qs, num_images, hybrid, err, recs, bcnt, list_off, list_base, NL, qtile, chunk,
                                       capacity, item_off, tile_off, params, stream);
    if (ndim == 3)
        return launch_prepare_typed<3>(qs, num_images, hybrid, err, recs, bcnt, list_off, list_base, NL, qtile, chunk,
                                       capacity, item_off, tile_off, params, stream);
    return launch_prepare_typed<4>(qs, num_images, hybrid, err, recs, bcnt, list_off, list_base, NL, qtile, chunk,
                                   capacity, item_off, tile_off, params, stream);
}

}  // namespace ect
