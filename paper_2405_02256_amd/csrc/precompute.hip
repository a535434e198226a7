// Per-vertex classification of lower-star critical values and their ordered
// compaction into per-sign-vector lists (gfx950).
//
// For a vertex k and sign vector eps, the lower star is the set of cells of
// the vertex's star on which k is the highest vertex for any xi of sign eps:
// along every axis where such a cell extends, it extends towards -eps_a.  So
//   L(eps, k) = sum over delta in {0,1}^n of (-1)^|delta| phi(cell(k, -delta*eps))
// over existing cells (Delta^- of Sec. 3, enumerated as in Sec. 4.2 and
// Appendix A), and Delta^ord(eps, k) = L(-eps, k) - L(eps, k) because the upper
// star for eps is the lower star for -eps.
//
// Cell values come straight from the pixels (nothing is materialised):
//   primal  a cell takes the min over its coface pixels (Sec. 4.1);
//   dual    a cell takes the min over its vertex pixels (Sec. 5).
// Pixel coordinates are clamped into the image: a clamped duplicate never
// changes a min over existing cofaces, and cells that do not exist are masked
// by the existence test on the vertex index.
//
// Compaction is single pass and ordered: every workgroup takes the next tile
// id from a counter, counts its nonzero values per list with wave ballots,
// publishes the counts and resolves its global offset by decoupled look-back
// over the preceding tiles (the workgroup's waves inspect 64 predecessors each
// per round, for every list at once), then writes its entries in vertex
// order.  Lists therefore come out sorted by linear vertex index, and
// identically on every run.
#include "ect_internal.h"

namespace ect {

namespace {

// Look-back status word: flag (bits 63-62), run parity (bit 61), count.  A
// word is current when its parity bit matches the run's: every word left by
// run r-1 reads as "not yet published" in run r, so re-runs need no reset
// launch.  The run number comes from a 64-bit counter in the plan's workspace
// that is never reset:
//   resident grids (every workgroup fits on the chip at once): tile =
//     blockIdx.x, the counter holds the run number; every workgroup reads it
//     first, and the last tile increments it once its look-back is complete,
//     which implies that every tile has published a word, so has read it;
//   larger grids: the counter hands out tickets in start order (tile =
//     ticket % num_tiles, run = ticket / num_tiles), so a workgroup only
//     waits on tiles whose workgroups have started.
constexpr uint64_t kFlagAggregate = 1ull << 62;
constexpr uint64_t kFlagInclusive = 2ull << 62;
constexpr uint64_t kFlagMask = 3ull << 62;
constexpr uint64_t kParityBit = 1ull << 61;
constexpr uint64_t kValueMask = (1ull << 61) - 1;
constexpr int kLookbackSpinLimit = 1 << 22;

__device__ __forceinline__ uint32_t udiv(uint32_t v, uint32_t d, double inv_d, uint32_t* rem) {
    uint32_t q = (uint32_t)((double)v * inv_d);
    int64_t r = (int64_t)v - (int64_t)q * d;
    if (r < 0) { q -= 1; r += d; }
    else if (r >= (int64_t)d) { q += 1; r -= d; }
    *rem = (uint32_t)r;
    return q;
}

template <int N>
__host__ __device__ constexpr int pow3() { return N == 1 ? 3 : (N == 2 ? 9 : 27); }

// Star cell index: sigma_a in {-1, 0, +1} -> digit sigma_a + 1 in base 3.
template <int N>
__device__ __forceinline__ constexpr int star_index(const int* sigma) {
    int s = 0, m = 1;
    for (int a = 0; a < N; ++a) { s += (sigma[a] + 1) * m; m *= 3; }
    return s;
}

template <typename T>
__device__ __forceinline__ int32_t px_load(const T* __restrict__ img, int64_t i) {
    return (int32_t)img[i];
}

// Pixels a vertex's star depends on: primal, the 2^N pixels k_a - 1 + d_a
// (d in {0,1}^N); dual, the 3^N pixels k + t (t in {-1,0,1}^N).  Coordinates
// are clamped into the image.
template <int N, int CONS>
__host__ __device__ constexpr int nb_count() { return CONS == ECT_PRIMAL ? (1 << N) : pow3<N>(); }

template <int N, int CONS, typename T>
__device__ __forceinline__ void load_neighbourhood(const T* __restrict__ img, const ImageDesc& d, const int* k,
                                                   int32_t* p) {
#pragma unroll
    for (int c = 0; c < nb_count<N, CONS>(); ++c) {
        int64_t idx = 0, stride = 1;
        int r = c;
#pragma unroll
        for (int a = 0; a < N; ++a) {
            int x;
            if constexpr (CONS == ECT_PRIMAL) {
                x = k[a] - 1 + ((c >> a) & 1);
            } else {
                x = k[a] + (r % 3) - 1;
                r /= 3;
            }
            x = x < 0 ? 0 : (x > d.dims[a] - 1 ? d.dims[a] - 1 : x);
            idx += (int64_t)x * stride;
            stride *= d.dims[a];
        }
        p[c] = px_load(img, idx);
    }
}

// Critical values of one vertex from its neighbourhood: L[e] for the 2^N sign
// vectors, D[e] for the 2^(N-1) sign vectors with eps_{N-1} = +1.
template <int N, int CONS>
__device__ __forceinline__ void vertex_values(const int32_t* p, const ImageDesc& d, const int* k, int32_t* L,
                                              int32_t* D) {
    constexpr int S = pow3<N>();
    int32_t val[S];
    if constexpr (CONS == ECT_PRIMAL) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            // sigma digits: 0 -> -1 (pixel d=0 only), 1 -> 0 (both), 2 -> +1 (pixel d=1 only)
            int32_t m = 0x7fffffff;
#pragma unroll
            for (int c = 0; c < (1 << N); ++c) {
                bool ok = true;
                int r = s;
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    int dig = r % 3;
                    r /= 3;
                    int bit = (c >> a) & 1;
                    if ((dig == 0 && bit != 0) || (dig == 2 && bit != 1)) ok = false;
                }
                if (ok) m = min(m, p[c]);
            }
            val[s] = m;
        }
    } else {
        // a cell extending by sigma takes the min over the pixels k + t with t_a in {0, sigma_a}
#pragma unroll
        for (int s = 0; s < S; ++s) {
            int32_t m = 0x7fffffff;
#pragma unroll
            for (int c = 0; c < S; ++c) {
                bool ok = true;
                int rs = s, rc = c;
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    int sg = rs % 3 - 1, t = rc % 3 - 1;
                    rs /= 3;
                    rc /= 3;
                    if (!(t == 0 || t == sg)) ok = false;
                }
                if (ok) m = min(m, p[c]);
            }
            val[s] = m;
        }
    }
    // existence: a cell extending towards -1 (+1) along a needs k_a >= 1 (k_a <= N_a - 1)
    bool hm[N], hp[N];
#pragma unroll
    for (int a = 0; a < N; ++a) { hm[a] = k[a] >= 1; hp[a] = k[a] <= d.N[a] - 1; }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        bool ex = true;
        int r = s;
#pragma unroll
        for (int a = 0; a < N; ++a) {
            int dig = r % 3;
            r /= 3;
            if (dig == 0 && !hm[a]) ex = false;
            if (dig == 2 && !hp[a]) ex = false;
        }
        if (!ex) val[s] = 0;
    }
#pragma unroll
    for (int e = 0; e < (1 << N); ++e) {
        int32_t acc = 0;
#pragma unroll
        for (int del = 0; del < (1 << N); ++del) {
            int sigma[N];
            int par = 0;
#pragma unroll
            for (int a = 0; a < N; ++a) {
                int eps = ((e >> a) & 1) ? -1 : 1;
                int dl = (del >> a) & 1;
                sigma[a] = dl ? -eps : 0;
                par += dl;
            }
            int32_t v = val[star_index<N>(sigma)];
            acc += (par & 1) ? -v : v;
        }
        L[e] = acc;
    }
    constexpr int full = (1 << N) - 1;
#pragma unroll
    for (int e = 0; e < (1 << (N - 1)); ++e) D[e] = L[e ^ full] - L[e];
}

// Once per plan: clear the error word, the ticket counter and the status words.
__global__ void reset_kernel(uint32_t* __restrict__ err, uint64_t* __restrict__ ticket, uint64_t* __restrict__ status,
                             int64_t nstatus) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (i == 0) { err[0] = 0u; err[1] = 0u; *ticket = 0ull; }
    for (; i < nstatus; i += stride) status[i] = 0ull;
}

// Sum over lanes i < count of the values of words[i * stride] (wave 0, every
// lane gets the sum), waiting until each of those words is current (run
// parity) and published.  Returns false if the spin limit was reached.
template <int NL>
__device__ __forceinline__ bool sum_published(const uint64_t* words, int64_t count, uint64_t parity, uint64_t* sums,
                                              uint32_t* err) {
    const int lane = threadIdx.x & 63;
    for (int spins = 0;; ++spins) {
        uint64_t wv[NL];
#pragma unroll
        for (int l = 0; l < NL; ++l)
            wv[l] = lane < count ? __hip_atomic_load(words + (int64_t)lane * NL + l, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)
                                 : (kFlagAggregate | parity);
        bool ready = true;
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const bool ok = (wv[l] & kParityBit) == parity && (wv[l] & kFlagMask) != 0;
            ready = ready && __ballot(!ok) == 0;
        }
        if (ready) {
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                uint64_t v = lane < count ? (wv[l] & kValueMask) : 0ull;
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
                sums[l] = v;
            }
            return true;
        }
        if (spins > kLookbackSpinLimit) {
            if (lane == 0) raise_error(err, ECT_DEVERR_LOOKBACK);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

template <int N, int CONS, typename T>
__global__ void __launch_bounds__(kPrecomputeThreads)
classify_compact(const T* __restrict__ pixels, const ImageDesc* __restrict__ descs,
                 const int64_t* __restrict__ tile_start, int32_t num_images, int64_t num_tiles,
                 uint32_t* __restrict__ err, uint64_t* __restrict__ ticket, uint64_t* __restrict__ status,
                 uint64_t* __restrict__ gstatus, int64_t* __restrict__ list_off, Point* __restrict__ points,
                 int64_t capacity, int resident) {
    constexpr int NC = 1 << N;
    constexpr int NO = 1 << (N - 1);
    constexpr int NL = NC + NO;
    constexpr int W = kPrecomputeThreads / 64;
    constexpr int J = kVertsPerThread;

    __shared__ uint64_t s_ticket;
    __shared__ int32_t s_cnt[J][W][NL];   // per (round, wave, list) counts, then exclusive offsets
    __shared__ int64_t s_base[NL];
    __shared__ uint64_t s_lb_sum[W][NL];
    __shared__ int s_lb_state[W][NL];   // 0: no inclusive prefix in the part, 1: found one, 2: a word not ready

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    if (tid == 0)
        s_ticket = resident ? __hip_atomic_load(ticket, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                            : __hip_atomic_fetch_add(ticket, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const uint64_t tk = s_ticket;
    const int64_t tile = resident ? (int64_t)blockIdx.x : (int64_t)(tk % (uint64_t)num_tiles);
    const uint64_t run = resident ? tk : tk / (uint64_t)num_tiles;
    const uint64_t parity = (run & 1ull) ? kParityBit : 0ull;

    // image owning this tile: last i with tile_start[i] <= tile
    int lo = 0, hi = num_images - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (tile_start[mid] <= tile) lo = mid; else hi = mid - 1;
    }
    const ImageDesc d = descs[lo];
    const int img_id = lo;
    const T* __restrict__ img = pixels + d.pixel_offset;
    const int64_t vbase = (tile - d.tile_start) * kTileVerts;
    const double inv0 = 1.0 / (double)d.V[0];
    const double inv1 = 1.0 / (double)d.V[1];

    int32_t vals[J][NL];
    int kk[J][3];
    bool valid[J];
    // every round's pixel loads are issued before any vertex is classified
    int32_t nb[J][nb_count<N, CONS>()];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        int64_t v = vbase + j * kPrecomputeThreads + tid;
        valid[j] = v < d.nvert;
        uint32_t r0, r1;
        uint32_t q0 = udiv((uint32_t)(valid[j] ? v : 0), (uint32_t)d.V[0], inv0, &r0);
        uint32_t q1 = N == 3 ? udiv(q0, (uint32_t)d.V[1], inv1, &r1) : 0u;
        kk[j][0] = (int)r0;
        kk[j][1] = N == 3 ? (int)r1 : (int)q0;
        kk[j][2] = N == 3 ? (int)q1 : 0;
        load_neighbourhood<N, CONS, T>(img, d, kk[j], nb[j]);
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
        int32_t L[NC], D[NO];
        vertex_values<N, CONS>(nb[j], d, kk[j], L, D);
#pragma unroll
        for (int l = 0; l < NC; ++l) vals[j][l] = valid[j] ? L[l] : 0;
#pragma unroll
        for (int l = 0; l < NO; ++l) vals[j][NC + l] = valid[j] ? D[l] : 0;
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            uint64_t b = __ballot(vals[j][l] != 0);
            if (lane == 0) s_cnt[j][wave][l] = __popcll(b);
        }
    }
    __syncthreads();

    // tile aggregates (wave 0, lane l < NL owns list l); per-(round, wave)
    // counts become exclusive offsets inside the tile
    uint64_t agg = 0;
    if (wave == 0 && lane < NL) {
        int32_t run = 0;
#pragma unroll
        for (int j = 0; j < J; ++j)
#pragma unroll
            for (int w = 0; w < W; ++w) {
                int32_t c = s_cnt[j][w][lane];
                s_cnt[j][w][lane] = run;
                run += c;
            }
        agg = (uint64_t)run;
        if (tile > 0 || resident)   // the two-level scan also reads tile 0's aggregate
            __hip_atomic_store(status + tile * NL + lane, kFlagAggregate | parity | agg, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    if (resident) {
        // Two-level scan (every tile is running, so none waits on an unstarted
        // one): tiles form groups of 64; wave 0 sums the aggregates of the
        // tile's predecessors in its group, the group's last tile publishes
        // the group total, and the totals of the preceding groups complete the
        // prefix.  Each tile reads at most 63 + groups words per list, where a
        // window look-back over simultaneously finishing tiles reads hundreds.
        if (wave == 0) {
            const int64_t g = tile >> 6, k = tile & 63;
            uint64_t loc[NL], grp[NL];
            bool ok = sum_published<NL>(status + (g << 6) * NL, k, parity, loc, err);
            if (ok && (k == 63 || tile == num_tiles - 1) && lane < NL) {
                uint64_t mine = 0;
#pragma unroll
                for (int l = 0; l < NL; ++l) if (lane == l) mine = loc[l];
                __hip_atomic_store(gstatus + g * NL + lane, kFlagAggregate | parity | (mine + agg), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            if (ok) ok = sum_published<NL>(gstatus, g, parity, grp, err);
            // every group total is in, so every tile has read the run number
            if (tile == num_tiles - 1 && lane == 0)
                __hip_atomic_store(ticket, tk + 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (lane < NL) {
                uint64_t mine = 0;
#pragma unroll
                for (int l = 0; l < NL; ++l) if (lane == l) mine = ok ? loc[l] + grp[l] : 0;
                s_base[lane] = (int64_t)mine;
                if (tile == d.tile_start) list_off[(int64_t)img_id * NL + lane] = (int64_t)mine;
                if (tile == num_tiles - 1) list_off[(int64_t)num_images * NL + lane] = (int64_t)(mine + agg);
            }
        }
    } else {
    // Decoupled look-back over windows of 64 * W predecessor tiles: lane i of
    // wave w inspects tile base - 64 w - i for every list at once.  A status
    // word carries both its flag and its count, so relaxed device-scope
    // atomics suffice (no fence, hence no L2 write-back between the chip's
    // non-coherent L2 slices); the list entries are only read by later
    // kernels.  Per list, the nearest tile holding an inclusive prefix ends
    // the walk; every tile in front of it must have published its aggregate,
    // otherwise the window is read again.  The waves' window parts are
    // combined in order through LDS.
    {
        uint64_t excl[NL];
        int64_t wbase[NL];
        bool done[NL];
#pragma unroll
        for (int l = 0; l < NL; ++l) { excl[l] = 0; wbase[l] = tile - 1; done[l] = tile == 0; }
        int spins = 0;
        bool all_done = tile == 0;
        while (!all_done) {
            // every list's word is requested before any is examined, so the
            // loads are in flight together
            uint64_t wvs[NL];
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                const int64_t j = wbase[l] - 64 * wave - lane;
                wvs[l] = (!done[l] && j >= 0)
                             ? __hip_atomic_load(status + j * NL + l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                             : (kFlagInclusive | parity);
            }
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                if (done[l]) continue;
                const uint64_t wv = wvs[l];
                const uint64_t f = wv & kFlagMask;
                const bool current = (wv & kParityBit) == parity;
                const uint64_t incl = __ballot(current && f == kFlagInclusive);
                const uint64_t notready = __ballot(!current || f == 0);
                const int first = incl ? (int)__ffsll((unsigned long long)incl) - 1 : 64;
                const uint64_t upto = first >= 63 ? ~0ull : ((1ull << (first + 1)) - 1ull);
                uint64_t v = (lane <= first) ? (wv & kValueMask) : 0ull;
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
                if (lane == 0) {
                    s_lb_sum[wave][l] = v;
                    s_lb_state[wave][l] = (notready & upto) ? 2 : (first < 64 ? 1 : 0);
                }
            }
            __syncthreads();
            // every thread combines the W parts in order (same result everywhere)
            bool waiting = false;
            all_done = true;
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                if (done[l]) continue;
                uint64_t total = 0;
                int state = 0;
                for (int w = 0; w < W; ++w) {
                    const int st = s_lb_state[w][l];
                    if (st == 2) { state = 2; break; }
                    total += s_lb_sum[w][l];
                    if (st == 1) { state = 1; break; }
                }
                if (state == 2) { waiting = true; all_done = false; continue; }
                excl[l] += total;
                if (state == 1) done[l] = true;
                else { wbase[l] -= 64 * W; all_done = false; }
            }
            __syncthreads();   // the parts are rewritten by the next round
            if (waiting) {
                if (++spins > kLookbackSpinLimit) {
                    if (tid == 0) raise_error(err, ECT_DEVERR_LOOKBACK);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        if (wave == 0 && lane < NL) {
            uint64_t mine = 0;
#pragma unroll
            for (int l = 0; l < NL; ++l) if (lane == l) mine = excl[l];
            __hip_atomic_store(status + tile * NL + lane, kFlagInclusive | parity | (mine + agg), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            s_base[lane] = (int64_t)mine;
            if (tile == d.tile_start) list_off[(int64_t)img_id * NL + lane] = (int64_t)mine;
            if (tile == num_tiles - 1) list_off[(int64_t)num_images * NL + lane] = (int64_t)(mine + agg);
        }
    }
    }
    __syncthreads();

#pragma unroll
    for (int j = 0; j < J; ++j) {
        Point pt;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            pt.x[a] = a < N ? __fma_rn(d.spacing[a], (double)kk[j][a], d.origin[a]) : 0.0;
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const bool nz = vals[j][l] != 0;
            const uint64_t b = __ballot(nz);
            if (nz) {
                const int rank = __popcll(b & ((1ull << lane) - 1ull));
                const int64_t pos = s_base[l] + s_cnt[j][wave][l] + rank;
                pt.val = (double)vals[j][l];
                points[(int64_t)l * capacity + pos] = pt;
            }
        }
    }
}

template <int N, int CONS, typename T>
hipError_t launch_typed(const Plan& p, bool first, hipStream_t stream) {
    const PlanLayout& L = p.lay;
    uint32_t* err = (uint32_t*)(p.ws + L.err);
    uint64_t* ticket = (uint64_t*)(p.ws + L.err + 8);
    uint64_t* status = (uint64_t*)(p.ws + L.status);
    uint64_t* gstatus = status + L.num_tiles * num_lists(N);   // group totals of the two-level scan
    const int64_t nstatus = (L.num_tiles + (L.num_tiles + 63) / 64) * num_lists(N);
    hipError_t e = hipSuccess;
    if (first) {
        int rblocks = (int)std::min<int64_t>((nstatus + 255) / 256 + 1, 4096);
        hipLaunchKernelGGL(reset_kernel, dim3(rblocks), dim3(256), 0, stream, err, ticket, status, nstatus);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    e = stage_mark(ECT_STAGE_PRECOMPUTE, false, stream);
    if (e != hipSuccess) return e;
    if (p.precompute_resident < 0) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, classify_compact<N, CONS, T>, kPrecomputeThreads,
                                                         0) != hipSuccess)
            per_cu = 0;
        // the two-level scan covers 64 groups of 64 tiles
        p.precompute_resident = ((int64_t)per_cu * p.num_cus >= L.num_tiles && L.num_tiles <= 64 * 64) ? 1 : 0;
    }
    hipLaunchKernelGGL((classify_compact<N, CONS, T>), dim3((unsigned)L.num_tiles), dim3(kPrecomputeThreads),
                       0, stream, (const T*)p.pixels, (const ImageDesc*)(p.ws + L.desc),
                       (const int64_t*)(p.ws + L.tile_start), p.num_images, L.num_tiles, err, ticket, status, gstatus,
                       (int64_t*)(p.ws + L.list_off), (Point*)(p.ws + L.points), L.capacity,
                       (int)p.precompute_resident);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return stage_mark(ECT_STAGE_PRECOMPUTE, true, stream);
}

template <int N, int CONS>
hipError_t launch_dtype(const Plan& p, bool first, hipStream_t s) {
    switch (p.dtype) {
        case ECT_U8: return launch_typed<N, CONS, uint8_t>(p, first, s);
        case ECT_I16: return launch_typed<N, CONS, int16_t>(p, first, s);
        default: return launch_typed<N, CONS, int32_t>(p, first, s);
    }
}

}  // namespace

hipError_t launch_precompute(const Plan& p, bool first, hipStream_t stream) {
    if (p.ndim == 2)
        return p.construction == ECT_PRIMAL ? launch_dtype<2, ECT_PRIMAL>(p, first, stream)
                                            : launch_dtype<2, ECT_DUAL>(p, first, stream);
    return p.construction == ECT_PRIMAL ? launch_dtype<3, ECT_PRIMAL>(p, first, stream)
                                        : launch_dtype<3, ECT_DUAL>(p, first, stream);
}

}  // namespace ect
