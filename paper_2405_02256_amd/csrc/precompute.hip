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
// Compaction is ordered: every tile counts its nonzero values per list with
// wave ballots and needs the counts of all earlier tiles.  When every tile's
// workgroup fits on the chip at once, one pass does it: a tile publishes its
// counts and resolves its offset by a two-level scan (its group of 64 tiles,
// then the group totals) before writing its entries in vertex order.  Larger
// plans count, scan the counts in one workgroup, and classify again to write
// (three launches, no workgroup ever waits on another).  Lists come out
// sorted by linear vertex index, and identically on every run.
#include <type_traits>

#include "query_body.h"

namespace ect {

namespace {

// Status word of the single pass: flag (bits 63-62), run parity (bit 61),
// count.  A word is current when its parity bit matches the run's: every word
// left by run r-1 reads as "not yet published" in run r, so re-runs need no
// reset launch.  The run number is a 64-bit counter in the plan's workspace
// that every workgroup reads first; the last tile advances it once every group
// total is in, which implies that every tile has published a word, hence has
// read it.
constexpr uint64_t kFlagAggregate = 1ull << 62;
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
__host__ __device__ constexpr int pow3() {
    int p = 1;
    for (int a = 0; a < N; ++a) p *= 3;
    return p;
}

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
template <typename T>
__device__ __forceinline__ int32_t px_load(const T* __restrict__ img, uint32_t i) {
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

// Two-axis primal images, the common case, with the shared subexpressions
// written out: the four pixels around vertex k (a = (k0-1, k1-1), b = (k0,
// k1-1), c = (k0-1, k1), d = (k0, k1), clamped into the image), the vertex
// value (min of the four), the four edge values (min of the two pixels on
// either side) and the four squares, masked where the cell does not exist;
// then L(eps) = vertex - edge along -eps_0 - edge along -eps_1 + square
// towards (-eps_0, -eps_1), and D(eps) = L(-eps) - L(eps).
__device__ __forceinline__ void vertex_values_2p(int32_t a, int32_t b, int32_t c, int32_t d, int k0, int k1, int N0,
                                                 int N1, int32_t* L, int32_t* D) {
    const bool hm0 = k0 >= 1, hp0 = k0 <= N0 - 1, hm1 = k1 >= 1, hp1 = k1 <= N1 - 1;
    const int32_t v = min(min(a, b), min(c, d));
    const int32_t exm = hm0 ? min(a, c) : 0, exp_ = hp0 ? min(b, d) : 0;   // edges towards -x, +x
    const int32_t eym = hm1 ? min(a, b) : 0, eyp = hp1 ? min(c, d) : 0;    // edges towards -y, +y
    const int32_t sa = (hm0 && hm1) ? a : 0, sb = (hp0 && hm1) ? b : 0;
    const int32_t sc = (hm0 && hp1) ? c : 0, sd = (hp0 && hp1) ? d : 0;
    L[0] = v - exm - eym + sa;    // eps = (+, +): the cells towards -x, -y
    L[1] = v - exp_ - eym + sb;   // eps = (-, +)
    L[2] = v - exm - eyp + sc;    // eps = (+, -)
    L[3] = v - exp_ - eyp + sd;   // eps = (-, -)
    D[0] = L[3] - L[0];
    D[1] = L[2] - L[1];
}

// Once per plan: clear the error word, the run counter and the status words.
__global__ void reset_kernel(uint32_t* __restrict__ err, uint64_t* __restrict__ run_ctr, uint64_t* __restrict__ status,
                             int64_t nstatus) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (i == 0) { err[0] = 0u; err[1] = 0u; *run_ctr = 0ull; }
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
        // back off: the polls are uncached loads, and thousands of waiting
        // waves polling at full rate slow down the stores they wait for
        const int naps = spins < 16 ? spins + 1 : 16;
        for (int i = 0; i < naps; ++i) __builtin_amdgcn_s_sleep(2);
    }
}

// Critical values of one tile's vertices (thread tid holds vertices
// vbase + j * kPrecomputeThreads + tid) and the per-(round, wave, list)
// counts of nonzero values in s_cnt; the caller synchronises before reading
// s_cnt.
template <int N>
struct TileValues {
    static constexpr int NC = 1 << N, NO = 1 << (N - 1), NL = NC + NO, J = verts_per_thread(N);
    ImageDesc d;
    int img_id;
    int32_t vals[J][NL];
    int kk[J][kMaxDim];
};

template <int N, int CONS, typename T>
__device__ __forceinline__ void tile_values(const T* __restrict__ pixels, const ImageDesc* __restrict__ descs,
                                            const int32_t* __restrict__ tile_img, int32_t num_images,
                                            int64_t tile, TileValues<N>& tv,
                                            int32_t (*s_cnt)[kPrecomputeThreads / 64][TileValues<N>::NL]) {
    constexpr int NC = TileValues<N>::NC, NO = TileValues<N>::NO, NL = TileValues<N>::NL;
    constexpr int J = TileValues<N>::J;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lo = tile_img[tile];   // the image owning this tile
    tv.d = descs[lo];
    tv.img_id = lo;
    const ImageDesc& d = tv.d;
    const T* __restrict__ img = pixels + d.pixel_offset;
    const int64_t vbase = (tile - d.tile_start) * tile_verts(N);
    const double inv0 = 1.0 / (double)d.V[0];
    const double inv1 = 1.0 / (double)d.V[1];
    const double inv2 = 1.0 / (double)d.V[2];
    bool valid[J];
    // every round's pixel loads are issued before any vertex is classified
    int32_t nb[J][nb_count<N, CONS>()];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        int64_t v = vbase + j * kPrecomputeThreads + tid;
        valid[j] = v < d.nvert;
        // linear vertex index -> coordinates (axis 0 fastest); the last axis
        // takes the final quotient
        uint32_t r0, r1 = 0, r2 = 0;
        const uint32_t q0 = udiv((uint32_t)(valid[j] ? v : 0), (uint32_t)d.V[0], inv0, &r0);
        const uint32_t q1 = N >= 3 ? udiv(q0, (uint32_t)d.V[1], inv1, &r1) : 0u;
        const uint32_t q2 = N >= 4 ? udiv(q1, (uint32_t)d.V[2], inv2, &r2) : 0u;
#pragma unroll
        for (int a = 0; a < kMaxDim; ++a) tv.kk[j][a] = 0;
        tv.kk[j][0] = (int)r0;
        if constexpr (N == 2) {
            tv.kk[j][1] = (int)q0;
        } else if constexpr (N == 3) {
            tv.kk[j][1] = (int)r1;
            tv.kk[j][2] = (int)q1;
        } else {
            tv.kk[j][1] = (int)r1;
            tv.kk[j][2] = (int)r2;
            tv.kk[j][3] = (int)q2;
        }
        if constexpr (N == 2 && CONS == ECT_PRIMAL) {
            // 32-bit offsets from the image base (images hold fewer than 2^31 pixels)
            const int k0 = tv.kk[j][0], k1 = tv.kk[j][1];
            const int c0 = max(k0 - 1, 0), c1 = min(k0, d.dims[0] - 1);
            const int r0 = max(k1 - 1, 0) * d.dims[0], r1 = min(k1, d.dims[1] - 1) * d.dims[0];
            nb[j][0] = px_load(img, (uint32_t)(r0 + c0));
            nb[j][1] = px_load(img, (uint32_t)(r0 + c1));
            nb[j][2] = px_load(img, (uint32_t)(r1 + c0));
            nb[j][3] = px_load(img, (uint32_t)(r1 + c1));
        } else {
            load_neighbourhood<N, CONS, T>(img, d, tv.kk[j], nb[j]);
        }
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
        int32_t L[NC], D[NO];
        if constexpr (N == 2 && CONS == ECT_PRIMAL)
            vertex_values_2p(nb[j][0], nb[j][1], nb[j][2], nb[j][3], tv.kk[j][0], tv.kk[j][1], d.N[0], d.N[1], L, D);
        else
            vertex_values<N, CONS>(nb[j], d, tv.kk[j], L, D);
#pragma unroll
        for (int l = 0; l < NC; ++l) tv.vals[j][l] = valid[j] ? L[l] : 0;
#pragma unroll
        for (int l = 0; l < NO; ++l) tv.vals[j][NC + l] = valid[j] ? D[l] : 0;
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            uint64_t b = __ballot(tv.vals[j][l] != 0);
            if (lane == 0) s_cnt[j][wave][l] = __popcll(b);
        }
    }
}

// Flat variant for plans of at most kFlatTiles tiles: the sum over every
// predecessor's word directly (up to kFlatChunks * 64 of them, all loads of a
// poll in flight together), which saves the group-total round trip of the
// two-level scan.
constexpr int kFlatChunks = 5;
constexpr int64_t kFlatTiles = kFlatChunks * 64 + 1;

template <int NL>
__device__ __forceinline__ bool sum_published_flat(const uint64_t* words, int64_t count, uint64_t parity,
                                                   uint64_t* sums, uint32_t* err) {
    const int lane = threadIdx.x & 63;
    for (int spins = 0;; ++spins) {
        uint64_t wv[kFlatChunks][NL];
#pragma unroll
        for (int c = 0; c < kFlatChunks; ++c)
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                const int64_t i = (int64_t)c * 64 + lane;
                wv[c][l] = i < count ? __hip_atomic_load(words + i * NL + l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                     : (kFlagAggregate | parity);
            }
        bool ready = true;
#pragma unroll
        for (int c = 0; c < kFlatChunks; ++c)
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                const bool ok = (wv[c][l] & kParityBit) == parity && (wv[c][l] & kFlagMask) != 0;
                ready = ready && __ballot(!ok) == 0;
            }
        if (ready) {
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                uint64_t v = 0;
#pragma unroll
                for (int c = 0; c < kFlatChunks; ++c)
                    v += ((int64_t)c * 64 + lane < count) ? (wv[c][l] & kValueMask) : 0ull;
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
        const int naps = spins < 16 ? spins + 1 : 16;
        for (int i = 0; i < naps; ++i) __builtin_amdgcn_s_sleep(2);
    }
}

// Wave 0, lane l < NL: turn list l's counts into exclusive offsets inside the
// tile and return the tile's total for list l (0 elsewhere).
template <int NL, int J>
__device__ __forceinline__ uint64_t tile_offsets(int32_t (*s_cnt)[kPrecomputeThreads / 64][NL]) {
    const int lane = threadIdx.x & 63;
    if (lane >= NL) return 0;
    int32_t cnt = 0;
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
        for (int w = 0; w < kPrecomputeThreads / 64; ++w) {
            int32_t c = s_cnt[j][w][lane];
            s_cnt[j][w][lane] = cnt;
            cnt += c;
        }
    return (uint64_t)cnt;
}

// Write the tile's list entries in vertex order from the list bases s_base
// and the in-tile offsets.
template <int N>
__device__ __forceinline__ void emit_points(const TileValues<N>& tv,
                                            int32_t (*s_cnt)[kPrecomputeThreads / 64][TileValues<N>::NL],
                                            const int64_t* s_base, ListEntry* __restrict__ points,
                                            int64_t capacity) {
    constexpr int NL = TileValues<N>::NL;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < TileValues<N>::J; ++j) {
        const uint32_t code = entry_code(tv.d, tv.kk[j], N);
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const bool nz = tv.vals[j][l] != 0;
            const uint64_t b = __ballot(nz);
            if (nz) {
                const int rank = __popcll(b & ((1ull << lane) - 1ull));
                const int64_t pos_l = s_base[l] + s_cnt[j][wave][l] + rank;
                points[(int64_t)l * capacity + pos_l] = ListEntry{code, tv.vals[j][l]};
            }
        }
    }
}

// Last tile of a compaction launch that buckets a shared hybrid query set
// (wave 0, after its points): wait for the query workgroup's pair counts (a
// bounded wait), build the work list from them and the two ordinary lists'
// sizes (np, lane b holding pair b's; negative if the look-back failed) and
// consume the word so that a later launch without queries cannot see it.
__device__ __forceinline__ void prep_worklist(const QueryPrep& prep, uint64_t* prep_word, int64_t np,
                                              uint32_t* err) {
    const int lane = threadIdx.x & 63;
    bool ok = __ballot(lane < 2 && np < 0) == 0;
    uint64_t w = 0;
    for (int spins = 0;; ++spins) {
        w = __hip_atomic_load(prep_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (w & kFlagAggregate) break;
        if (spins > kLookbackSpinLimit) {
            if (lane == 0) raise_error(err, ECT_DEVERR_LOOKBACK);
            ok = false;
            break;
        }
        const int naps = spins < 16 ? spins + 1 : 16;
        for (int i = 0; i < naps; ++i) __builtin_amdgcn_s_sleep(2);
    }
    const int64_t q = lane == 0 ? (int64_t)(w & 0xFFFFFFull) : (lane == 1 ? (int64_t)((w >> 24) & 0xFFFFFFull) : 0);
    if (ok) {
        worklist_wave(2, q, np, prep.qtile, prep.chunk0, prep.capacity, err, prep.item_off, prep.tile_off,
                      prep.params);
    } else if (lane == 0) {
        prep.params[0] = 0;
        prep.params[1] = 0;
        prep.params[2] = prep.chunk0;
    }
    if (lane == 0) __hip_atomic_store(prep_word, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Single pass, for plans whose tiles all fit on the chip at once (one
// workgroup per tile, all resident): wave 0 of a tile sums the aggregates of
// its predecessors in its group of 64 (level 1), the group's last tile
// publishes the group total, and the totals of the preceding groups complete
// the prefix (level 2).  Every word a tile waits on belongs to a running or
// finished workgroup, so the waits end.
template <int N, int CONS, typename T, bool FLAT>
__global__ void __launch_bounds__(kPrecomputeThreads)
classify_compact(const T* __restrict__ pixels, const ImageDesc* __restrict__ descs,
                 const int32_t* __restrict__ tile_img, int32_t num_images, int64_t num_tiles,
                 uint32_t* __restrict__ err, uint64_t* __restrict__ run_ctr, uint64_t* __restrict__ status,
                 uint64_t* __restrict__ gstatus, int64_t* __restrict__ list_off, ListEntry* __restrict__ points,
                 int64_t capacity, QueryPrep prep, uint64_t* __restrict__ prep_word) {
    constexpr int NL = TileValues<N>::NL;
    constexpr int W = kPrecomputeThreads / 64;
    __shared__ uint64_t s_run;
    // with queries, workgroup 0 sorts them (dispatched first, so that it runs
    // beside the tiles from the start) and the tiles follow
    const bool with_prep = FLAT && N == 2 && prep.vecs != nullptr;
    constexpr int64_t kPrepGroups = 1;
    if constexpr (FLAT && N == 2) {
        // the query workgroup: sort the shared hybrid queries and publish the
        // pair counts in one word (it waits on nothing, so the tiles' waits
        // still end)
        if (with_prep && blockIdx.x == 0) {
            __shared__ int32_t s_pbin[2 * kSubBins];
            __shared__ int32_t s_pw[kPrecomputeThreads / 64], s_ptot[2], s_pstart[2];
            sort_shared_queries<2>(prep.vecs, prep.rows, err, (QRecT<2>*)prep.recs, prep.bcnt, s_pbin, s_pw, s_ptot,
                                   s_pstart);
            if (threadIdx.x == 0)
                __hip_atomic_store(prep_word, kFlagAggregate | (uint64_t)s_ptot[0] | ((uint64_t)s_ptot[1] << 24),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
    }
    __shared__ int32_t s_cnt[TileValues<N>::J][W][NL];   // per (round, wave, list) counts, then offsets
    __shared__ int64_t s_base[NL];
    __shared__ int64_t s_total[NL];   // last tile: list totals (-1: look-back failed)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t tile = (int64_t)blockIdx.x - (with_prep ? kPrepGroups : 0);
    if (tid == 0) s_run = __hip_atomic_load(run_ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    TileValues<N> tv;
    tile_values<N, CONS, T>(pixels, descs, tile_img, num_images, tile, tv, s_cnt);
    __syncthreads();
    const uint64_t run = s_run;
    const uint64_t parity = (run & 1ull) ? kParityBit : 0ull;
    if (wave == 0) {
        const uint64_t agg = tile_offsets<NL, TileValues<N>::J>(s_cnt);
        if (lane < NL)
            __hip_atomic_store(status + tile * NL + lane, kFlagAggregate | parity | agg, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        const int64_t g = tile >> 6, k = tile & 63;
        uint64_t loc[NL], grp[NL];
        bool ok;
        if constexpr (FLAT) {
            // one level: every predecessor's word
            ok = sum_published_flat<NL>(status, tile, parity, loc, err);
#pragma unroll
            for (int l = 0; l < NL; ++l) grp[l] = 0;
            if (tile == num_tiles - 1 && lane == 0)
                __hip_atomic_store(run_ctr, run + 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
        ok = sum_published<NL>(status + (tile - k) * NL, k, parity, loc, err);
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
            __hip_atomic_store(run_ctr, run + 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane < NL) {
            uint64_t mine = 0;
#pragma unroll
            for (int l = 0; l < NL; ++l) if (lane == l) mine = ok ? loc[l] + grp[l] : 0;
            s_base[lane] = (int64_t)mine;
            if (tile == tv.d.tile_start) list_off[(int64_t)tv.img_id * NL + lane] = (int64_t)mine;
            if (tile == num_tiles - 1) {
                list_off[(int64_t)num_images * NL + lane] = (int64_t)(mine + agg);
                s_total[lane] = ok ? (int64_t)(mine + agg) : -1;
            }
        }
    }
    __syncthreads();
    emit_points<N>(tv, s_cnt, s_base, points, capacity);
    // the last tile builds the queries' work list after writing its own
    // points, so that its stores drain while it waits for the query workgroup
    if constexpr (FLAT && N == 2) {
        if (with_prep && tile == num_tiles - 1 && wave == 0)
            prep_worklist(prep, prep_word, s_total[4 + (lane & 1)], err);
    }
}

// Three passes, for plans with more tiles than the chip holds at once (no
// workgroup ever waits on another): count each tile's entries per list,
// scan the counts in tile order, then classify again and write.
template <int N, int CONS, typename T>
__global__ void __launch_bounds__(kPrecomputeThreads)
tile_count_kernel(const T* __restrict__ pixels, const ImageDesc* __restrict__ descs,
                  const int32_t* __restrict__ tile_img, int32_t num_images, int32_t* __restrict__ counts,
                  uint32_t* __restrict__ packed) {
    constexpr int NL = TileValues<N>::NL;
    constexpr int J = TileValues<N>::J;
    __shared__ int32_t s_cnt[J][kPrecomputeThreads / 64][NL];
    const int64_t tile = blockIdx.x;
    TileValues<N> tv;
    tile_values<N, CONS, T>(pixels, descs, tile_img, num_images, tile, tv, s_cnt);
    __syncthreads();
    constexpr int W = kPrecomputeThreads / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (wave == 0 && lane < NL) {
        int32_t tot = 0;
#pragma unroll
        for (int j = 0; j < J; ++j)
#pragma unroll
            for (int w = 0; w < W; ++w) tot += s_cnt[j][w][lane];
        counts[tile * NL + lane] = tot;
    }
    if (!packed) return;
    // the tile's entries in vertex order inside its own slots, packed as
    // value << kPackShift | vertex index in the tile (tile_copy_kernel
    // places them once the offsets are known).  Each wave finds where its
    // rounds start itself: lane j * NL + l sums list l's counts of the rounds
    // and waves before (j, wave).
    static_assert(J * NL <= 64, "one lane per (round, list)");
    int32_t start = 0;
    if (lane < J * NL) {
        const int jj = lane / NL, l = lane % NL;
        for (int j = 0; j < J; ++j)
            for (int w = 0; w < W; ++w)
                if (j < jj || (j == jj && w < wave)) start += s_cnt[j][w][l];
    }
    uint32_t* __restrict__ slots = packed + tile * NL * (int64_t)tile_verts(N);
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const uint32_t local = (uint32_t)(j * kPrecomputeThreads + threadIdx.x);
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const bool nz = tv.vals[j][l] != 0;
            const uint64_t b = __ballot(nz);
            const int32_t st = __shfl(start, j * NL + l, 64);
            if (nz) {
                const int pos = st + __popcll(b & ((1ull << lane) - 1ull));
                slots[l * tile_verts(N) + pos] = ((uint32_t)tv.vals[j][l] << kPackShift) | local;
            }
        }
    }
}

// Two-axis primal images, count pass of three-pass plans.  Same counts and
// packed slots as tile_count_kernel, with the work per vertex cut down: one
// wave per tile, 16 rounds of 64 consecutive vertices (lane l, round j:
// vertex j * 64 + l of the tile).  The pixel rows the tile touches are
// staged once into the wave's part of LDS with dword loads (byte loads of
// four pixels per vertex kept the vector memory pipeline busy for most of
// the pass), unless they exceed it (very wide images read global memory).
// The wave's entries of a list are contiguous in the tile's order, so their
// slots come from the ballot masks (a running scalar count plus the bit count
// below the lane); they collect in LDS and leave in whole-wave stores (see
// flush_entries); the vertex coordinates advance by 64 per round instead of
// a division per vertex; the cell values have their shared subexpressions
// written out (vertex_values_2p).
constexpr int kSpanDwords = 512;   // LDS per wave for the staged pixel rows (2 KiB)

// The wave's packed entries of list l collect in LDS (kEntryBuf per list)
// and go out in whole-wave stores: one store instruction per entry slot kept
// the texture address unit busy for most of the pass.  flush_entries writes
// list l's collected entries to slots at its running count.
constexpr int kEntryBuf = 128;

__device__ __forceinline__ void flush_entries(const uint32_t* buf, uint32_t n, char* __restrict__ slots,
                                              uint32_t at) {
    const int lane = threadIdx.x & 63;
    // entries other lanes of the wave put in LDS
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    for (uint32_t i = (uint32_t)lane; i < n; i += 64u) *(uint32_t*)(slots + (at + i) * 4u) = buf[i];
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
}

// The values of one vertex per lane (k0, k1; `valid` lanes only) and their
// entries: per list, the wave's nonzero entries in lane order are appended to
// the list's LDS buffer (flushed in whole-wave stores when it fills).
template <typename T, bool STAGED>
struct CountCtx {
    const unsigned char* lds;
    const T* __restrict__ img;
    int rlo, rhi, W0, N0, N1;
    char* __restrict__ slots;
    uint32_t* base;
    uint32_t* buf;
    uint32_t buffered[6];

    __device__ __forceinline__ int32_t pix(int rr, int cc) const {
        if constexpr (STAGED) {
            const uint32_t o = __umul24((uint32_t)(rr - rlo), (uint32_t)W0) + (uint32_t)cc;
            return (int32_t)((const T*)lds)[o];
        } else {
            return px_load(img, (uint32_t)(rr * W0 + cc));
        }
    }

    // the four pixels of a vertex star, clamped into the image and into the
    // staged rows (lanes past the last vertex included)
    __device__ __forceinline__ void pixels(int k0, int k1, int32_t& pa, int32_t& pb, int32_t& pc, int32_t& pd) const {
        const int c0 = max(k0 - 1, 0), c1 = min(k0, W0 - 1);
        const int r0 = min(max(k1 - 1, 0), rhi), r1 = min(k1, rhi);
        pa = pix(r0, c0);
        pb = pix(r0, c1);
        pc = pix(r1, c0);
        pd = pix(r1, c1);
    }

    __device__ __forceinline__ void classify(int k0, int k1, bool valid, uint32_t local, int32_t pa, int32_t pb,
                                             int32_t pc, int32_t pd) {
        constexpr int NL = 6;
        int32_t L[4], D[2];
        vertex_values_2p(pa, pb, pc, pd, k0, k1, N0, N1, L, D);
        const int32_t vals[NL] = {L[0], L[1], L[2], L[3], D[0], D[1]};
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const bool nz = valid && vals[l] != 0;
            const uint64_t m = __builtin_amdgcn_ballot_w64(nz);
            if (m != 0) {
                if (slots) {
                    if (buffered[l] + 64u > (uint32_t)kEntryBuf) {
                        flush_entries(buf + l * kEntryBuf, buffered[l], slots, base[l]);
                        base[l] += buffered[l];
                        buffered[l] = 0u;
                    }
                    if (nz) {
                        // buffered + number of the wave's entries on lower lanes
                        const uint32_t pos = __builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, buffered[l]));
                        buf[l * kEntryBuf + pos] = ((uint32_t)vals[l] << kPackShift) | local;
                    }
                    buffered[l] += (uint32_t)__builtin_popcountll(m);
                } else {
                    base[l] += (uint32_t)__builtin_popcountll(m);
                }
            }
        }
    }

    __device__ __forceinline__ void finish() {
        if (slots) {
#pragma unroll
            for (int l = 0; l < 6; ++l) {
                if (buffered[l] != 0u) flush_entries(buf + l * kEntryBuf, buffered[l], slots, base[l]);
                base[l] += buffered[l];
            }
        }
    }
};

// The 16 rounds of one tile; STAGED: pixels from the staged rows in LDS
// (row rr at (rr - rlo) * W0), else from global memory.  base[l]: slots
// written for list l (scalar).  With staged rows, a vertex whose four pixels
// are equal and whose star lies inside the image has only zero values, so a
// round only tests its vertices and queues the others in LDS (in vertex
// order); full waves of queued vertices are then classified, which keeps the
// entries in vertex order and spends the classification on the vertices near
// the edge of a region or of the image.
template <typename T, bool STAGED>
__device__ __forceinline__ void count_rounds_2p(const unsigned char* lds, const T* __restrict__ img, int rlo, int rhi,
                                                int W0, int V0, int N0, int N1, int nv, int q64, int r64, int k0,
                                                int k1, int64_t first, char* __restrict__ slots, uint32_t* base,
                                                uint32_t* buf, uint32_t* queue) {
    constexpr int R = tile_verts(2) / 64;
    const int lane = threadIdx.x & 63;
    CountCtx<T, STAGED> cx{lds, img, rlo, rhi, W0, N0, N1, slots, base, buf, {0u, 0u, 0u, 0u, 0u, 0u}};
    if constexpr (!STAGED) {
#pragma unroll 2
        for (int round = 0; round < R; ++round) {
            const bool valid = round * 64 + lane < nv;
            int32_t pa, pb, pc, pd;
            cx.pixels(k0, k1, pa, pb, pc, pd);
            cx.classify(k0, k1, valid, (uint32_t)(round * 64 + lane), pa, pb, pc, pd);
            k0 += r64;
            k1 += q64;
            if (k0 >= V0) {
                k0 -= V0;
                ++k1;
            }
        }
    } else {
        // queue entry: k0 (21 bits) | k1 - the tile's first row (11 bits);
        // lane 0 holds the tile's first vertex
        const int row0 = __builtin_amdgcn_readfirstlane(k1);
        uint32_t qn = 0;   // queued vertices (uniform, below 64 between rounds)
        auto drain = [&](uint32_t n) {
            // classify queue[0, n) (n <= 64), then move the rest to the front
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            const bool on = (uint32_t)lane < n;
            const uint32_t e = on ? queue[lane] : 0u;
            const int qk0 = (int)(e & 0x1FFFFFu), qk1 = row0 + (int)(e >> 21);
            const uint32_t local = (uint32_t)((int64_t)qk1 * V0 + qk0 - first);
            int32_t pa, pb, pc, pd;
            cx.pixels(qk0, qk1, pa, pb, pc, pd);
            cx.classify(qk0, qk1, on, local, pa, pb, pc, pd);
            const uint32_t rest = qn - n;
            const uint32_t t = (uint32_t)lane < rest ? queue[n + lane] : 0u;
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            if ((uint32_t)lane < rest) queue[lane] = t;
            qn = rest;
        };
        for (int round = 0; round < R; ++round) {
            const bool valid = round * 64 + lane < nv;
            int32_t pa, pb, pc, pd;
            cx.pixels(k0, k1, pa, pb, pc, pd);
            const bool inside = (uint32_t)(k0 - 1) < (uint32_t)(N0 - 1) && (uint32_t)(k1 - 1) < (uint32_t)(N1 - 1);
            const bool flat = pa == pb && pa == pc && pa == pd;
            const bool need = valid && !(inside && flat);
            const uint64_t m = __builtin_amdgcn_ballot_w64(need);
            if (m != 0) {
                if (need) {
                    const uint32_t pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, qn));
                    queue[pos] = (uint32_t)k0 | ((uint32_t)(k1 - row0) << 21);
                }
                qn += (uint32_t)__builtin_popcountll(m);
                if (qn >= 64u) drain(64u);
            }
            k0 += r64;
            k1 += q64;
            if (k0 >= V0) {
                k0 -= V0;
                ++k1;
            }
        }
        if (qn > 0u) drain(qn);
    }
    cx.finish();
}

template <typename T>
__global__ void __launch_bounds__(kPrecomputeThreads)
tile_count_2p_kernel(const T* __restrict__ pixels, const ImageDesc* __restrict__ descs,
                     const int32_t* __restrict__ tile_img, int64_t num_tiles, int32_t* __restrict__ counts,
                     uint32_t* __restrict__ packed) {
    constexpr int NL = 6, R = tile_verts(2) / 64;
    __shared__ uint32_t s_span[kPrecomputeThreads / 64][kSpanDwords];
    __shared__ uint32_t s_ent[kPrecomputeThreads / 64][NL * kEntryBuf];
    __shared__ uint32_t s_queue[kPrecomputeThreads / 64][128];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t tile = (int64_t)blockIdx.x * (kPrecomputeThreads / 64) + wave;
    if (tile >= num_tiles) return;
    const ImageDesc& d = descs[tile_img[tile]];
    const T* __restrict__ img = pixels + d.pixel_offset;
    const int V0 = d.V[0], N0 = d.N[0], N1 = d.N[1], W0 = d.dims[0], H1 = d.dims[1];
    const int64_t first = (tile - d.tile_start) * tile_verts(2);
    // vertices of the tile that exist (the image's last tile is short)
    const int nv = (int)min<int64_t>(d.nvert - first, (int64_t)tile_verts(2));
    const double invV0 = 1.0 / (double)V0;
    uint32_t r;
    const uint32_t q = udiv((uint32_t)(first + lane), (uint32_t)V0, invV0, &r);
    int k0 = (int)r, k1 = (int)q;
    uint32_t r64;
    const int q64 = (int)udiv(64u, (uint32_t)V0, invV0, &r64);
    // pixel rows rlo..rhi hold every pixel of the tile's vertex stars
    uint32_t rdummy;
    const int k1f = (int)(first / V0);
    const int k1l = (int)udiv((uint32_t)(first + nv - 1), (uint32_t)V0, invV0, &rdummy);
    const int rlo = min(max(k1f - 1, 0), H1 - 1), rhi = min(k1l, H1 - 1);
    const int64_t span_lo = (int64_t)rlo * W0 * (int64_t)sizeof(T);
    const int64_t span_hi = ((int64_t)rhi + 1) * W0 * (int64_t)sizeof(T);
    // dword-aligned start of the span (mis bytes before it); offsets are
    // relative to the image's first byte
    const char* __restrict__ ib = (const char*)img;
    const int mis = (int)(((uintptr_t)ib + (uintptr_t)span_lo) & 3u);
    const int64_t o0 = span_lo - mis;
    const int ndw = (int)((span_hi - o0 + 3) >> 2);
    const bool staged = ndw <= kSpanDwords;
    unsigned char* s_bytes = (unsigned char*)s_span[wave];
    if (staged) {
        // dwords wholly inside the span in one load; the partial first and
        // last ones byte by byte (nothing outside the image is read)
        for (int i = lane; i < ndw; i += 64) {
            const int64_t o = o0 + 4 * (int64_t)i;
            uint32_t w;
            if (o >= span_lo && o + 4 <= span_hi) {
                w = *(const uint32_t*)(ib + o);
            } else {
                w = 0u;
                for (int b = 0; b < 4; ++b)
                    if (o + b >= span_lo && o + b < span_hi) w |= (uint32_t)(unsigned char)ib[o + b] << (8 * b);
            }
            s_span[wave][i] = w;
        }
        // the wave's own LDS writes come before its reads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // slots of this tile: 32-bit byte offsets from a uniform base; base[l] is
    // the next free slot of list l (a scalar)
    char* __restrict__ slots = packed ? (char*)(packed + tile * NL * (int64_t)tile_verts(2)) : nullptr;
    uint32_t base[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) base[l] = (uint32_t)(l * tile_verts(2));
    if (staged)
        count_rounds_2p<T, true>(s_bytes + mis, img, rlo, rhi, W0, V0, N0, N1, nv, q64, (int)r64, k0, k1, first,
                                 slots, base, s_ent[wave], s_queue[wave]);
    else
        count_rounds_2p<T, false>(s_bytes, img, rlo, rhi, W0, V0, N0, N1, nv, q64, (int)r64, k0, k1, first, slots,
                                  base, s_ent[wave], s_queue[wave]);
    int32_t c = 0;
#pragma unroll
    for (int l = 0; l < NL; ++l)
        if (lane == l) c = (int32_t)(base[l] - (uint32_t)(l * tile_verts(2)));
    if (lane < NL) counts[tile * NL + lane] = c;
}

// Three-pass plans with packed entries: place tile t's entries (list l's
// count from the count pass, in vertex order) at the list's prefix.  A wave
// takes kCopyTiles consecutive tiles: their counts and list prefixes come in
// with scalar loads, then the slots of every list's first 64 entries of all
// its tiles go out as one batch of loads (lane i: entry i), so the tiles'
// memory round trips overlap; each entry is stored with its vertex
// coordinates decoded from the index.  Entries past the 64th of a list in a
// tile (rare) follow in a loop.
constexpr int kCopyTiles = 2;

template <int N>
__device__ __forceinline__ ListEntry copy_entry(const ImageDesc& d, int64_t vbase, double inv0, double inv1,
                                                double inv2, uint32_t w) {
    const uint32_t v = (uint32_t)(vbase + (w & kPackLocalMask));
    uint32_t r0, r1 = 0, r2 = 0;
    const uint32_t q0 = udiv(v, (uint32_t)d.V[0], inv0, &r0);
    const uint32_t q1 = N >= 3 ? udiv(q0, (uint32_t)d.V[1], inv1, &r1) : 0u;
    const uint32_t q2 = N >= 4 ? udiv(q1, (uint32_t)d.V[2], inv2, &r2) : 0u;
    int k[kMaxDim] = {(int)r0, 0, 0, 0};
    if constexpr (N == 2) {
        k[1] = (int)q0;
    } else if constexpr (N == 3) {
        k[1] = (int)r1;
        k[2] = (int)q1;
    } else {
        k[1] = (int)r1;
        k[2] = (int)r2;
        k[3] = (int)q2;
    }
    return ListEntry{entry_code(d, k, N), (int32_t)w >> kPackShift};
}

template <int N>
__global__ void __launch_bounds__(kPrecomputeThreads)
tile_copy_kernel(const ImageDesc* __restrict__ descs, const int32_t* __restrict__ tile_img, int64_t num_tiles,
                 const int32_t* __restrict__ counts, const int64_t* __restrict__ prefix,
                 const uint32_t* __restrict__ packed, ListEntry* __restrict__ points, int64_t capacity) {
    constexpr int NL = TileValues<N>::NL;
    constexpr int TV = tile_verts(N);
    const int lane = threadIdx.x & 63;
    const int64_t t0 =
        ((int64_t)blockIdx.x * (kPrecomputeThreads / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) *
        kCopyTiles;
    if (t0 >= num_tiles) return;
    int32_t cnt[kCopyTiles][NL];
    int64_t pre[kCopyTiles][NL];
#pragma unroll
    for (int j = 0; j < kCopyTiles; ++j) {
        const bool ok = t0 + j < num_tiles;
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            cnt[j][l] = ok ? counts[(t0 + j) * NL + l] : 0;
            pre[j][l] = ok ? prefix[(t0 + j) * NL + l] : 0;
        }
    }
    uint32_t w[kCopyTiles][NL];
#pragma unroll
    for (int j = 0; j < kCopyTiles; ++j) {
        const uint32_t* __restrict__ slots = packed + (t0 + j) * NL * (int64_t)TV;
#pragma unroll
        for (int l = 0; l < NL; ++l) w[j][l] = lane < cnt[j][l] ? slots[l * TV + lane] : 0u;
    }
#pragma unroll
    for (int j = 0; j < kCopyTiles; ++j) {
        const int64_t tile = t0 + j;
        if (tile >= num_tiles) break;
        const ImageDesc& d = descs[tile_img[tile]];
        const int64_t vbase = (tile - d.tile_start) * TV;
        const double inv0 = 1.0 / (double)d.V[0], inv1 = 1.0 / (double)d.V[1], inv2 = 1.0 / (double)d.V[2];
        const uint32_t* __restrict__ slots = packed + tile * NL * (int64_t)TV;
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            ListEntry* __restrict__ out = points + (int64_t)l * capacity + pre[j][l];
            if (lane < cnt[j][l]) out[lane] = copy_entry<N>(d, vbase, inv0, inv1, inv2, w[j][l]);
            for (int pos = 64 + lane; pos < cnt[j][l]; pos += 64)
                out[pos] = copy_entry<N>(d, vbase, inv0, inv1, inv2, slots[l * TV + pos]);
        }
    }
}

// Exclusive prefix of the tile counts of every list in tile order (64-bit),
// in three coalesced launches over blocks of kScanTiles tiles: block sums,
// one workgroup scanning the block sums, and per-block scans that add the
// block's base, write the prefixes and the list offsets of the images whose
// first tile lies in the block.
constexpr int kScanTiles = 1024;

// Inclusive scan over a 1024-thread workgroup of one value per thread and
// channel (wave shuffles; one thread per channel scans the 16 wave totals in
// LDS); the channel totals go to s_tot.  A block covers kScanTiles tiles of
// at most tile_verts(n) <= 1024 entries per list, so in-block values fit in
// 32 bits and every channel goes in one pass; callers add 64-bit bases.
template <int NL>
__device__ __forceinline__ void block_scan_channels(int32_t (&v)[NL], int32_t (*s_w)[NL], int32_t* s_tot) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int l = 0; l < NL; ++l) {
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t o = __shfl_up(v[l], off, 64);
            if (lane >= off) v[l] += o;
        }
        if (lane == 63) s_w[wave][l] = v[l];
    }
    __syncthreads();
    // thread l: exclusive prefix of the 16 wave totals of channel l, in place
    if ((int)threadIdx.x < NL) {
        int32_t run = 0;
        for (int w = 0; w < 16; ++w) {
            const int32_t c = s_w[w][threadIdx.x];
            s_w[w][threadIdx.x] = run;
            run += c;
        }
        s_tot[threadIdx.x] = run;
    }
    __syncthreads();
#pragma unroll
    for (int l = 0; l < NL; ++l) v[l] += s_w[wave][l];
}

// Per-block sums of the tile counts (a reduction per list).
template <int NL>
__global__ void __launch_bounds__(1024)
tile_block_sum_kernel(const int32_t* __restrict__ counts, int64_t num_tiles, int64_t* __restrict__ blk) {
    __shared__ int32_t s_w[16][NL];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t t = (int64_t)blockIdx.x * kScanTiles + threadIdx.x;
    int32_t v[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) v[l] = t < num_tiles ? counts[t * NL + l] : 0;
#pragma unroll
    for (int l = 0; l < NL; ++l) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[l] += __shfl_xor(v[l], off, 64);
        if (lane == 0) s_w[wave][l] = v[l];
    }
    __syncthreads();
    if ((int)threadIdx.x < NL) {
        int64_t sum = 0;
        for (int w = 0; w < 16; ++w) sum += s_w[w][threadIdx.x];
        blk[(int64_t)blockIdx.x * NL + threadIdx.x] = sum;
    }
}

// One workgroup: exclusive scan of the block sums, in place; the grand totals
// close the list offsets.
template <int NL>
__global__ void __launch_bounds__(1024)
tile_block_scan_kernel(int64_t* __restrict__ blk, int64_t nblk, int32_t num_images, int64_t* __restrict__ list_off) {
    __shared__ int32_t s_w[16][NL];
    __shared__ int32_t s_tot[NL];
    __shared__ int64_t s_carry[NL];
    if ((int)threadIdx.x < NL) s_carry[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t base = 0; base < nblk; base += 1024) {
        const int64_t b = base + threadIdx.x;
        int32_t v[NL], x[NL];
#pragma unroll
        for (int l = 0; l < NL; ++l) x[l] = v[l] = b < nblk ? (int32_t)blk[b * NL + l] : 0;
        block_scan_channels<NL>(v, s_w, s_tot);
        if (b < nblk)
#pragma unroll
            for (int l = 0; l < NL; ++l) blk[b * NL + l] = s_carry[l] + (int64_t)(v[l] - x[l]);
        __syncthreads();
        if ((int)threadIdx.x < NL) s_carry[threadIdx.x] += s_tot[threadIdx.x];
        __syncthreads();
    }
    if ((int)threadIdx.x < NL) list_off[(int64_t)num_images * NL + threadIdx.x] = s_carry[threadIdx.x];
}

// Per-block scans plus the block's base: the tile prefixes, and the list
// offsets of every image whose first tile is one of the block's tiles.
template <int NL>
__global__ void __launch_bounds__(1024)
tile_block_apply_kernel(const int32_t* __restrict__ counts, int64_t num_tiles, const int64_t* __restrict__ blk,
                        const int64_t* __restrict__ tile_start, int32_t num_images, int64_t* __restrict__ prefix,
                        int64_t* __restrict__ list_off) {
    __shared__ int32_t s_w[16][NL];
    __shared__ int32_t s_tot[NL];
    const int64_t t = (int64_t)blockIdx.x * kScanTiles + threadIdx.x;
    int32_t v[NL], x[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) x[l] = v[l] = t < num_tiles ? counts[t * NL + l] : 0;
    // the image (if any) whose first tile is t; tile starts strictly increase
    int lo = 0, hi = num_images;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (tile_start[mid] < t) lo = mid + 1; else hi = mid;
    }
    const bool first = t < num_tiles && lo < num_images && tile_start[lo] == t;
    block_scan_channels<NL>(v, s_w, s_tot);
    if (t < num_tiles) {
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const int64_t p = blk[(int64_t)blockIdx.x * NL + l] + (int64_t)(v[l] - x[l]);
            prefix[t * NL + l] = p;
            if (first) list_off[(int64_t)lo * NL + l] = p;
        }
    }
}

template <int N, int CONS, typename T>
__global__ void __launch_bounds__(kPrecomputeThreads)
tile_write_kernel(const T* __restrict__ pixels, const ImageDesc* __restrict__ descs,
                  const int32_t* __restrict__ tile_img, int32_t num_images, const int64_t* __restrict__ prefix,
                  ListEntry* __restrict__ points, int64_t capacity) {
    constexpr int NL = TileValues<N>::NL;
    __shared__ int32_t s_cnt[TileValues<N>::J][kPrecomputeThreads / 64][NL];
    __shared__ int64_t s_base[NL];
    const int64_t tile = blockIdx.x;
    TileValues<N> tv;
    tile_values<N, CONS, T>(pixels, descs, tile_img, num_images, tile, tv, s_cnt);
    if (threadIdx.x < NL) s_base[threadIdx.x] = prefix[tile * NL + threadIdx.x];
    __syncthreads();
    if ((threadIdx.x >> 6) == 0) tile_offsets<NL, TileValues<N>::J>(s_cnt);
    __syncthreads();
    emit_points<N>(tv, s_cnt, s_base, points, capacity);
}

template <int N, int CONS, typename T>
hipError_t launch_typed(const Plan& p, bool first, hipStream_t stream, const QueryPrep* prep) {
    const PlanLayout& L = p.lay;
    const int NL = num_lists(N);
    uint32_t* err = (uint32_t*)(p.ws + L.err);
    uint64_t* run_ctr = (uint64_t*)(p.ws + L.err + 8);
    uint64_t* status = (uint64_t*)(p.ws + L.status);
    uint64_t* gstatus = status + L.num_tiles * NL;   // [ceil(tiles / 64)][NL] group totals
    // tile words, group totals, and one row whose first word carries the
    // query workgroup's pair counts
    const int64_t nstatus = (L.num_tiles + (L.num_tiles + 63) / 64 + 1) * NL;
    uint64_t* prep_word = status + (L.num_tiles + (L.num_tiles + 63) / 64) * NL;
    const QueryPrep qp = prep ? *prep : QueryPrep{};
    const bool single = L.num_tiles <= p.precompute_grid;
    hipError_t e = hipSuccess;
    if (first && single) {
        int rblocks = (int)std::min<int64_t>((nstatus + 255) / 256 + 1, 4096);
        hipLaunchKernelGGL(reset_kernel, dim3(rblocks), dim3(256), 0, stream, err, run_ctr, status, nstatus);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    e = stage_mark(ECT_STAGE_PRECOMPUTE, false, stream);
    if (e != hipSuccess) return e;
    const T* px = (const T*)p.pixels;
    const ImageDesc* desc = (const ImageDesc*)(p.ws + L.desc);
    const int64_t* ts = (const int64_t*)(p.ws + L.tile_start);
    const int32_t* ti = (const int32_t*)(p.ws + L.tile_img);
    int64_t* lo = (int64_t*)(p.ws + L.list_off);
    ListEntry* pts = (ListEntry*)(p.ws + L.points);
    if (single) {
        if (N == 2 && L.num_tiles <= kFlatTiles && L.num_tiles <= p.precompute_grid_flat) {
            // one more workgroup when it buckets the queries (the caller checked that it fits)
            const int64_t grid = L.num_tiles + (qp.vecs ? 1 : 0);
            hipLaunchKernelGGL((classify_compact<N, CONS, T, true>), dim3((unsigned)grid), dim3(kPrecomputeThreads),
                               0, stream, px, desc, ti, p.num_images, L.num_tiles, err, run_ctr, status, gstatus, lo,
                               pts, L.capacity, qp, prep_word);
        } else {
            hipLaunchKernelGGL((classify_compact<N, CONS, T, false>), dim3((unsigned)L.num_tiles),
                               dim3(kPrecomputeThreads), 0, stream, px, desc, ti, p.num_images, L.num_tiles, err,
                               run_ctr, status, gstatus, lo, pts, L.capacity, QueryPrep{}, prep_word);
        }
    } else {
        // the status region holds the counts (int32), the prefixes (int64) and
        // the block sums (int64)
        int32_t* counts = (int32_t*)status;
        int64_t* prefix = (int64_t*)(p.ws + L.status) + (L.num_tiles * NL + 1) / 2;
        int64_t* blk = prefix + L.num_tiles * NL;
        const int64_t nblk = (L.num_tiles + kScanTiles - 1) / kScanTiles;
        if (first) {
            // first use of the error word by this plan
            hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, stream, err, run_ctr, status, (int64_t)0);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        // packed entries (small pixel types only: their values fit the packed field)
        uint32_t* packed = (L.packed_bytes > 0 && sizeof(T) < 4) ? (uint32_t*)(p.ws + L.packed) : nullptr;
        if constexpr (N == 2 && CONS == ECT_PRIMAL)
            hipLaunchKernelGGL((tile_count_2p_kernel<T>),
                               dim3((unsigned)((L.num_tiles + kPrecomputeThreads / 64 - 1) / (kPrecomputeThreads / 64))),
                               dim3(kPrecomputeThreads), 0, stream, px, desc, ti, L.num_tiles, counts, packed);
        else
            hipLaunchKernelGGL((tile_count_kernel<N, CONS, T>), dim3((unsigned)L.num_tiles), dim3(kPrecomputeThreads),
                               0, stream, px, desc, ti, p.num_images, counts, packed);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        constexpr int NLc = TileValues<N>::NL;
        hipLaunchKernelGGL(tile_block_sum_kernel<NLc>, dim3((unsigned)nblk), dim3(1024), 0, stream, counts,
                           L.num_tiles, blk);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(tile_block_scan_kernel<NLc>, dim3(1), dim3(1024), 0, stream, blk, nblk, p.num_images, lo);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(tile_block_apply_kernel<NLc>, dim3((unsigned)nblk), dim3(1024), 0, stream, counts,
                           L.num_tiles, blk, ts, p.num_images, prefix, lo);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (packed)
            hipLaunchKernelGGL((tile_copy_kernel<N>),
                               dim3((unsigned)((L.num_tiles + kCopyTiles * (kPrecomputeThreads / 64) - 1) /
                                               (kCopyTiles * (kPrecomputeThreads / 64)))),
                               dim3(kPrecomputeThreads), 0, stream, desc, ti, L.num_tiles, counts, prefix, packed, pts,
                               L.capacity);
        else
            hipLaunchKernelGGL((tile_write_kernel<N, CONS, T>), dim3((unsigned)L.num_tiles), dim3(kPrecomputeThreads),
                               0, stream, px, desc, ti, p.num_images, prefix, pts, L.capacity);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return stage_mark(ECT_STAGE_PRECOMPUTE, true, stream);
}

template <int N, int CONS, typename T>
int64_t slots_typed(bool flat) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu,
                                                     flat ? classify_compact<N, CONS, T, true>
                                                          : classify_compact<N, CONS, T, false>,
                                                     kPrecomputeThreads, 0) !=
        hipSuccess)
        return 0;
    return per_cu;
}

template <int N, int CONS>
hipError_t launch_dtype(const Plan& p, bool first, hipStream_t s, const QueryPrep* prep) {
    switch (p.dtype) {
        case ECT_U8: return launch_typed<N, CONS, uint8_t>(p, first, s, prep);
        case ECT_I16: return launch_typed<N, CONS, int16_t>(p, first, s, prep);
        default: return launch_typed<N, CONS, int32_t>(p, first, s, prep);
    }
}

}  // namespace

int64_t precompute_slots_per_cu(int ndim, int construction, int dtype, bool flat) {
    auto pick = [&](auto n, auto c) -> int64_t {
        constexpr int N = decltype(n)::value, C = decltype(c)::value;
        switch (dtype) {
            case ECT_U8: return slots_typed<N, C, uint8_t>(flat);
            case ECT_I16: return slots_typed<N, C, int16_t>(flat);
            default: return slots_typed<N, C, int32_t>(flat);
        }
    };
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    using I4 = std::integral_constant<int, 4>;
    using P = std::integral_constant<int, ECT_PRIMAL>;
    using Du = std::integral_constant<int, ECT_DUAL>;
    if (ndim == 2) return construction == ECT_PRIMAL ? pick(I2{}, P{}) : pick(I2{}, Du{});
    if (ndim == 3) return construction == ECT_PRIMAL ? pick(I3{}, P{}) : pick(I3{}, Du{});
    return construction == ECT_PRIMAL ? pick(I4{}, P{}) : pick(I4{}, Du{});
}

bool precompute_takes_queries(const Plan& p) {
    const PlanLayout& L = p.lay;
    // the tiles and the query workgroup all resident at once
    return p.ndim == 2 && p.num_images == 1 && L.num_tiles <= p.precompute_grid &&
           L.num_tiles + 1 <= kFlatTiles && L.num_tiles + 1 <= p.precompute_grid_flat;
}

hipError_t launch_precompute(const Plan& p, bool first, hipStream_t stream, const QueryPrep* prep) {
    if (prep && prep->vecs && !precompute_takes_queries(p)) return hipErrorInvalidValue;
    if (p.ndim == 2)
        return p.construction == ECT_PRIMAL ? launch_dtype<2, ECT_PRIMAL>(p, first, stream, prep)
                                            : launch_dtype<2, ECT_DUAL>(p, first, stream, prep);
    if (p.ndim == 3)
        return p.construction == ECT_PRIMAL ? launch_dtype<3, ECT_PRIMAL>(p, first, stream, prep)
                                            : launch_dtype<3, ECT_DUAL>(p, first, stream, prep);
    return p.construction == ECT_PRIMAL ? launch_dtype<4, ECT_PRIMAL>(p, first, stream, prep)
                                        : launch_dtype<4, ECT_DUAL>(p, first, stream, prep);
}

}  // namespace ect
