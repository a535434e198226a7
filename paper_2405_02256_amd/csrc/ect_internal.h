// Internal definitions shared by the host plan code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ect.h"

namespace ect {

constexpr int kMaxDim = 4;
constexpr int kPrecomputeThreads = 256;              // threads per precompute workgroup
// Packed list entry of a three-pass plan: critical value << kPackShift | vertex
// index in its tile (< 1024).  8- and 16-bit pixels bound |value| by
// 2 * 2^n * 32767 < 2^21, so the value keeps its sign in the upper 22 bits.
constexpr int kPackShift = 10;
constexpr uint32_t kPackLocalMask = (1u << kPackShift) - 1u;
constexpr int64_t kPackedMaxBytes = (int64_t)8 << 30;   // larger plans classify again instead
// Vertices per thread per precompute tile: four for n <= 3 (their loads in
// flight together); one for n = 4, whose 81-cell stars and 24 lists fill the
// registers on their own.
__host__ __device__ constexpr int verts_per_thread(int n) { return n == 4 ? 1 : 4; }
__host__ __device__ constexpr int tile_verts(int n) { return kPrecomputeThreads * verts_per_thread(n); }
constexpr int kMaxLists = 24;                        // 2^n classical + 2^(n-1) ordinary, n = 4

__host__ __device__ constexpr int num_classical(int n) { return 1 << n; }
__host__ __device__ constexpr int num_ordinary(int n) { return 1 << (n - 1); }
__host__ __device__ constexpr int num_lists(int n) { return num_classical(n) + num_ordinary(n); }

// One critical point as the evaluation kernels use it (in registers and
// LDS): canonical FP64 vertex coordinates (x_a = fma(h_a, k_a, o_a); unused
// axes 0) and its critical value.
struct alignas(32) Point {
    double x[3];
    double val;
};
struct alignas(16) Point4 {
    double x[4];
    double val;
    double pad;
};
template <int N> struct PointSel { using type = Point; };
template <> struct PointSel<4> { using type = Point4; };
template <int N> using PointT = typename PointSel<N>::type;

// One critical point as the lists store it: the vertex index k packed into
// one 32-bit word (axis a in the bit field of width kbits[a] at kshift[a],
// the same fields for every image of a plan) and the critical value.  The
// coordinates are rebuilt with the canonical fma when a kernel stages the
// point, so the evaluation sees exactly the FP64 values a full record would
// hold, from a quarter of the bytes.
struct alignas(8) ListEntry {
    uint32_t code;
    int32_t val;
};
inline size_t entry_bytes() { return sizeof(ListEntry); }

// The entries of list l (lists are regions of `capacity` entries).
__host__ __device__ __forceinline__ const ListEntry* list_entries(const void* base, int64_t capacity, int64_t l) {
    return (const ListEntry*)base + l * capacity;
}

// Per-image constants, uploaded once per plan.
struct alignas(16) ImageDesc {
    int64_t pixel_offset;   // element offset of the image in the pixel buffer
    int64_t nvert;          // number of vertices
    int64_t tile_start;     // first precompute tile of this image
    int32_t dims[kMaxDim];  // pixels per axis (1 for unused axes)
    int32_t N[kMaxDim];     // top cells per axis
    int32_t V[kMaxDim];     // vertices per axis (N + 1)
    uint32_t kshift[kMaxDim];   // list entries: bit offset of axis a's vertex index
    uint32_t kmask[kMaxDim];    // and its mask (0 for unused axes)
    double origin[kMaxDim];
    double spacing[kMaxDim];
    double lo[kMaxDim], hi[kMaxDim];   // vertex coordinate range per axis (lo <= hi)
};

// Packed vertex index of an entry (k_a < 2^kbits[a]).
__host__ __device__ __forceinline__ uint32_t entry_code(const ImageDesc& d, const int* k, int n) {
    uint32_t c = 0;
    for (int a = 0; a < n; ++a) c |= (uint32_t)k[a] << d.kshift[a];
    return c;
}

// The point of an entry: vertex index from the bit fields, canonical FP64
// coordinates (the same fma as everywhere else), value.
template <int N>
__device__ __forceinline__ PointT<N> decode_entry(const ListEntry e, const ImageDesc& d) {
    PointT<N> p{};
#pragma unroll
    for (int a = 0; a < N; ++a) {
        const uint32_t k = (e.code >> d.kshift[a]) & d.kmask[a];
        p.x[a] = __fma_rn(d.spacing[a], (double)k, d.origin[a]);
    }
    p.val = (double)e.val;
    return p;
}

// Layout of the precompute workspace (byte offsets from its base).
struct PlanLayout {
    size_t err;             // uint32 device error word, uint32 spare, uint64 run counter
    size_t desc;            // ImageDesc[num_images]
    size_t tile_start;      // int64[num_images + 1]
    size_t tile_img;        // int32[num_tiles]: the image each precompute tile belongs to
    size_t list_off;        // int64[(num_images + 1) * NL]: start of image i in list l
    size_t status;          // uint64 ordered-compaction status words: tiles, group totals, carries (x NL)
    size_t points;          // ListEntry[NL * capacity]
    size_t packed;          // uint32[num_tiles * NL * tile_verts]: three-pass plans of 8/16-bit pixels
    size_t packed_bytes;    // 0: no packed region (the write pass classifies again)
    size_t total;
    int64_t num_tiles;
    int64_t capacity;       // entries per list region (= total vertices)
};

}  // namespace ect

// Host handle behind ect_plan.
struct ect_plan_s {
    int32_t ndim = 0;
    int32_t num_images = 0;
    int32_t dtype = 0;
    int32_t construction = 0;
    int32_t num_cus = 0;                    // compute units of the plan's device
    int32_t device = -1;                    // HIP device current at ect_precompute
    int64_t precompute_grid = 1;            // tiles the single-pass compaction handles (all resident)
    int64_t precompute_grid_flat = 0;       // the same for its one-level variant (n = 2, small plans)
    const void* pixels = nullptr;
    char* ws = nullptr;
    ect::PlanLayout lay{};
    ect::ImageDesc* h_desc = nullptr;   // host copy
    int64_t* h_list_off = nullptr;      // host copy [(num_images+1) * NL], as of the last ect_precompute
    int64_t total_verts = 0;
    int64_t max_image_verts = 0;
    // bumped by every call that can change list sizes or the work-list shape
    // (ect_plan_rerun, ect_plan_set_tuning)
    uint64_t lists_epoch = 0;
    // the hybrid query buckets and work list last written into a workspace
    struct {
        const void* ws = nullptr;
        const double* vecs = nullptr;
        const int64_t* offsets = nullptr;
        int64_t count = 0;
        uint64_t epoch = 0;
        bool valid = false;
        bool ahead = false;   // written by ect_plan_rerun_prepare, not used by an evaluation yet
    } last_prep;
    int64_t tune_hybrid_chunk = 0;          // 0: automatic
    int64_t tune_hybrid_target_items = 2048;
    int32_t tune_ect_dirs_per_group = 0;    // 0: automatic
    int32_t tune_ect_chunks = 0;            // 0: automatic
};

namespace ect {

using Plan = ::ect_plan_s;

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Device error word helpers.
__device__ inline void raise_error(uint32_t* err, uint32_t bits) {
    __hip_atomic_fetch_or(err, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sign-vector index of a direction: bit a set iff !(xi_a >= 0).
template <int N>
__device__ __forceinline__ int sign_index(const double* xi) {
    int e = 0;
#pragma unroll
    for (int a = 0; a < N; ++a) e |= (xi[a] >= 0.0) ? 0 : (1 << a);
    return e;
}

// Canonical FP64 projection u = fma(xi_{n-1}, x_{n-1}, ... fma(xi_1, x_1, xi_0*x_0)).
template <int N>
__device__ __forceinline__ double project(const double* xi, const double* x) {
    double u = __dmul_rn(xi[0], x[0]);
#pragma unroll
    for (int a = 1; a < N; ++a) u = __fma_rn(xi[a], x[a], u);
    return u;
}

// Optional profiling events around the main kernel of each stage.
struct StageEvents {
    hipEvent_t before = nullptr, after = nullptr;
};
extern StageEvents g_stage_events[4];
inline hipError_t stage_mark(int stage, bool after, hipStream_t s) {
    hipEvent_t e = after ? g_stage_events[stage].after : g_stage_events[stage].before;
    return e ? hipEventRecord(e, s) : hipSuccess;
}

// Kernel launch helpers (host side, defined in the .hip files).
// first: also clear the plan's error word, ticket counter and look-back words
// (plan creation); re-runs launch the classification kernel alone.
// A shared hybrid query set bucketed inside the compaction launch (two-axis,
// single-image plans of the one-level look-back): one extra workgroup sorts
// the queries (records, pair counts) and publishes the pair counts in one
// word; the last tile builds the work list from them and the list totals.
struct QueryPrep {
    const double* vecs = nullptr;   // null: no queries
    int64_t rows = 0;
    void* recs = nullptr;
    int32_t* bcnt = nullptr;
    int qtile = 0;
    int64_t chunk0 = 0, capacity = 0;
    int64_t* item_off = nullptr;
    int64_t* tile_off = nullptr;
    int64_t* params = nullptr;
};

hipError_t launch_precompute(const Plan& p, bool first, hipStream_t stream, const QueryPrep* prep = nullptr);
// Whether launch_precompute can take a QueryPrep for this plan.
bool precompute_takes_queries(const Plan& p);
// Compaction workgroups one compute unit holds at once (0 if unknown); flat:
// the one-level look-back variant.
int64_t precompute_slots_per_cu(int ndim, int construction, int dtype, bool flat = false);

}  // namespace ect
