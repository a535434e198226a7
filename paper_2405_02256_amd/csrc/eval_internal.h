// Internal declarations of the evaluation stages (bucketing, work lists, ECT,
// hybrid transforms).
#pragma once

#include "ect_internal.h"

namespace ect {

constexpr int kBucketThreads = 256;

// A query in bucket order: its vector (unused axes 0) and code = 2 * row + negated,
// where row is relative to the image's first query row and `negated` marks a
// query evaluated on the mirrored list of its orthant pair.
struct alignas(32) QRec {
    double v[3];
    int64_t code;
};
struct alignas(16) QRec4 {
    double v[4];
    int64_t code;
    int64_t pad;
};
template <int N> struct QRecSel { using type = QRec; };
template <> struct QRecSel<4> { using type = QRec4; };
template <int N> using QRecT = typename QRecSel<N>::type;

inline size_t qrec_bytes(int ndim) { return ndim == 4 ? sizeof(QRec4) : sizeof(QRec); }
constexpr int kEctThreads = 256;      // ECT workgroup: points stream across its lanes
constexpr int kEctWideThreads = 512;  // shared-set ECT workgroup when the launch has few of them
constexpr int kEctMaxDirs = 8;        // directions per ECT workgroup
constexpr int kComboEctDirs = 2;      // at most this many in the combined ECT + hybrid launch
constexpr size_t kComboEctLds = 4096; // and at most this much dynamic LDS (thresholds + histograms)
constexpr int kEctMaxThresholds = 4096;
constexpr int kHybridThreads = 256;  // four waves share one staged chunk of points
constexpr int kHybridSplit = 4;      // the waves split the chunk's points between them ...
constexpr int kHybridTile = kHybridThreads / kHybridSplit;  // ... for one tile of 64 queries
constexpr int kHybridStage = 256;    // points staged in LDS at a time

constexpr int64_t kSmallMaxRows = 65536;   // query sets bucketed by a single workgroup
constexpr int kSmallMaxEntries = 4096;     // (image, bucket) entries counted in LDS there

// Bucket the queries by sign vector and build the work list (one launch for
// small sets; fill + bucket + work list otherwise).  item_off == nullptr:
// buckets only (ECT sets, not the hybrid path's shared-set kernel).
hipError_t launch_prepare(int ndim, const ect_query_set& qs, int num_images, bool hybrid, uint32_t* err,
                          void* recs, int32_t* bcnt, const int64_t* list_off, int list_base, int NL, int qtile,
                          int64_t chunk, int64_t capacity, int64_t* item_off, int64_t* tile_off, int64_t* params,
                          hipStream_t stream);

// First record slot of bucket b of image img (see queries.hip).
__device__ __forceinline__ int64_t bucket_start(const int64_t* offsets, int64_t count, int64_t img, int B, int b) {
    if (!offsets) return (int64_t)b * count;
    const int64_t r0 = offsets[img];
    return (int64_t)B * r0 + (int64_t)b * (offsets[img + 1] - r0);
}

struct EctArgs {
    const void* points;       // ListEntry records
    const int64_t* list_off;
    const ImageDesc* desc;
    int64_t capacity;
    int num_images;
    int NL;
    const double* vecs;
    const int64_t* offsets;   // device or null
    int64_t count;
    const double* thresholds;
    int M;
    int thr_per_image;
    int32_t* out;
    const void* recs;         // QRecT<n> records
    const int32_t* bcnt;
    const int64_t* item_off;
    uint32_t* err;
    int dirs_per_group;
    int64_t chunks;           // shared sets: point chunks per direction group (1: no split)
    int32_t* part;            // shared sets with chunks > 1: per-chunk histograms
    int threads;              // workgroup size of the threshold kernels: 64, kEctThreads, or
                              // kEctWideThreads (shared sets only)
};

// Mean classical list length up to which one-wave workgroups evaluate the ECT.
constexpr double kEctSmallList = 2048.0;

// Shared direction sets over many images with short lists (ect_batch_kernel):
// one workgroup per (image, sign vector) after the set was bucketed once.
constexpr int kBatchThreads = 256;
constexpr int kBatchDirs = 16;          // directions of a bucket per pass
constexpr int kBatchMaxThresholds = 256;
// Dynamic LDS of ect_batch_kernel: the thresholds between two sentinels, then
// (16-byte aligned) the histograms of one pass, rows at an odd stride.
__host__ __device__ constexpr size_t batch_hist_offset(int M) {
    return (sizeof(double) * (size_t)(M + 2) + 15) / 16 * 16;
}
// (a row has M + 1 bins, the last one catching projections above every threshold)
__host__ __device__ constexpr int batch_row_stride(int M) { return (M + 1) | 1; }
__host__ __device__ constexpr size_t batch_ect_lds(int M) {
    return batch_hist_offset(M) + sizeof(int32_t) * (size_t)kBatchDirs * (size_t)batch_row_stride(M);
}
// a.recs / a.bcnt hold the shared set bucketed by sign vector (launch_prepare).
hipError_t launch_ect_batch(int ndim, const EctArgs& a, hipStream_t stream);

// direct_groups > 0: shared query set, num_images * direct_groups * a.chunks
// workgroups of ect_direct_kernel (no bucketing), then, with a.chunks > 1, the
// in-order sum of the chunk histograms; else the bucketed kernel.
// radon: the Radon transform at the thresholds instead of the ECT (same grid).
hipError_t launch_ect(int ndim, const EctArgs& a, int64_t grid, int64_t direct_groups, bool radon,
                      hipStream_t stream);

constexpr int kJi0SmallCoeffs = 10;   // FP32-path small-argument Ji0 polynomial

struct HybridArgs {
    const void* points;       // ListEntry records
    const int64_t* list_off;
    const ImageDesc* desc;
    int64_t capacity;
    int num_images;
    int NL;
    int list_base;            // index of the first ordinary list
    const double* vecs;
    const int64_t* offsets;
    int64_t count;
    double s;
    const double* s_dev;      // device scale (read by the kernels instead of s) or null
    double* out_f;            // Fourier [rows][2]
    double* out_l;            // Laplace [rows]
    double* out_b;            // Bessel [rows]
    double* log_scale;        // Laplace log-scale [rows] or null
    const double* fwd_out;    // backward: forward output of the kernel
    const double* grad_out;   // backward
    double* grad_xi;          // backward: [rows][n] (ragged) or per-image partial [images][count][n]
    double* grad_s_part;      // backward: per-row contribution to d/ds
    const void* recs;         // QRecT<n> records
    const int32_t* bcnt;
    const int64_t* item_off;
    const int64_t* tile_off;
    const int64_t* params;    // [0] items, [1] tiles, [2] chunk
    double* partials;
    int32_t* tile_ent;        // per query tile: its work-list entry if split into chunks, else -1
    uint32_t* err;
    double ji0c[kJi0SmallCoeffs];   // filled at launch (kernel arguments live in scalar registers)
};

// Mask of the s = 0 pass: HT_0 = sum over ordinary points of D <xi, x> (the
// constant kernel kappa(0) = 1 with primitive t), written to every output
// pointer that is set (Fourier: real part, imaginary part 0).
constexpr unsigned kHybridLinear = 8;

// Main kernel (grid work items) then, for multi-chunk tiles, the in-order
// reduction (tiles work groups).  mask: bit k = ect_kernel k (backward: one
// bit), or kHybridLinear.
hipError_t launch_hybrid(int ndim, unsigned mask, int precision, bool backward, const HybridArgs& a,
                         int64_t grid, int64_t tiles, hipStream_t stream);
hipError_t launch_grad_reduce(int ndim, const double* part, int num_images, int64_t count, bool shared,
                              double* grad_xi, const double* gs_part, int64_t rows, double* grad_s,
                              hipStream_t stream);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t stream);

// The shared-set ECT (ect_blocks = groups * chunks direct workgroups) and a
// forward hybrid pass (grid work items) in one launch; the chunk sums of the
// ECT (e.chunks > 1) and the hybrid reduction are launched separately.
hipError_t launch_ect_hybrid(int ndim, unsigned mask, int precision, const HybridArgs& h, const EctArgs& e,
                             int64_t grid, int64_t ect_blocks, int64_t ect_groups, hipStream_t stream);
// ect_chunk_sum_kernel after a chunked shared-set ECT of `grid` workgroups.
hipError_t launch_ect_chunk_sum(const EctArgs& e, int64_t grid, int64_t groups, hipStream_t stream);

}  // namespace ect
