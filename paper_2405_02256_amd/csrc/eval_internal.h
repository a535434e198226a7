// Internal declarations of the evaluation stages (bucketing, work lists, ECT,
// hybrid transforms).
#pragma once

#include "ect_internal.h"

namespace ect {

constexpr int kBucketThreads = 256;
constexpr int kEctThreads = 256;      // ECT workgroup: points stream across its lanes
constexpr int kEctMaxDirs = 8;        // directions per ECT workgroup
constexpr int kEctMaxThresholds = 4096;
constexpr int kHybridLanes = 64;      // one wave per hybrid work item, one query per lane and slot

hipError_t launch_bucket(int ndim, const ect_query_set& qs, int num_images, bool hybrid, uint32_t* err,
                         int64_t* perm, int64_t* bstart, int32_t* bcnt, hipStream_t stream);

hipError_t launch_worklist(int num_images, int B, int list_base, int NL, bool shared_queries,
                           const int32_t* bcnt, const int64_t* list_off, int qtile, int64_t chunk,
                           int64_t capacity, uint32_t* err, int64_t* item_off, int64_t* tile_off,
                           int64_t* params, hipStream_t stream);

struct EctArgs {
    const Point* points;
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
    const int64_t* perm;
    const int64_t* bstart;
    const int32_t* bcnt;
    const int64_t* item_off;
    uint32_t* err;
    int dirs_per_group;
};

hipError_t launch_ect(int ndim, const EctArgs& a, int64_t grid, hipStream_t stream);

struct HybridArgs {
    const Point* points;
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
    double* out;
    double* log_scale;
    const double* fwd_out;    // backward: forward output
    const double* grad_out;   // backward
    double* grad_xi;          // backward: [rows][n] (ragged) or per-image partial [images][count][n]
    double* grad_s_part;      // backward: per-row contribution to d/ds
    const int64_t* perm;
    const int64_t* bstart;
    const int32_t* bcnt;
    const int64_t* item_off;
    const int64_t* tile_off;
    const int64_t* params;    // [0] items, [1] tiles, [2] chunk
    double* partials;
    uint32_t* counters;
    uint32_t* err;
};

hipError_t launch_hybrid_fwd(int ndim, int kernel, int precision, const HybridArgs& a, int64_t grid,
                             hipStream_t stream);
hipError_t launch_hybrid_bwd(int ndim, int kernel, int precision, const HybridArgs& a, int64_t grid,
                             hipStream_t stream);
hipError_t launch_grad_reduce(int ndim, const double* part, int num_images, int64_t count, bool shared,
                              double* grad_xi, const double* gs_part, int64_t rows, double* grad_s,
                              hipStream_t stream);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t stream);

}  // namespace ect
