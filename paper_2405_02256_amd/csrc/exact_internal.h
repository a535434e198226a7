// Internal declarations of the exact-representation stage (exact.hip).
#pragma once

#include "ect_internal.h"

namespace ect {

// What the exact stage records about one query row.
struct alignas(8) ExactRow {
    double xi[3];
    int64_t base;     // first output entry of the row
    int64_t pc, po;   // first classical / ordinary point (index into the point array)
    int64_t nc, no;   // their counts (no: Radon only)
    int32_t sign_o;   // factor on the stored ordinary values (Radon)
    int32_t valid;    // 1 usable, 0 non-finite direction, -1 offsets leave no room
};

struct ExactArgs {
    const Point* points;
    const int64_t* list_off;
    int64_t list_capacity;    // entries per list region of the point array
    int num_images;
    int NL;
    const double* vecs;
    const int64_t* offsets;   // device or null
    int64_t count;
    int64_t rows;
    int32_t kind;             // ect_exact_kind
    uint32_t* err;
    const int64_t* row_off;   // [rows + 1]
    int64_t* row_off_out;     // layout: written
    int64_t capacity;         // output entries
    ExactRow* rowrec;
    uint32_t* seg_begin;
    uint32_t* seg_end;
    uint64_t* keys_in;
    uint64_t* keys_out;
    int32_t* vals_in;
    int32_t* vals_out;
    int32_t* cum;             // Radon: running classical sums at the distinct projections
    double* T;
    int32_t* E;
    int64_t* len;
};

__host__ __device__ inline int64_t exact_segments(int32_t kind, int64_t rows) {
    return kind == ECT_EXACT_ECT ? rows : 2 * rows;
}

// Workspace of the row-offset scan (layout call) and of the segmented sort.
size_t exact_layout_scan_bytes(int64_t rows);
size_t exact_sort_bytes(int32_t kind, int64_t rows, int64_t capacity);

// Entries per row, exclusive scan into a.row_off_out ([rows + 1]).
hipError_t launch_exact_layout(int ndim, const ExactArgs& a, int64_t* need, void* scan_tmp, size_t scan_bytes,
                               hipStream_t stream);
hipError_t launch_exact(int ndim, const ExactArgs& a, void* sort_tmp, size_t sort_bytes, hipStream_t stream);
hipError_t launch_exact_eval(int32_t kind, int64_t rows, const int64_t* row_off, const double* T, const int32_t* E,
                             const int64_t* len, int64_t capacity, const double* thr, int32_t M, int32_t per_row,
                             int32_t* out, hipStream_t stream);

}  // namespace ect
