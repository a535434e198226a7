// Internal declarations of the exact-representation stage (exact.hip).
#pragma once

#include "ect_internal.h"

namespace ect {

// What the exact stage records about one query row.
struct alignas(8) ExactRow {
    double xi[kMaxDim];
    int64_t base;     // first output entry of the row
    int64_t pc, po;   // first classical / ordinary point (index into the point array)
    int64_t nc, no;   // their counts (no: Radon only)
    int64_t img;      // the row's image
    int32_t sign_o;   // factor on the stored ordinary values (Radon)
    int32_t valid;    // 1 usable, 0 non-finite direction, -1 offsets leave no room
};

struct ExactArgs {
    const void* points;       // ListEntry records
    const ImageDesc* desc;    // per image: the entries' bit fields, origin and spacing
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
    uint64_t* keys_a;         // [capacity] x 2: sorted tiles and merge passes of lists longer than one tile
    uint64_t* keys_b;
    int32_t* vals_a;
    int32_t* vals_b;
    double* ct;               // Radon [capacity]: distinct classical projections, at the row's classical slots
    int32_t* cum;             // Radon [capacity]: their running classical sums
    double* T;
    int32_t* E;
    int64_t* len;
};

// Workspace of the row-offset scan (layout call).
size_t exact_layout_scan_bytes(int64_t rows);

// Entries per row, exclusive scan into a.row_off_out ([rows + 1]).
hipError_t launch_exact_layout(int ndim, const ExactArgs& a, int64_t* need, void* scan_tmp, size_t scan_bytes,
                               hipStream_t stream);
// One workgroup per row (exact_kernel); max_len: the longest list a row may
// read as far as the host knows (it picks the LDS tile; longer lists take the
// multi-tile path).
hipError_t launch_exact(int ndim, const ExactArgs& a, int64_t max_len, hipStream_t stream);
hipError_t launch_exact_eval(int32_t kind, int64_t rows, const int64_t* row_off, const double* T, const int32_t* E,
                             const int64_t* len, int64_t capacity, const double* thr, int32_t M, int32_t per_row,
                             int32_t* out, hipStream_t stream);

}  // namespace ect
