/*
 * ect.h -- C ABI of the MI355X (gfx950) library for topological integral
 * transforms of weighted cubical complexes built from 2D images and 3D volumes.
 *
 * The library follows the method's problem statement:
 *   input    an n-dimensional array turned into a weighted cubical complex
 *            (Sec. 4.1: one top cell per pixel, lower cells take the min of
 *            their cofaces; Sec. 5: the dual rule, pixels on vertices and higher
 *            cells take the min of their vertices);
 *   queries  directions xi (Sec. 2.2, Sec. 4.3) and thresholds t (Sec. 4.3,
 *            vectorization);
 *   outputs  ECT(xi, t) = chi(phi restricted to {xi <= t}) and the hybrid
 *            transform HT(xi) = integral kappa(t) R(xi, t) dt (Sec. 2.2),
 *            computed from per-sign-vector critical points (Sec. 3, Lemma 3.1
 *            and Lemma 3.2).
 *
 * Conventions shared by every call:
 *   - Pointers marked DEVICE are HIP device pointers, HOST pointers are plain
 *     host memory.  The caller owns every buffer; the library allocates no
 *     device memory.  Work memory is passed as a workspace: calling with
 *     ws == NULL writes the number of bytes needed to *ws_bytes and returns
 *     ECT_OK without doing anything else.
 *   - Every call that takes a stream only enqueues work on it and returns;
 *     results are valid once the stream has been synchronised.  The calls
 *     that say "synchronises" block until their stream is idle.
 *   - Evaluation calls (ect_eval, hybrid_eval*, ect_plan_export) only read a
 *     plan's lists: several may run at the same time on different streams as
 *     long as each has its own workspace.  ect_plan_rerun rewrites the lists,
 *     so the caller orders it after every evaluation still reading them.
 *   - Embedding axis 0 is the fastest-varying memory axis of an image.  A
 *     vertex with integer index k_a along axis a sits at
 *     x_a = fma(spacing_a, k_a, origin_a); the default origin centres the
 *     complex (origin_a = -N_a/2, N_a = number of top cells along a) and the
 *     default spacing is 1 (pixel units).
 *   - The projection of vertex x on xi is the canonical FP64 expression
 *     u = fma(xi_{n-1}, x_{n-1}, ... fma(xi_1, x_1, xi_0 * x_0)), the same on
 *     every code path, which makes the integer ECT exact: it equals the
 *     definition evaluated over all cells with this projection.
 *   - The sign vector of xi has eps_a = +1 when xi_a >= 0 (including -0.0)
 *     and -1 otherwise.  Sign-vector index e: bit a set means eps_a = -1.
 *   - Kernels with scale s != 0: kappa_s(t) = kappa(s t) and its primitive
 *     kbar_s(t) = kbar(s t) / s, with
 *         ECT_FOURIER  kappa = exp(-i t), kbar = i exp(-i t) = sin t + i cos t
 *         ECT_LAPLACE  kappa = exp(-t),   kbar = -exp(-t)
 *         ECT_BESSEL   kappa = J0,        kbar = Ji0(t) = integral_0^t J0
 *     so that HT(xi) = sum over ordinary critical points x of
 *     Delta^ord(eps, x) * kbar_s(<xi, x>) (the sign that the definition of HT
 *     gives; see the readings of the method).
 *   - No C++ exception crosses this boundary.  Errors found on the host are
 *     returned before anything is enqueued and leave outputs untouched;
 *     errors that depend on device data set bits of the plan's device error
 *     word (ECT_DEVERR_*), read with ect_plan_check().
 */
#ifndef ECT_H
#define ECT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#pragma GCC visibility push(default)

typedef enum {
    ECT_OK = 0,
    ECT_E_INVALID = 1,      /* bad argument (null pointer, bad enum, size, non-finite scalar) */
    ECT_E_NOMEM = 2,        /* workspace smaller than required, or host allocation failed */
    ECT_E_DEVICE = 3,       /* a HIP runtime call failed */
    ECT_E_UNSUPPORTED = 4,  /* valid request outside what this build implements */
    ECT_E_RANGE = 5,        /* a value does not fit the output type */
    ECT_E_SCRATCH = 6       /* hybrid_eval_noalloc: the call needs more work memory than the
                               static scratch array holds (ECT_NOALLOC_SCRATCH_BYTES) */
} ect_status;

typedef enum { ECT_PRIMAL = 0, ECT_DUAL = 1 } ect_construction;
typedef enum { ECT_U8 = 0, ECT_I16 = 1, ECT_I32 = 2 } ect_dtype;
typedef enum { ECT_FOURIER = 0, ECT_LAPLACE = 1, ECT_BESSEL = 2 } ect_kernel;

/* ECT_FP32: FP64 phases and argument reduction, FP32 kernel values, FP64
 * accumulation and FP64 fixed-order reduction.  ECT_FP64: everything in FP64. */
typedef enum { ECT_FP32 = 0, ECT_FP64 = 1 } ect_precision;

/* Device error word bits (ect_plan_check). */
#define ECT_DEVERR_THRESHOLDS    0x2u  /* thresholds not non-decreasing: that image's ECT rows are zero */
#define ECT_DEVERR_NONFINITE     0x4u  /* a non-finite direction: its outputs are NaN / zero */
#define ECT_DEVERR_LOOKBACK      0x8u  /* ordered compaction gave up waiting (never expected) */
#define ECT_DEVERR_OVERFLOW      0x10u /* a Laplace output overflowed without a log-scale output */
#define ECT_DEVERR_CAPACITY      0x20u /* hybrid work list larger than its workspace */
#define ECT_DEVERR_LAYOUT        0x40u /* exact representation: a row's offsets leave no room for it */
#define ECT_DEVERR_SCALE         0x80u /* a device kernel scale (hybrid_eval_multi_s, ...) is 0 or not finite */

/* A batch of images.  Every image of a batch has the same ndim, dtype and
 * construction; sizes may differ (ragged batch). */
typedef struct {
    int32_t ndim;                  /* 2, 3 or 4 (n-dimensional arrays, Sec. 4.1) */
    int32_t num_images;            /* >= 1 */
    const int32_t* dims;           /* HOST [num_images][ndim]: pixels along axis a (>= 1; dual needs >= 1) */
    const int64_t* pixel_offsets;  /* HOST [num_images]: element offset of image i in `pixels` */
    const void* pixels;            /* DEVICE: element type `dtype`, each image contiguous, axis 0 fastest;
                                      read by ect_precompute / ect_plan_rerun only */
    int32_t dtype;                 /* ect_dtype; int32 values must lie in [-2^26, 2^26] */
    int32_t construction;          /* ect_construction */
    const double* origin;          /* HOST [num_images][ndim] or NULL (centred) */
    const double* spacing;         /* HOST [num_images][ndim] or NULL (1.0) */
} ect_image_batch;

/* A set of query vectors (ECT directions or hybrid xi), FP64.
 * Shared set (offsets == NULL): `count` vectors used by every image; row of
 * query k of image i is i*count + k.  Ragged set: image i owns rows
 * offsets[i] .. offsets[i+1]-1 and `count` is the total number of rows
 * (offsets[num_images]). */
typedef struct {
    const double* vecs;            /* DEVICE [rows][ndim]; may be NULL when count is 0 */
    const int64_t* offsets;        /* DEVICE [num_images+1], non-decreasing, or NULL */
    int64_t count;
} ect_query_set;

typedef struct ect_plan_s* ect_plan;  /* host handle; the critical-point lists live in the workspace */

/* ect_precompute -- per-vertex critical values for every sign vector and
 * their ordered compaction into lists (Sec. 3 definitions of Delta^- and
 * Delta^ord, Sec. 4.2 preprocessing, Lemma 3.2 for why 2^n sign vectors
 * suffice).  For each image and each eps it builds the classical list
 * {(x, Delta^-(eps,x)) : Delta^- != 0}; for each eps with eps_{n-1} = +1 it
 * builds the ordinary list {(x, Delta^ord(eps,x)) : Delta^ord != 0}; the
 * lists of eps_{n-1} = -1 are the same points with negated values, because
 * the upper star for eps is the lower star for -eps.  Lists are ordered by
 * linear vertex index.
 *   batch     HOST descriptor (copied; `pixels` must stay valid while the
 *             plan may rerun)
 *   ws        DEVICE workspace of *ws_bytes bytes, 256-byte aligned; it holds
 *             the lists and must outlive the plan
 *   stream    HIP stream for the work
 *   out       receives the plan handle (only when ws != NULL)
 * Synchronises once at the end to read the list sizes back to the host.
 * A list entry is 8 bytes: the vertex index packed into 32 bits (axis a takes
 * ceil(log2 V_a) bits, V_a the largest vertex count along axis a over the
 * batch) and the critical value.
 * Returns ECT_E_INVALID for a malformed batch, ECT_E_NOMEM when *ws_bytes is
 * too small, ECT_E_UNSUPPORTED when an image has 2^31 vertices or more or the
 * bit fields of the vertex index need more than 32 bits (e.g. beyond
 * 65535^2 pixels, 2047^3 voxels or 255^4 in the primal construction). */
ect_status ect_precompute(const ect_image_batch* batch, void* ws, size_t* ws_bytes,
                          hipStream_t stream, ect_plan* out);

/* Re-run the precompute kernels of an existing plan on its pixel buffer (same
 * shapes, new contents).  Enqueues kernels only (no copies, no allocation, no
 * synchronisation), so it can be captured into a HIP graph: one kernel launch,
 * no reset launch before it.  List sizes held on the host are NOT refreshed;
 * device-side consumers read the new sizes. */
ect_status ect_plan_rerun(ect_plan plan, hipStream_t stream);

/* ect_eval -- ECT(xi, t_j) at every direction xi of `dirs` and every
 * threshold t_j (Sec. 2.2 definition; Lemma 3.1: ECT(xi, .) is the sum of
 * Delta^-(eps, x) 1[<xi,x>, inf) over classical points; Sec. 4.3
 * vectorization at explicit thresholds).  Exact int32 result.
 *   dirs            query set (DEVICE vectors)
 *   thresholds      DEVICE [M] (thresholds_per_image == 0) or [num_images][M];
 *                   non-decreasing per image, closed sublevel sets (u <= t)
 *   out             DEVICE int32 [rows][M], row-major
 *   ws, ws_bytes    DEVICE workspace (ws == NULL: size query).  A shared
 *                   set (offsets == NULL) needs none: the size is 0 and any
 *                   non-NULL ws runs the call.  Ragged sets are bucketed by
 *                   sign vector in the workspace first.
 * Unsorted thresholds or non-finite directions are detected on the device
 * (error word). */
ect_status ect_eval(ect_plan plan, ect_query_set dirs, const double* thresholds, int32_t M,
                    int32_t thresholds_per_image, int32_t* out, void* ws, size_t* ws_bytes,
                    hipStream_t stream);

/* radon_eval -- the Radon transform R(xi, t_j) = chi of the slice {<xi,.> = t_j}
 * (Sec. 2.2) at every direction of `dirs` and every threshold, from the
 * critical points (Lemma 3.1, with the sign the definition gives):
 *   R(xi, t) = sum over classical points of Delta^-(eps,x) [<xi,x> = t]
 *            - sum over ordinary points of D(eps,x) [<xi,x> < t],
 * with the canonical FP64 projection, so the integer result equals the slice
 * Euler characteristic of the cells exactly, ties included.  Arguments,
 * layout, workspace and errors as ect_eval. */
ect_status radon_eval(ect_plan plan, ect_query_set dirs, const double* thresholds, int32_t M,
                      int32_t thresholds_per_image, int32_t* out, void* ws, size_t* ws_bytes,
                      hipStream_t stream);

/* Exact representations along each direction (Sec. 4.3).
 *   ECT_EXACT_ECT    (T, E): T[0] = -inf, then the distinct projections of the
 *                    classical points of eps(xi) in increasing order; E[i] =
 *                    ECT(xi, t) for T[i] <= t < T[i+1] (running sums of the
 *                    critical values, equal projections merged).
 *   ECT_EXACT_RADON  (T, E', Tc, Ec): T[0] = -inf, then the distinct
 *                    projections of the ordinary points of the orthant pair,
 *                    E'[i] = R(xi, t) for T[i] < t < T[i+1] away from Tc
 *                    (running sums of -D(eps,x)); Tc the distinct classical
 *                    projections, Ec[k] = R(xi, Tc[k]) = E'[largest i with
 *                    T[i] < Tc[k]] + the classical values at Tc[k].
 * Projections use the canonical FP64 expression, so every entry is exact. */
typedef enum { ECT_EXACT_ECT = 0, ECT_EXACT_RADON = 1 } ect_exact_kind;

/* ect_exact_layout -- entries each query row needs and their offsets:
 * row_off[r] = first entry of row r, row_off[rows] = total (the capacity the
 * caller allocates for T and E).  ECT: classical points + 1 per row; Radon:
 * ordinary points + 1 + classical points (an upper bound: merged projections
 * leave the rest of a row unused); a non-finite direction: 1.
 *   row_off         DEVICE int64 [rows + 1], written
 *   ws, ws_bytes    DEVICE workspace (ws == NULL: size query)
 * Reads the list sizes on the device, so it follows ect_plan_rerun. */
ect_status ect_exact_layout(ect_plan plan, ect_query_set dirs, int32_t kind, int64_t* row_off, void* ws,
                            size_t* ws_bytes, hipStream_t stream);

/* ect_exact -- the exact representation of every query row (sort by
 * projection, merge of equal projections, running sums; Sec. 4.3).
 *   row_off         DEVICE int64 [rows + 1] from ect_exact_layout on the same
 *                   plan contents and query set
 *   capacity        entries of T and E (>= row_off[rows], < 2^32)
 *   T, E            DEVICE double / int32 [capacity]: row r writes entries
 *                   from row_off[r]: ECT: (T, E) of length len[r]; Radon:
 *                   (T, E') of length len[2r], then (Tc, Ec) of length
 *                   len[2r+1].  Entries past those are left unspecified.
 *   len             DEVICE int64 [rows] (ECT) or [rows][2] (Radon)
 *   ws, ws_bytes    DEVICE workspace (ws == NULL: size query; depends on
 *                   kind, rows and capacity)
 * A row whose offsets leave it less room than ect_exact_layout gives, or
 * reach past capacity, gets length 0 and raises ECT_DEVERR_LAYOUT; a
 * non-finite direction gets T = [-inf], E = [0] (Radon: no Tc) and raises
 * ECT_DEVERR_NONFINITE. */
ect_status ect_exact(ect_plan plan, ect_query_set dirs, int32_t kind, const int64_t* row_off, int64_t capacity,
                     double* T, int32_t* E, int64_t* len, void* ws, size_t* ws_bytes, hipStream_t stream);

/* ect_exact_eval -- evaluation of exact representations at thresholds by
 * binary search (Sec. 4.3): ECT: E[largest i with T[i] <= t]; Radon: Ec[k]
 * where Tc[k] == t, else E'[largest i with T[i] < t].  Any thresholds (no
 * order needed); t = NaN, or a row of length 0, gives 0.
 *   rows, row_off, T, E, len, capacity   as written by ect_exact
 *   thresholds      DEVICE double [M] (thresholds_per_row == 0) or [rows][M]
 *   out             DEVICE int32 [rows][M]
 * A row whose entries would reach past capacity gives zeros. */
ect_status ect_exact_eval(int32_t kind, int64_t rows, const int64_t* row_off, const double* T, const int32_t* E,
                          const int64_t* len, int64_t capacity, const double* thresholds, int32_t M,
                          int32_t thresholds_per_row, int32_t* out, hipStream_t stream);

/* hybrid_eval -- HT(xi) = integral kappa_s(t) R(xi,t) dt (Sec. 2.2), evaluated
 * as the sum over ordinary critical points of Delta^ord(eps,x) kbar_s(<xi,x>)
 * (Lemma 3.1 with the sign that the definition gives).
 *   kernel, s       ect_kernel and scale (s finite).  s = 0 is the limit of
 *                   the scaled kernels: kappa_0 = kappa(0) = 1 for all three,
 *                   so HT_0(xi) = integral of R(xi, t) dt = sum over ordinary
 *                   points of Delta^ord <xi, x> (Fourier: that real part and
 *                   imaginary part 0; Laplace log_scale 0)
 *   precision       ect_precision
 *   xi              query set (DEVICE vectors)
 *   out             DEVICE double [rows] (Laplace, Bessel) or [rows][2]
 *                   (Fourier: real, imaginary)
 *   log_scale       DEVICE double [rows] or NULL.  Laplace only: when given,
 *                   out holds HT * exp(-log_scale), where log_scale = m2 ln 2
 *                   for an integer m2 that follows the largest exponent
 *                   -s <xi,x> over the query's ordinary points (within
 *                   [max - 256 ln 2, max + ln 2)), so that no term overflows
 *                   and the largest never underflows, wherever the object
 *                   sits in its frame; when NULL out holds HT, scaled back
 *                   exactly by 2^m2, and an HT beyond the FP64 range sets
 *                   ECT_DEVERR_OVERFLOW.  Other kernels: must be NULL.
 * Deterministic: repeated calls give bitwise identical outputs. */
ect_status hybrid_eval(ect_plan plan, int32_t kernel, double s, int32_t precision,
                       ect_query_set xi, double* out, double* log_scale,
                       void* ws, size_t* ws_bytes, hipStream_t stream);

/* hybrid_eval_noalloc -- hybrid_eval for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses
 * that forbid hipMalloc): the same computation, kernels and outputs as
 * hybrid_eval(plan, kernel, s, precision, xi, out, log_scale, ...), bit for
 * bit, with the work memory taken from a static device array of
 * ECT_NOALLOC_SCRATCH_BYTES bytes inside the library instead of a caller
 * workspace.  Each GPU the library runs on holds its own copy of that array
 * until the process ends; its address is looked up once per device, on the
 * first call with that device current.  The call allocates nothing, on the
 * host or the device.
 *   arguments       as hybrid_eval (no workspace)
 * The current device must be the plan's device (ECT_E_INVALID otherwise).
 * A call whose hybrid_eval workspace would exceed ECT_NOALLOC_SCRATCH_BYTES
 * returns ECT_E_SCRATCH before enqueuing anything.  Every call on one GPU
 * shares that GPU's array and overwrites what the previous call left there:
 * calls that may overlap on one GPU (different streams, or different host
 * threads, without ordering between them) race and must not be issued.
 * A following hybrid_eval_backward cannot reuse its buckets. */
#define ECT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
ect_status hybrid_eval_noalloc(ect_plan plan, int32_t kernel, double s, int32_t precision,
                               ect_query_set xi, double* out, double* log_scale, hipStream_t stream);

/* hybrid_eval_multi -- several hybrid transforms in one pass over the same
 * (query, critical point) pairs, sharing the projection <xi, x> and the staged
 * points.  kernel_mask: bit k set evaluates ect_kernel k (1..7).  Each output
 * has the layout hybrid_eval gives for its kernel and must be non-NULL when
 * its bit is set; log_scale_laplace as hybrid_eval's log_scale (Laplace only).
 * Results equal those of separate hybrid_eval calls bit for bit. */
ect_status hybrid_eval_multi(ect_plan plan, uint32_t kernel_mask, double s, int32_t precision,
                             ect_query_set xi, double* out_fourier, double* out_laplace, double* out_bessel,
                             double* log_scale_laplace, void* ws, size_t* ws_bytes, hipStream_t stream);

/* hybrid_eval_multi_s, hybrid_eval_backward_s -- hybrid_eval_multi and
 * hybrid_eval_backward with the kernel scale read by the kernels from device
 * memory: a learnable scale (the kernel's s in kappa(s t)) can then change
 * between replays of a captured HIP graph without a copy to the host.
 *   s               DEVICE double scalar, read when the kernels run; it must
 *                   be finite and nonzero (the constant-kernel limit s = 0 is
 *                   not available here): otherwise ECT_DEVERR_SCALE is raised
 *                   and the outputs are not finite
 * Every other argument, layout and error as in hybrid_eval_multi and
 * hybrid_eval_backward; the outputs equal theirs at the same value of s bit
 * for bit. */
ect_status hybrid_eval_multi_s(ect_plan plan, uint32_t kernel_mask, const double* s, int32_t precision,
                               ect_query_set xi, double* out_fourier, double* out_laplace, double* out_bessel,
                               double* log_scale_laplace, void* ws, size_t* ws_bytes, hipStream_t stream);
ect_status hybrid_eval_backward_s(ect_plan plan, int32_t kernel, const double* s, int32_t precision,
                                  ect_query_set xi, const double* out, const double* grad_out, double* grad_xi,
                                  double* grad_s, uint32_t flags, void* ws, size_t* ws_bytes, hipStream_t stream);

/* ect_hybrid_eval_multi -- ect_eval(plan, dirs, thresholds, M,
 * thresholds_per_image, ect_out) and hybrid_eval_multi(plan, kernel_mask, s,
 * precision, xi, out_fourier, out_laplace, out_bessel, log_scale_laplace) in
 * one call with one workspace; every argument means what it means there, and
 * the outputs equal those of the two separate calls bit for bit.  For a
 * shared direction set with at most two directions per ECT workgroup and
 * small threshold arrays (M (8 + 4 d) <= 4096 bytes of LDS, d the directions
 * per workgroup) and s != 0, the ECT workgroups run in the same launch as
 * the hybrid work items, so the short ECT work fills the hybrid pass's idle
 * compute units instead of running before it; otherwise the two run one
 * after the other.  The hybrid part's buckets and work list sit at the start
 * of ws, so a following hybrid_eval_backward with the same ws and
 * ECT_BWD_REUSE_PREPARED reuses them.  Errors: those of either call. */
ect_status ect_hybrid_eval_multi(ect_plan plan, ect_query_set dirs, const double* thresholds, int32_t M,
                                 int32_t thresholds_per_image, int32_t* ect_out, uint32_t kernel_mask, double s,
                                 int32_t precision, ect_query_set xi, double* out_fourier, double* out_laplace,
                                 double* out_bessel, double* log_scale_laplace, void* ws, size_t* ws_bytes,
                                 hipStream_t stream);

/* ect_plan_rerun_prepare -- ect_plan_rerun, and in the same launch the
 * bucketing and work list that the next hybrid evaluation (hybrid_eval,
 * hybrid_eval_multi or ect_hybrid_eval_multi, forward) of the shared query set
 * xi with workspace ws would write first; that call then skips them.  The
 * query workgroup runs beside the compaction's tiles instead of after them.
 * Used for two-axis, single-image plans whose compaction runs in one pass with
 * room for one more workgroup, and for 1 .. 65536 query rows; otherwise this
 * is ect_plan_rerun and the evaluation buckets the set itself.  ws_bytes: the
 * size hybrid_eval needs for xi (ws == NULL: size query).  The set must not
 * change until that evaluation is enqueued; any call in between that writes
 * ws, re-runs or retunes the plan cancels the skip.  xi.offsets must be NULL
 * (ECT_E_INVALID otherwise). */
ect_status ect_plan_rerun_prepare(ect_plan plan, ect_query_set xi, void* ws, size_t* ws_bytes, hipStream_t stream);

/* hybrid_eval_backward -- vector-Jacobian product of hybrid_eval (without
 * log_scale) with respect to xi and to the scale s.  With kappa the kernel,
 * dHT/dxi_a = sum Delta^ord x_a kappa(s <xi,x>) and
 * dHT/ds = (1/s) [sum Delta^ord <xi,x> kappa(s <xi,x>) - HT].  s must be
 * nonzero (s = 0 returns ECT_E_UNSUPPORTED).
 *   out         DEVICE: the forward output of the same call (needed for d/ds)
 *   grad_out    DEVICE, layout of out
 *   grad_xi     DEVICE double [rows][ndim] for a ragged set; for a shared set
 *               [count][ndim], summed over images in image order
 *   grad_s      DEVICE double scalar (sum over all rows) or NULL
 *   flags       0, or ECT_BWD_REUSE_PREPARED: ws still holds the query
 *               buckets and work list written by the last hybrid_eval /
 *               hybrid_eval_multi / hybrid_eval_backward call on this plan
 *               with this ws and this query set (same vector and offset
 *               pointers, same count, unchanged contents), enqueued earlier
 *               on the same stream with no use of ws in between; the
 *               bucketing pass is then skipped.  The host checks what it
 *               can (workspace and query pointers, count, no ect_plan_rerun or
 *               ect_plan_set_tuning since) and returns ECT_E_INVALID when the
 *               last preparation does not match; unchanged contents are the
 *               caller's promise.  Forward and backward calls need the same
 *               workspace size.
 * Valid away from directions with a zero coordinate (the transform has kinks
 * there). */
#define ECT_BWD_REUSE_PREPARED 0x1u
ect_status hybrid_eval_backward(ect_plan plan, int32_t kernel, double s, int32_t precision,
                                ect_query_set xi, const double* out, const double* grad_out,
                                double* grad_xi, double* grad_s, uint32_t flags,
                                void* ws, size_t* ws_bytes, hipStream_t stream);

/* Number of list entries per image, read from the host copy made at the end
 * of ect_precompute.  classical: HOST int64 [num_images][2^ndim];
 * ordinary: HOST int64 [num_images][2^(ndim-1)] (lists of eps with
 * eps_{n-1} = +1, index e < 2^(ndim-1)).  Either may be NULL. */
ect_status ect_plan_counts(ect_plan plan, int64_t* classical, int64_t* ordinary);

/* Copy one list of one image to the host (tests, caching).  kind 0 =
 * classical (list = e in [0, 2^ndim)), kind 1 = ordinary (list = e in
 * [0, 2^(ndim-1))).  coords: HOST int32 [capacity][ndim] vertex indices k;
 * values: HOST int32 [capacity].  *count receives the list length; at most
 * `capacity` entries are written.  Synchronises the plan's stream. */
ect_status ect_plan_export(ect_plan plan, int32_t image, int32_t kind, int32_t list,
                           int32_t* coords, int32_t* values, int64_t capacity, int64_t* count,
                           hipStream_t stream);

/* Read and clear the device error word: the ECT_DEVERR_* bits raised since
 * the plan was created or last checked.  Synchronises. */
ect_status ect_plan_check(ect_plan plan, uint32_t* device_error_flags, hipStream_t stream);

/* Free the host handle (the workspace stays with the caller). */
ect_status ect_plan_destroy(ect_plan plan);

/* Tuning knobs of one plan (used by the autotuner): hybrid point-chunk
 * length per work item (0 = automatic, else 16 .. 2^40), target number of
 * hybrid work items when automatic (1 .. 2^24), directions per ECT workgroup
 * (1..8, 0 = automatic) and, for shared direction sets, the number of parts
 * each list is split into for one group of directions (0 = automatic, else
 * 1 .. 4096; 1 = no split).  Out-of-range values return ECT_E_INVALID and
 * leave the plan unchanged.
 * They only change the schedule: the ECT is exact whatever they are, hybrid
 * results differ only by the rounding of the chunked sums, and identical
 * settings give bitwise identical results. */
ect_status ect_plan_set_tuning(ect_plan plan, int64_t hybrid_chunk, int64_t hybrid_target_items,
                               int32_t ect_dirs_per_group, int32_t ect_chunks);

/* Profiling hook (process-wide): when set, the library records `before` on
 * the call's stream right before it launches the main kernel of `stage` and
 * `after` right after it, so that hipEventElapsedTime measures that kernel
 * alone (the small bucketing and work-list kernels of the call fall outside).
 * stage: ECT_STAGE_*.  Pass NULL events to disable.  Not thread-safe. */
#define ECT_STAGE_PRECOMPUTE   0
#define ECT_STAGE_ECT          1
#define ECT_STAGE_HYBRID       2
#define ECT_STAGE_HYBRID_BWD   3
ect_status ect_set_stage_events(int32_t stage, hipEvent_t before, hipEvent_t after);

/* Static description of a status code. */
const char* ect_status_string(ect_status status);

/* Library version, "major.minor.patch". */
const char* ect_version(void);

#pragma GCC visibility pop

#ifdef __cplusplus
}
#endif

#endif /* ECT_H */
