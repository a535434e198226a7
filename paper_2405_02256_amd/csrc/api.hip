// Host side of the C ABI: argument validation, workspace layouts, plan
// bookkeeping and kernel launches.  No exception crosses the boundary and no
// device memory is allocated here.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "eval_internal.h"
#include "exact_internal.h"

using namespace ect;

namespace ect {
StageEvents g_stage_events[4];
}

namespace {

constexpr size_t kAlign = 256;
constexpr int64_t kAheadMaxRows = 65536;   // query rows one workgroup buckets inside the compaction launch
constexpr int kAccSlotsHost = 5;  // doubles per query in a partial record (sums and the Laplace shift)

struct EvalLayout {
    size_t recs, bcnt, item_off, tile_off, params, partials, tile_ent, gpart, gspart, total;
    int64_t groups, entries, grid, capacity, tiles;
};

bool valid_query_set(const ect_query_set& q, int num_images) {
    if (q.count < 0 || (!q.vecs && q.count > 0)) return false;
    (void)num_images;
    return true;
}

int64_t query_rows(const ect_query_set& q, int num_images) {
    return q.offsets ? q.count : q.count * (int64_t)num_images;
}

// Workspace shared by the evaluation calls: bucketing and work list.  Bucket
// b of image i owns B * Q_i record slots (see queries.hip).
void layout_common(const Plan& p, const ect_query_set& q, int B, EvalLayout* L, size_t* off) {
    const bool shared = q.offsets == nullptr;
    const int64_t groups = shared ? 1 : p.num_images;
    L->groups = groups;
    L->entries = (int64_t)p.num_images * B;
    size_t o = *off;
    L->recs = o; o = align_up(o + qrec_bytes(p.ndim) * (size_t)B * std::max<int64_t>(q.count, 1), kAlign);
    L->bcnt = o; o = align_up(o + sizeof(int32_t) * groups * B, kAlign);
    L->item_off = o; o = align_up(o + sizeof(int64_t) * (L->entries + 1), kAlign);
    L->tile_off = o; o = align_up(o + sizeof(int64_t) * (L->entries + 1), kAlign);
    L->params = o; o = align_up(o + sizeof(int64_t) * 4, kAlign);
    *off = o;
}

// Largest list of each ordinary (or classical) kind, from the host copy of
// the list offsets made by ect_precompute.
int64_t max_list(const Plan& p, int base, int count) {
    const int NL = num_lists(p.ndim);
    int64_t m = 0;
    for (int i = 0; i < p.num_images; ++i)
        for (int b = 0; b < count; ++b) {
            int64_t n = p.h_list_off[(int64_t)(i + 1) * NL + base + b] - p.h_list_off[(int64_t)i * NL + base + b];
            m = std::max(m, n);
        }
    return m;
}

double mean_list(const Plan& p, int base, int count) {
    const int NL = num_lists(p.ndim);
    double s = 0;
    for (int b = 0; b < count; ++b)
        s += (double)(p.h_list_off[(int64_t)p.num_images * NL + base + b] - p.h_list_off[base + b]);
    return s / std::max(1, p.num_images * count);
}

int64_t hybrid_chunk_for(const Plan& p, int64_t rows) {
    if (p.tune_hybrid_chunk > 0) return p.tune_hybrid_chunk;
    const int P = num_ordinary(p.ndim);
    const double avg = mean_list(p, num_classical(p.ndim), P);
    const double pairs = (double)rows * avg;
    double c = pairs / ((double)kHybridTile * (double)p.tune_hybrid_target_items);
    int64_t ci = (int64_t)std::ceil(std::max(32.0, c) / 16.0) * 16;
    return ci;
}

void layout_hybrid(const Plan& p, const ect_query_set& q, bool backward, EvalLayout* L, int64_t* chunk) {
    const int P = num_ordinary(p.ndim);
    size_t o = 0;
    layout_common(p, q, P, L, &o);
    const bool shared = q.offsets == nullptr;
    const int64_t rows = query_rows(q, p.num_images);
    // query tiles: sum over (image, pair) of ceil(count / 64) <= rows/64 + images*P
    const int64_t tiles = shared ? (int64_t)p.num_images * ((q.count + kHybridTile - 1) / kHybridTile + P)
                                 : (rows + kHybridTile - 1) / kHybridTile + (int64_t)p.num_images * P;
    *chunk = hybrid_chunk_for(p, rows);
    const int64_t maxn = max_list(p, num_classical(p.ndim), P);
    const int64_t maxch = std::max<int64_t>(1, (maxn + *chunk - 1) / *chunk);
    L->tiles = tiles;
    L->grid = tiles * maxch;
    L->capacity = L->grid;
    L->partials = o; o = align_up(o + sizeof(double) * kAccSlotsHost * kHybridTile * std::max<int64_t>(L->capacity, 1), kAlign);
    L->tile_ent = o; o = align_up(o + sizeof(int32_t) * std::max<int64_t>(tiles, 1), kAlign);
    // gradient partials are reserved for forward calls too, so that one
    // workspace size serves a forward call and the backward call reusing its
    // buckets and work list
    (void)backward;
    L->gpart = o; o = align_up(o + sizeof(double) * p.ndim * std::max<int64_t>(rows, 1), kAlign);
    L->gspart = o; o = align_up(o + sizeof(double) * std::max<int64_t>(rows, 1), kAlign);
    L->total = o;
}

void layout_ect(const Plan& p, const ect_query_set& q, int td, EvalLayout* L) {
    const int B = num_classical(p.ndim);
    size_t o = 0;
    layout_common(p, q, B, L, &o);
    const bool shared = q.offsets == nullptr;
    const int64_t rows = query_rows(q, p.num_images);
    L->grid = shared ? (int64_t)p.num_images * ((q.count + td - 1) / td + B)
                     : (rows + td - 1) / td + (int64_t)p.num_images * B;
    L->total = o;
}

ect_status from_hip(hipError_t e) { return e == hipSuccess ? ECT_OK : ECT_E_DEVICE; }

bool is_finite(double v) { return std::isfinite(v); }

}  // namespace

// Work memory of hybrid_eval_noalloc: one static array per device.  In host
// code `scratch` names a host-side stand-in, never the device memory; the
// device address comes from hipGetSymbolAddress with that device current and
// is the only one passed to kernels.
static __device__ __align__(256) unsigned char scratch[ECT_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 256;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of the current device's scratch array, looked up on the
// first call with that device current.
ect_status scratch_address(int dev, void** ptr) {
    if (dev < 0 || dev >= kMaxScratchDevices) return ECT_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ECT_E_DEVICE;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return ECT_OK;
}

}  // namespace

extern "C" {

const char* ect_version(void) { return "0.1.0"; }

const char* ect_status_string(ect_status s) {
    switch (s) {
        case ECT_OK: return "ok";
        case ECT_E_INVALID: return "invalid argument";
        case ECT_E_NOMEM: return "workspace too small or host allocation failed";
        case ECT_E_DEVICE: return "HIP runtime error";
        case ECT_E_UNSUPPORTED: return "unsupported request";
        case ECT_E_RANGE: return "value out of range";
        case ECT_E_SCRATCH: return "request needs more work memory than the static scratch array holds";
    }
    return "unknown status";
}

ect_status ect_precompute(const ect_image_batch* batch, void* ws, size_t* ws_bytes, hipStream_t stream,
                          ect_plan* out) {
    if (!batch || !ws_bytes) return ECT_E_INVALID;
    const int n = batch->ndim;
    if (n < 2 || n > kMaxDim) return ECT_E_INVALID;
    if (batch->num_images < 1 || !batch->dims || !batch->pixel_offsets || !batch->pixels) return ECT_E_INVALID;
    if (batch->dtype < ECT_U8 || batch->dtype > ECT_I32) return ECT_E_INVALID;
    if (batch->construction != ECT_PRIMAL && batch->construction != ECT_DUAL) return ECT_E_INVALID;
    const int NL = num_lists(n);
    const int ni = batch->num_images;

    std::vector<ImageDesc> desc(ni);
    std::vector<int64_t> tstart(ni + 1);
    int64_t tiles = 0, verts = 0, maxv = 0;
    for (int i = 0; i < ni; ++i) {
        ImageDesc& d = desc[i];
        std::memset(&d, 0, sizeof(d));
        if (batch->pixel_offsets[i] < 0) return ECT_E_INVALID;
        d.pixel_offset = batch->pixel_offsets[i];
        int64_t nv = 1;
        for (int a = 0; a < kMaxDim; ++a) {
            if (a < n) {
                const int32_t dim = batch->dims[(int64_t)i * n + a];
                if (dim < 1 || dim > (1 << 20)) return ECT_E_INVALID;
                d.dims[a] = dim;
                d.N[a] = batch->construction == ECT_PRIMAL ? dim : dim - 1;
                d.V[a] = d.N[a] + 1;
                d.origin[a] = batch->origin ? batch->origin[(int64_t)i * n + a] : -0.5 * (double)d.N[a];
                d.spacing[a] = batch->spacing ? batch->spacing[(int64_t)i * n + a] : 1.0;
                if (!is_finite(d.origin[a]) || !is_finite(d.spacing[a])) return ECT_E_INVALID;
            } else {
                d.dims[a] = 1; d.N[a] = 0; d.V[a] = 1; d.origin[a] = 0.0; d.spacing[a] = 1.0;
            }
            nv *= d.V[a];
            const double x0 = d.origin[a];
            const double x1 = std::fma(d.spacing[a], (double)d.N[a], d.origin[a]);
            d.lo[a] = std::min(x0, x1);
            d.hi[a] = std::max(x0, x1);
        }
        if (nv >= (int64_t)1 << 31) return ECT_E_UNSUPPORTED;
        d.nvert = nv;
        d.tile_start = tiles;
        tstart[i] = tiles;
        tiles += (nv + tile_verts(n) - 1) / tile_verts(n);
        verts += nv;
        maxv = std::max(maxv, nv);
    }
    tstart[ni] = tiles;
    if (tiles >= (int64_t)1 << 31) return ECT_E_UNSUPPORTED;
    // bit fields of the list entries' vertex index: axis a takes enough bits
    // for the largest vertex count along it over the plan's images
    {
        uint32_t shift = 0;
        uint32_t bits[kMaxDim] = {0, 0, 0, 0};
        for (int a = 0; a < n; ++a) {
            int32_t vmax = 1;
            for (int i = 0; i < ni; ++i) vmax = std::max(vmax, desc[i].V[a]);
            while (((int64_t)1 << bits[a]) < (int64_t)vmax) ++bits[a];
        }
        for (int a = 0; a < n; ++a) shift += bits[a];
        if (shift > 32) return ECT_E_UNSUPPORTED;
        shift = 0;
        for (int i = 0; i < ni; ++i) {
            uint32_t sh = 0;
            for (int a = 0; a < kMaxDim; ++a) {
                desc[i].kshift[a] = a < n ? sh : 0u;
                desc[i].kmask[a] = a < n ? (uint32_t)(((uint64_t)1 << bits[a]) - 1u) : 0u;
                if (a < n) sh += bits[a];
            }
        }
    }

    PlanLayout L{};
    size_t o = 0;
    L.err = o; o = align_up(o + 16, kAlign);   // uint32 error word, uint32 spare, uint64 run counter
    L.desc = o; o = align_up(o + sizeof(ImageDesc) * ni, kAlign);
    L.tile_start = o; o = align_up(o + sizeof(int64_t) * (ni + 1), kAlign);
    L.tile_img = o; o = align_up(o + sizeof(int32_t) * tiles, kAlign);
    L.list_off = o; o = align_up(o + sizeof(int64_t) * (int64_t)(ni + 1) * NL, kAlign);
    // single pass: tile aggregates and totals of 64-tile groups; three passes:
    // tile counts (int32) and their prefixes (int64).  The size does not
    // depend on the device.
    L.status = o; o = align_up(o + sizeof(uint64_t) * (2 * tiles + (tiles + 63) / 64 + 1) * NL, kAlign);
    L.points = o; o = align_up(o + entry_bytes() * verts * NL, kAlign);
    // plans beyond the single pass's largest grid (64 groups of 64 tiles, on
    // any device) run three passes; with 8- or 16-bit pixels the count pass
    // leaves its entries packed in per-tile slots, so the last pass only
    // places them instead of classifying every vertex again
    const int64_t packed_bytes = (int64_t)sizeof(uint32_t) * tiles * NL * tile_verts(n);
    L.packed = o;
    L.packed_bytes = (tiles > 64 * 64 && batch->dtype != ECT_I32 && packed_bytes <= kPackedMaxBytes)
                         ? (size_t)packed_bytes : 0;
    o = align_up(o + L.packed_bytes, kAlign);
    L.total = o;
    L.num_tiles = tiles;
    L.capacity = verts;
    if (!ws) {
        *ws_bytes = L.total;
        return ECT_OK;
    }
    if (*ws_bytes < L.total) return ECT_E_NOMEM;
    if (((uintptr_t)ws) % kAlign) return ECT_E_INVALID;
    if (!out) return ECT_E_INVALID;

    Plan* p = new (std::nothrow) Plan();
    if (!p) return ECT_E_NOMEM;
    p->ndim = n;
    p->num_images = ni;
    p->dtype = batch->dtype;
    p->construction = batch->construction;
    p->pixels = batch->pixels;
    p->ws = (char*)ws;
    p->lay = L;
    p->total_verts = verts;
    p->max_image_verts = maxv;
    p->h_desc = new (std::nothrow) ImageDesc[ni];
    p->h_list_off = new (std::nothrow) int64_t[(int64_t)(ni + 1) * NL];
    if (!p->h_desc || !p->h_list_off) {
        ect_plan_destroy(p);
        return ECT_E_NOMEM;
    }
    std::memcpy(p->h_desc, desc.data(), sizeof(ImageDesc) * ni);
    // compaction workgroups the chip holds at once: plans with at most that
    // many tiles (and at most 64 groups of 64) use the single pass
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&p->num_cus, hipDeviceAttributeMultiprocessorCount, dev);
    p->device = dev;
    const int64_t per_cu = e == hipSuccess ? precompute_slots_per_cu(n, batch->construction, batch->dtype) : 0;
    if (per_cu <= 0) {
        ect_plan_destroy(p);
        return ECT_E_DEVICE;
    }
    p->precompute_grid = std::min<int64_t>(per_cu * p->num_cus, 64 * 64);
    if (n == 2) p->precompute_grid_flat = precompute_slots_per_cu(n, batch->construction, batch->dtype, true) * p->num_cus;

    std::vector<int32_t> timg;
    try {
        timg.resize((size_t)tiles);
    } catch (...) {
        ect_plan_destroy(p);
        return ECT_E_NOMEM;
    }
    for (int i = 0; i < ni; ++i)
        for (int64_t t = tstart[i]; t < tstart[i + 1]; ++t) timg[(size_t)t] = i;
    e = hipMemcpyAsync(p->ws + L.desc, desc.data(), sizeof(ImageDesc) * ni, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->ws + L.tile_start, tstart.data(), sizeof(int64_t) * (ni + 1), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->ws + L.tile_img, timg.data(), sizeof(int32_t) * (size_t)tiles, hipMemcpyHostToDevice,
                           stream);
    if (e == hipSuccess) e = launch_precompute(*p, true, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->h_list_off, p->ws + L.list_off, sizeof(int64_t) * (int64_t)(ni + 1) * NL,
                           hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        ect_plan_destroy(p);
        return ECT_E_DEVICE;
    }
    *out = p;
    return ECT_OK;
}

ect_status ect_plan_rerun(ect_plan plan, hipStream_t stream) {
    if (!plan) return ECT_E_INVALID;
    ++plan->lists_epoch;
    plan->last_prep.ahead = false;
    return from_hip(launch_precompute(*plan, false, stream));
}

ect_status ect_plan_rerun_prepare(ect_plan plan, ect_query_set xi, void* ws, size_t* ws_bytes, hipStream_t stream) {
    if (!plan || !ws_bytes) return ECT_E_INVALID;
    if (!valid_query_set(xi, plan->num_images) || xi.offsets) return ECT_E_INVALID;
    Plan& p = *plan;
    EvalLayout L{};
    int64_t chunk = 0;
    layout_hybrid(p, xi, false, &L, &chunk);
    if (!ws) {
        *ws_bytes = L.total;
        return ECT_OK;
    }
    if (*ws_bytes < L.total) return ECT_E_NOMEM;
    const int64_t rows = query_rows(xi, p.num_images);
    ++p.lists_epoch;
    auto& lp = p.last_prep;
    lp.ahead = false;
    if (rows == 0 || rows > kAheadMaxRows || !precompute_takes_queries(p))
        return from_hip(launch_precompute(p, false, stream));   // the evaluation buckets the set itself
    char* w = (char*)ws;
    QueryPrep qp;
    qp.vecs = xi.vecs;
    qp.rows = rows;
    qp.recs = (void*)(w + L.recs);
    qp.bcnt = (int32_t*)(w + L.bcnt);
    qp.qtile = kHybridTile;
    qp.chunk0 = chunk;
    qp.capacity = L.capacity;
    qp.item_off = (int64_t*)(w + L.item_off);
    qp.tile_off = (int64_t*)(w + L.tile_off);
    qp.params = (int64_t*)(w + L.params);
    const hipError_t e = launch_precompute(p, false, stream, &qp);
    if (e != hipSuccess) {
        lp.valid = false;
        return ECT_E_DEVICE;
    }
    lp.ws = ws;
    lp.vecs = xi.vecs;
    lp.offsets = nullptr;
    lp.count = xi.count;
    lp.epoch = p.lists_epoch;
    lp.valid = true;
    lp.ahead = true;
    return ECT_OK;
}

// How a threshold evaluation runs: directions per workgroup, list chunks, and
// whether a shared set goes straight to the direct kernel.
struct ThresholdSetup {
    int td;
    int64_t chunks;
    bool direct;
    bool batch;     // ect_batch_kernel after one bucketing of the shared set
    int64_t direct_groups;
    int threads;
    EvalLayout L;
};

static ect_status threshold_setup(const Plan& p, const ect_query_set& dirs, const double* thresholds, int32_t M,
                                  const int32_t* out, bool radon, ThresholdSetup* S) {
    if (!valid_query_set(dirs, p.num_images) || !thresholds) return ECT_E_INVALID;
    if (!out && query_rows(dirs, p.num_images) > 0) return ECT_E_INVALID;
    if (M < 1) return ECT_E_INVALID;
    if (M > kEctMaxThresholds) return ECT_E_UNSUPPORTED;
    // directions per workgroup: enough workgroups to fill the chip first, then
    // more directions per streamed point
    const int64_t nrows = query_rows(dirs, p.num_images);
    int td = p.tune_ect_dirs_per_group > 0
                 ? p.tune_ect_dirs_per_group
                 : (dirs.offsets == nullptr ? kEctMaxDirs
                                            : (int)std::min<int64_t>(kEctMaxDirs, std::max<int64_t>(1, nrows / 1024)));
    const int64_t lds_budget = 60 * 1024;
    const int64_t arrays = radon ? 2 : 1;   // histograms (+ Radon point values) per direction
    td = (int)std::min<int64_t>(td, (lds_budget - 8 * (int64_t)M) / (4 * arrays * (int64_t)M));
    td = std::max(1, std::min(td, kEctMaxDirs));
    // shared sets go straight to the evaluation kernel (no bucketing); long
    // lists are split into chunks so that enough workgroups share each group
    // of directions (about two per compute unit, at least 4096 points each:
    // below that a workgroup's fixed cost outweighs streaming its part)
    S->td = td;
    // short lists: one-wave workgroups (more blocks in flight per compute unit)
    S->threads = mean_list(p, 0, num_classical(p.ndim)) <= kEctSmallList ? 64 : kEctThreads;
    S->direct = dirs.offsets == nullptr;
    S->batch = false;
    S->chunks = 1;
    S->direct_groups = 0;
    S->L = EvalLayout{};
    // many images with short lists and a shared direction set: lanes own
    // directions (ect_batch_kernel), after one bucketing of the set; chosen
    // automatically, or by the autotuner through the automatic setting
    const int64_t batch_blocks = (int64_t)p.num_images << p.ndim;
    if (S->direct && !radon && p.tune_ect_dirs_per_group == 0 && p.tune_ect_chunks == 0 &&
        M <= kBatchMaxThresholds && batch_blocks >= 2 * (int64_t)std::max(p.num_cus, 1) &&
        mean_list(p, 0, num_classical(p.ndim)) <= kEctSmallList) {
        S->direct = false;
        S->batch = true;
        layout_ect(p, dirs, td, &S->L);
        S->L.grid = batch_blocks;
        return ECT_OK;
    }
    if (S->direct) {
        S->direct_groups = (dirs.count + td - 1) / td;
        const int64_t groups = (int64_t)p.num_images * S->direct_groups;
        const double avg = mean_list(p, 0, num_classical(p.ndim));
        const int64_t want = (2 * (int64_t)std::max(p.num_cus, 1) + groups - 1) / std::max<int64_t>(groups, 1);
        S->chunks = p.tune_ect_chunks > 0 ? p.tune_ect_chunks
                                          : std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)(avg / 4096.0)));
        if (S->chunks > 1) S->L.total = sizeof(int32_t) * (size_t)(groups * S->chunks * td * (int64_t)M * arrays);
        S->L.grid = groups * S->chunks;
        // fewer than two workgroups per compute unit: twice the waves in each,
        // so that more of the list's loads are in flight, without the extra
        // launch that splitting the list into parts would need to add them up
        if (S->threads == kEctThreads && S->L.grid < 2 * (int64_t)std::max(p.num_cus, 1))
            S->threads = kEctWideThreads;
    } else {
        layout_ect(p, dirs, td, &S->L);
    }
    return ECT_OK;
}

static EctArgs threshold_args(const Plan& p, const ect_query_set& dirs, const double* thresholds, int32_t M,
                              int32_t thresholds_per_image, int32_t* out, char* w, const ThresholdSetup& S) {
    EctArgs a{};
    a.points = (const void*)(p.ws + p.lay.points);
    a.list_off = (const int64_t*)(p.ws + p.lay.list_off);
    a.desc = (const ImageDesc*)(p.ws + p.lay.desc);
    a.capacity = p.lay.capacity;
    a.num_images = p.num_images;
    a.NL = num_lists(p.ndim);
    a.vecs = dirs.vecs;
    a.offsets = dirs.offsets;
    a.count = dirs.count;
    a.thresholds = thresholds;
    a.M = M;
    a.thr_per_image = thresholds_per_image ? 1 : 0;
    a.out = out;
    a.recs = S.direct ? nullptr : (const void*)(w + S.L.recs);
    a.bcnt = S.direct ? nullptr : (const int32_t*)(w + S.L.bcnt);
    a.item_off = S.direct ? nullptr : (const int64_t*)(w + S.L.item_off);
    a.err = (uint32_t*)(p.ws + p.lay.err);
    a.dirs_per_group = S.td;
    a.chunks = S.chunks;
    a.part = S.chunks > 1 ? (int32_t*)w : nullptr;
    a.threads = S.threads;
    return a;
}

static ect_status threshold_eval(ect_plan plan, ect_query_set dirs, const double* thresholds, int32_t M,
                                 int32_t thresholds_per_image, int32_t* out, void* ws, size_t* ws_bytes,
                                 hipStream_t stream, bool radon) {
    if (!plan || !ws_bytes) return ECT_E_INVALID;
    const Plan& p = *plan;
    ThresholdSetup S;
    const ect_status st = threshold_setup(p, dirs, thresholds, M, out, radon, &S);
    if (st != ECT_OK) return st;
    if (!ws) {
        *ws_bytes = S.L.total;
        return ECT_OK;
    }
    if (*ws_bytes < S.L.total) return ECT_E_NOMEM;
    if (query_rows(dirs, p.num_images) == 0) return ECT_OK;
    char* w = (char*)ws;
    hipError_t e = hipSuccess;
    if (plan->last_prep.ws == ws) plan->last_prep.valid = false;   // buckets or chunk sums overwrite it
    if (!S.direct) {
        // the batch kernel needs the buckets only, not the bucketed kernel's work list
        e = launch_prepare(p.ndim, dirs, p.num_images, false, (uint32_t*)(p.ws + p.lay.err), (void*)(w + S.L.recs),
                           (int32_t*)(w + S.L.bcnt), (const int64_t*)(p.ws + p.lay.list_off), 0, num_lists(p.ndim),
                           S.td, 0, 0, S.batch ? nullptr : (int64_t*)(w + S.L.item_off),
                           S.batch ? nullptr : (int64_t*)(w + S.L.tile_off),
                           S.batch ? nullptr : (int64_t*)(w + S.L.params), stream);
    }
    if (e == hipSuccess) {
        const EctArgs a = threshold_args(p, dirs, thresholds, M, thresholds_per_image, out, w, S);
        e = S.batch ? launch_ect_batch(p.ndim, a, stream) : launch_ect(p.ndim, a, S.L.grid, S.direct_groups, radon, stream);
    }
    return from_hip(e);
}

ect_status ect_eval(ect_plan plan, ect_query_set dirs, const double* thresholds, int32_t M,
                    int32_t thresholds_per_image, int32_t* out, void* ws, size_t* ws_bytes, hipStream_t stream) {
    return threshold_eval(plan, dirs, thresholds, M, thresholds_per_image, out, ws, ws_bytes, stream, false);
}

ect_status radon_eval(ect_plan plan, ect_query_set dirs, const double* thresholds, int32_t M,
                      int32_t thresholds_per_image, int32_t* out, void* ws, size_t* ws_bytes, hipStream_t stream) {
    return threshold_eval(plan, dirs, thresholds, M, thresholds_per_image, out, ws, ws_bytes, stream, true);
}

// Arguments of the exact stage common to the layout and the build.
static ExactArgs exact_args(const Plan& p, const ect_query_set& dirs, int32_t kind) {
    ExactArgs a{};
    a.points = (const void*)(p.ws + p.lay.points);
    a.desc = (const ImageDesc*)(p.ws + p.lay.desc);
    a.list_off = (const int64_t*)(p.ws + p.lay.list_off);
    a.list_capacity = p.lay.capacity;
    a.num_images = p.num_images;
    a.NL = num_lists(p.ndim);
    a.vecs = dirs.vecs;
    a.offsets = dirs.offsets;
    a.count = dirs.count;
    a.rows = query_rows(dirs, p.num_images);
    a.kind = kind;
    a.err = (uint32_t*)(p.ws + p.lay.err);
    return a;
}

ect_status ect_exact_layout(ect_plan plan, ect_query_set dirs, int32_t kind, int64_t* row_off, void* ws,
                            size_t* ws_bytes, hipStream_t stream) {
    if (!plan || !ws_bytes || !row_off) return ECT_E_INVALID;
    if (kind != ECT_EXACT_ECT && kind != ECT_EXACT_RADON) return ECT_E_INVALID;
    if (!valid_query_set(dirs, plan->num_images)) return ECT_E_INVALID;
    const Plan& p = *plan;
    const int64_t rows = query_rows(dirs, p.num_images);
    const size_t scan = exact_layout_scan_bytes(rows);
    if (scan == 0) return ECT_E_DEVICE;
    const size_t need_off = 0;
    const size_t scan_off = align_up(sizeof(int64_t) * (size_t)(rows + 1), kAlign);
    const size_t total = scan_off + align_up(scan, kAlign);
    if (!ws) {
        *ws_bytes = total;
        return ECT_OK;
    }
    if (*ws_bytes < total) return ECT_E_NOMEM;
    if ((uintptr_t)ws % kAlign) return ECT_E_INVALID;
    if (plan->last_prep.ws == ws) plan->last_prep.valid = false;
    ExactArgs a = exact_args(p, dirs, kind);
    a.row_off_out = row_off;
    char* w = (char*)ws;
    return from_hip(launch_exact_layout(p.ndim, a, (int64_t*)(w + need_off), w + scan_off, scan, stream));
}

ect_status ect_exact(ect_plan plan, ect_query_set dirs, int32_t kind, const int64_t* row_off, int64_t capacity,
                     double* T, int32_t* E, int64_t* len, void* ws, size_t* ws_bytes, hipStream_t stream) {
    if (!plan || !ws_bytes || !row_off) return ECT_E_INVALID;
    if (kind != ECT_EXACT_ECT && kind != ECT_EXACT_RADON) return ECT_E_INVALID;
    if (!valid_query_set(dirs, plan->num_images)) return ECT_E_INVALID;
    if (capacity < 0) return ECT_E_INVALID;
    if (capacity >= ((int64_t)1 << 32)) return ECT_E_UNSUPPORTED;
    const Plan& p = *plan;
    const int64_t rows = query_rows(dirs, p.num_images);
    if (rows >= ((int64_t)1 << 30)) return ECT_E_UNSUPPORTED;
    if (rows > 0 && (!T || !E || !len)) return ECT_E_INVALID;
    const size_t cap = (size_t)std::max<int64_t>(capacity, 1);
    size_t o = 0;
    const size_t o_ka = o; o = align_up(o + sizeof(uint64_t) * cap, kAlign);
    const size_t o_kb = o; o = align_up(o + sizeof(uint64_t) * cap, kAlign);
    const size_t o_va = o; o = align_up(o + sizeof(int32_t) * cap, kAlign);
    const size_t o_vb = o; o = align_up(o + sizeof(int32_t) * cap, kAlign);
    const size_t o_cum = o; o = align_up(o + (kind == ECT_EXACT_RADON ? sizeof(int32_t) * cap : 0), kAlign);
    const size_t o_ct = o; o = align_up(o + (kind == ECT_EXACT_RADON ? sizeof(double) * cap : 0), kAlign);
    if (!ws) {
        *ws_bytes = o;
        return ECT_OK;
    }
    if (*ws_bytes < o) return ECT_E_NOMEM;
    if ((uintptr_t)ws % kAlign) return ECT_E_INVALID;
    if (plan->last_prep.ws == ws) plan->last_prep.valid = false;
    if (rows == 0) return ECT_OK;
    char* w = (char*)ws;
    ExactArgs a = exact_args(p, dirs, kind);
    a.row_off = row_off;
    a.capacity = capacity;
    a.keys_a = (uint64_t*)(w + o_ka);
    a.keys_b = (uint64_t*)(w + o_kb);
    a.vals_a = (int32_t*)(w + o_va);
    a.vals_b = (int32_t*)(w + o_vb);
    a.cum = kind == ECT_EXACT_RADON ? (int32_t*)(w + o_cum) : nullptr;
    a.ct = kind == ECT_EXACT_RADON ? (double*)(w + o_ct) : nullptr;
    a.T = T;
    a.E = E;
    a.len = len;
    const int64_t max_len = kind == ECT_EXACT_ECT ? max_list(p, 0, num_classical(p.ndim))
                                                  : max_list(p, 0, num_lists(p.ndim));
    return from_hip(launch_exact(p.ndim, a, max_len, stream));
}

ect_status ect_exact_eval(int32_t kind, int64_t rows, const int64_t* row_off, const double* T, const int32_t* E,
                          const int64_t* len, int64_t capacity, const double* thresholds, int32_t M,
                          int32_t thresholds_per_row, int32_t* out, hipStream_t stream) {
    if (kind != ECT_EXACT_ECT && kind != ECT_EXACT_RADON) return ECT_E_INVALID;
    if (rows < 0 || M < 1 || capacity < 0) return ECT_E_INVALID;
    if (rows == 0) return ECT_OK;
    if (!row_off || !T || !E || !len || !thresholds || !out) return ECT_E_INVALID;
    if (rows * (int64_t)((M + 255) / 256) >= ((int64_t)1 << 31)) return ECT_E_UNSUPPORTED;
    return from_hip(launch_exact_eval(kind, rows, row_off, T, E, len, capacity, thresholds, M,
                                      thresholds_per_row ? 1 : 0, out, stream));
}

static ect_status hybrid_common(ect_plan plan, unsigned mask, double s, int32_t precision, ect_query_set xi,
                                double* out_f, double* out_l, double* out_b, double* log_scale,
                                const double* fwd_out, const double* grad_out, double* grad_xi, double* grad_s,
                                void* ws, size_t* ws_bytes, hipStream_t stream, bool backward,
                                bool reuse = false, const EctArgs* combo = nullptr, int64_t combo_groups = 0,
                                const double* s_dev = nullptr) {
    if (!plan || !ws_bytes) return ECT_E_INVALID;
    if (mask == 0 || mask > 7) return ECT_E_INVALID;
    if (backward && (mask & (mask - 1))) return ECT_E_INVALID;
    if (precision != ECT_FP32 && precision != ECT_FP64) return ECT_E_INVALID;
    if (!std::isfinite(s)) return ECT_E_INVALID;
    if (s == 0.0 && backward) return ECT_E_UNSUPPORTED;   // forward only at the constant-kernel limit
    if (!valid_query_set(xi, plan->num_images)) return ECT_E_INVALID;
    const bool empty = query_rows(xi, plan->num_images) == 0;   // outputs of no rows may be NULL
    if (!backward) {
        if (!empty && (((mask & 1) && !out_f) || ((mask & 2) && !out_l) || ((mask & 4) && !out_b)))
            return ECT_E_INVALID;
        if (log_scale && !(mask & 2)) return ECT_E_INVALID;
    } else if (!empty && (!fwd_out || !grad_out || !grad_xi)) {
        return ECT_E_INVALID;
    }
    const Plan& p = *plan;
    EvalLayout L{};
    int64_t chunk = 0;
    layout_hybrid(p, xi, backward, &L, &chunk);
    if (!ws) {
        *ws_bytes = L.total;
        return ECT_OK;
    }
    if (*ws_bytes < L.total) return ECT_E_NOMEM;
    auto& lp = plan->last_prep;
    if (reuse && !(lp.valid && lp.ws == ws && lp.vecs == xi.vecs && lp.offsets == xi.offsets &&
                   lp.count == xi.count && lp.epoch == plan->lists_epoch))
        return ECT_E_INVALID;
    const int64_t rows = query_rows(xi, p.num_images);
    if (rows == 0) {
        // a sum over no rows: d/ds is 0 (a fill kernel, so the call can be captured)
        if (backward && grad_s) return from_hip(launch_fill_u32((uint32_t*)grad_s, 2, 0u, stream));
        return ECT_OK;
    }
    char* w = (char*)ws;
    const int NL = num_lists(p.ndim);
    uint32_t* err = (uint32_t*)(p.ws + p.lay.err);
    const bool shared = xi.offsets == nullptr;
    hipError_t e = hipSuccess;
    // buckets and work list written ahead by ect_plan_rerun_prepare for this
    // workspace and query set, since the last change of the lists
    const bool ahead = !backward && !reuse && lp.ahead && lp.valid && lp.ws == ws && lp.vecs == xi.vecs &&
                       lp.offsets == xi.offsets && lp.count == xi.count && lp.epoch == plan->lists_epoch;
    lp.ahead = false;
    if (!reuse && !ahead) {
        e = launch_prepare(p.ndim, xi, p.num_images, true, err, (void*)(w + L.recs), (int32_t*)(w + L.bcnt),
                           (const int64_t*)(p.ws + p.lay.list_off), num_classical(p.ndim), NL, kHybridTile, chunk,
                           L.capacity, (int64_t*)(w + L.item_off), (int64_t*)(w + L.tile_off),
                           (int64_t*)(w + L.params), stream);
        if (e != hipSuccess) {
            lp.valid = false;
            return ECT_E_DEVICE;
        }
        lp.ws = ws;
        lp.vecs = xi.vecs;
        lp.offsets = xi.offsets;
        lp.count = xi.count;
        lp.epoch = plan->lists_epoch;
        lp.valid = true;
    }
    HybridArgs a{};
    a.points = (const void*)(p.ws + p.lay.points);
    a.list_off = (const int64_t*)(p.ws + p.lay.list_off);
    a.desc = (const ImageDesc*)(p.ws + p.lay.desc);
    a.capacity = p.lay.capacity;
    a.num_images = p.num_images;
    a.NL = NL;
    a.list_base = num_classical(p.ndim);
    a.vecs = xi.vecs;
    a.offsets = xi.offsets;
    a.count = xi.count;
    a.s = s;
    a.s_dev = s_dev;
    a.out_f = out_f;
    a.out_l = out_l;
    a.out_b = out_b;
    a.log_scale = log_scale;
    a.fwd_out = fwd_out;
    a.grad_out = grad_out;
    a.recs = (const void*)(w + L.recs);
    a.bcnt = (const int32_t*)(w + L.bcnt);
    a.item_off = (const int64_t*)(w + L.item_off);
    a.tile_off = (const int64_t*)(w + L.tile_off);
    a.params = (const int64_t*)(w + L.params);
    a.tile_ent = (int32_t*)(w + L.tile_ent);
    a.partials = (double*)(w + L.partials);
    a.err = err;
    // s = 0: every requested output is the constant-kernel limit sum D <xi, x>
    if (!backward && combo) {
        // the shared-set ECT workgroups run in the launch of the hybrid work
        // items; then the ECT chunk sums and the hybrid reduction
        const int64_t ect_blocks = combo_groups * p.num_images * combo->chunks;
        e = launch_ect_hybrid(p.ndim, mask, precision, a, *combo, L.grid, ect_blocks, combo_groups, stream);
        if (e == hipSuccess) e = launch_ect_chunk_sum(*combo, ect_blocks, combo_groups, stream);
        if (e == hipSuccess) e = launch_hybrid(p.ndim, mask, precision, false, a, 0, L.tiles, stream);
        return from_hip(e);
    }
    if (!backward)
        return from_hip(launch_hybrid(p.ndim, s == 0.0 ? kHybridLinear : mask, precision, false, a, L.grid, L.tiles,
                                      stream));
    double* gpart = (double*)(w + L.gpart);
    a.grad_xi = shared ? gpart : grad_xi;
    a.grad_s_part = (double*)(w + L.gspart);
    e = launch_hybrid(p.ndim, mask, precision, true, a, L.grid, L.tiles, stream);
    if (e == hipSuccess)
        e = launch_grad_reduce(p.ndim, gpart, p.num_images, xi.count, shared, grad_xi, a.grad_s_part, rows,
                               grad_s, stream);
    return from_hip(e);
}

static double* kernel_out(int32_t kernel, int32_t which, double* out) { return kernel == which ? out : nullptr; }

ect_status hybrid_eval(ect_plan plan, int32_t kernel, double s, int32_t precision, ect_query_set xi, double* out,
                       double* log_scale, void* ws, size_t* ws_bytes, hipStream_t stream) {
    if (kernel < ECT_FOURIER || kernel > ECT_BESSEL || !out) return ECT_E_INVALID;
    return hybrid_common(plan, 1u << kernel, s, precision, xi, kernel_out(kernel, ECT_FOURIER, out),
                         kernel_out(kernel, ECT_LAPLACE, out), kernel_out(kernel, ECT_BESSEL, out), log_scale,
                         nullptr, nullptr, nullptr, nullptr, ws, ws_bytes, stream, false);
}

ect_status hybrid_eval_noalloc(ect_plan plan, int32_t kernel, double s, int32_t precision, ect_query_set xi,
                               double* out, double* log_scale, hipStream_t stream) {
    if (!plan) return ECT_E_INVALID;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return ECT_E_DEVICE;
    if (dev != plan->device) return ECT_E_INVALID;
    // argument checks and the workspace size, as hybrid_eval makes them
    size_t need = 0;
    ect_status st = hybrid_eval(plan, kernel, s, precision, xi, out, log_scale, nullptr, &need, stream);
    if (st != ECT_OK) return st;
    if (need > ECT_NOALLOC_SCRATCH_BYTES) return ECT_E_SCRATCH;
    void* ws = nullptr;
    st = scratch_address(dev, &ws);
    if (st != ECT_OK) return st;
    size_t have = ECT_NOALLOC_SCRATCH_BYTES;
    return hybrid_eval(plan, kernel, s, precision, xi, out, log_scale, ws, &have, stream);
}

ect_status hybrid_eval_multi(ect_plan plan, uint32_t kernel_mask, double s, int32_t precision, ect_query_set xi,
                             double* out_fourier, double* out_laplace, double* out_bessel, double* log_scale_laplace,
                             void* ws, size_t* ws_bytes, hipStream_t stream) {
    return hybrid_common(plan, kernel_mask, s, precision, xi, out_fourier, out_laplace, out_bessel,
                         log_scale_laplace, nullptr, nullptr, nullptr, nullptr, ws, ws_bytes, stream, false);
}

ect_status hybrid_eval_multi_s(ect_plan plan, uint32_t kernel_mask, const double* s, int32_t precision,
                               ect_query_set xi, double* out_fourier, double* out_laplace, double* out_bessel,
                               double* log_scale_laplace, void* ws, size_t* ws_bytes, hipStream_t stream) {
    if (!s) return ECT_E_INVALID;
    // the host sees a nonzero placeholder: the constant-kernel limit is not taken with a device scale
    return hybrid_common(plan, kernel_mask, 1.0, precision, xi, out_fourier, out_laplace, out_bessel,
                         log_scale_laplace, nullptr, nullptr, nullptr, nullptr, ws, ws_bytes, stream, false, false,
                         nullptr, 0, s);
}

ect_status hybrid_eval_backward_s(ect_plan plan, int32_t kernel, const double* s, int32_t precision,
                                  ect_query_set xi, const double* out, const double* grad_out, double* grad_xi,
                                  double* grad_s, uint32_t flags, void* ws, size_t* ws_bytes, hipStream_t stream) {
    if (!s) return ECT_E_INVALID;
    if (kernel < ECT_FOURIER || kernel > ECT_BESSEL) return ECT_E_INVALID;
    if (flags & ~(uint32_t)ECT_BWD_REUSE_PREPARED) return ECT_E_INVALID;
    return hybrid_common(plan, 1u << kernel, 1.0, precision, xi, nullptr, nullptr, nullptr, nullptr, out, grad_out,
                         grad_xi, grad_s, ws, ws_bytes, stream, true, (flags & ECT_BWD_REUSE_PREPARED) != 0, nullptr,
                         0, s);
}

ect_status ect_hybrid_eval_multi(ect_plan plan, ect_query_set dirs, const double* thresholds, int32_t M,
                                 int32_t thresholds_per_image, int32_t* ect_out, uint32_t kernel_mask, double s,
                                 int32_t precision, ect_query_set xi, double* out_fourier, double* out_laplace,
                                 double* out_bessel, double* log_scale_laplace, void* ws, size_t* ws_bytes,
                                 hipStream_t stream) {
    if (!plan || !ws_bytes) return ECT_E_INVALID;
    const Plan& p = *plan;
    ThresholdSetup S;
    ect_status st = threshold_setup(p, dirs, thresholds, M, ect_out, false, &S);
    if (st != ECT_OK) return st;
    // the hybrid part (its validation and size) at the start of the workspace,
    // so that a backward call given the same workspace can reuse its buckets
    size_t hyb = 0;
    st = hybrid_common(plan, kernel_mask, s, precision, xi, out_fourier, out_laplace, out_bessel, log_scale_laplace,
                       nullptr, nullptr, nullptr, nullptr, nullptr, &hyb, stream, false);
    if (st != ECT_OK) return st;
    const size_t ect_off = align_up(hyb, kAlign);
    const size_t total = ect_off + S.L.total;
    if (!ws) {
        *ws_bytes = total;
        return ECT_OK;
    }
    if (*ws_bytes < total) return ECT_E_NOMEM;
    char* w = (char*)ws;
    // one launch for a shared direction set whose thresholds and histograms
    // fit kComboEctLds bytes of LDS (every workgroup of the launch reserves
    // them, the hybrid ones included, so more would cost them occupancy)
    const size_t ect_lds = (sizeof(double) + sizeof(int32_t) * (size_t)S.td) * (size_t)M;
    const bool one_launch = S.direct && S.td <= kComboEctDirs && ect_lds <= kComboEctLds && s != 0.0 &&
                            query_rows(dirs, p.num_images) > 0 && query_rows(xi, p.num_images) > 0;
    if (!one_launch) {
        size_t eb = S.L.total;
        st = threshold_eval(plan, dirs, thresholds, M, thresholds_per_image, ect_out, w + ect_off, &eb, stream, false);
        if (st != ECT_OK) return st;
        return hybrid_common(plan, kernel_mask, s, precision, xi, out_fourier, out_laplace, out_bessel,
                             log_scale_laplace, nullptr, nullptr, nullptr, nullptr, ws, &hyb, stream, false);
    }
    const EctArgs ea = threshold_args(p, dirs, thresholds, M, thresholds_per_image, ect_out, w + ect_off, S);
    return hybrid_common(plan, kernel_mask, s, precision, xi, out_fourier, out_laplace, out_bessel, log_scale_laplace,
                         nullptr, nullptr, nullptr, nullptr, ws, &hyb, stream, false, false, &ea, S.direct_groups);
}

ect_status hybrid_eval_backward(ect_plan plan, int32_t kernel, double s, int32_t precision, ect_query_set xi,
                                const double* out, const double* grad_out, double* grad_xi, double* grad_s,
                                uint32_t flags, void* ws, size_t* ws_bytes, hipStream_t stream) {
    if (kernel < ECT_FOURIER || kernel > ECT_BESSEL) return ECT_E_INVALID;
    if (flags & ~(uint32_t)ECT_BWD_REUSE_PREPARED) return ECT_E_INVALID;
    return hybrid_common(plan, 1u << kernel, s, precision, xi, nullptr, nullptr, nullptr, nullptr, out, grad_out,
                         grad_xi, grad_s, ws, ws_bytes, stream, true, (flags & ECT_BWD_REUSE_PREPARED) != 0);
}

ect_status ect_plan_counts(ect_plan plan, int64_t* classical, int64_t* ordinary) {
    if (!plan) return ECT_E_INVALID;
    const int n = plan->ndim, NL = num_lists(n), NC = num_classical(n), NO = num_ordinary(n);
    for (int i = 0; i < plan->num_images; ++i) {
        const int64_t* a = plan->h_list_off + (int64_t)i * NL;
        const int64_t* b = a + NL;
        for (int l = 0; l < NC; ++l)
            if (classical) classical[(int64_t)i * NC + l] = b[l] - a[l];
        for (int l = 0; l < NO; ++l)
            if (ordinary) ordinary[(int64_t)i * NO + l] = b[NC + l] - a[NC + l];
    }
    return ECT_OK;
}

ect_status ect_plan_export(ect_plan plan, int32_t image, int32_t kind, int32_t list, int32_t* coords,
                           int32_t* values, int64_t capacity, int64_t* count, hipStream_t stream) {
    if (!plan || !count || capacity < 0) return ECT_E_INVALID;
    const Plan& p = *plan;
    const int n = p.ndim, NL = num_lists(n);
    if (image < 0 || image >= p.num_images) return ECT_E_INVALID;
    if (kind != 0 && kind != 1) return ECT_E_INVALID;
    const int nlist = kind == 0 ? num_classical(n) : num_ordinary(n);
    if (list < 0 || list >= nlist) return ECT_E_INVALID;
    if (capacity > 0 && (!coords || !values)) return ECT_E_INVALID;
    const int l = (kind == 0 ? 0 : num_classical(n)) + list;
    int64_t off[2];
    hipError_t e = hipMemcpyAsync(&off[0], p.ws + p.lay.list_off + sizeof(int64_t) * ((int64_t)image * NL + l),
                                  sizeof(int64_t), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&off[1], p.ws + p.lay.list_off + sizeof(int64_t) * ((int64_t)(image + 1) * NL + l),
                           sizeof(int64_t), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return ECT_E_DEVICE;
    const int64_t cnt = off[1] - off[0];
    *count = cnt;
    const int64_t take = std::min(cnt, capacity);
    if (take <= 0) return ECT_OK;
    const size_t pb = entry_bytes();
    std::vector<ListEntry> buf;
    try {
        buf.resize((size_t)take);
    } catch (...) {
        return ECT_E_NOMEM;
    }
    e = hipMemcpyAsync(buf.data(), p.ws + p.lay.points + pb * ((int64_t)l * p.lay.capacity + off[0]), pb * take,
                       hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return ECT_E_DEVICE;
    const ImageDesc& d = p.h_desc[image];
    for (int64_t k = 0; k < take; ++k) {
        for (int a = 0; a < n; ++a) coords[k * n + a] = (int32_t)((buf[(size_t)k].code >> d.kshift[a]) & d.kmask[a]);
        values[k] = buf[(size_t)k].val;
    }
    return ECT_OK;
}

ect_status ect_plan_check(ect_plan plan, uint32_t* flags, hipStream_t stream) {
    if (!plan || !flags) return ECT_E_INVALID;
    uint32_t v = 0;
    hipError_t e = hipMemcpyAsync(&v, plan->ws + plan->lay.err, sizeof(uint32_t), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    const uint32_t zero = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(plan->ws + plan->lay.err, &zero, sizeof(uint32_t), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return ECT_E_DEVICE;
    *flags = v;
    return ECT_OK;
}

ect_status ect_plan_destroy(ect_plan plan) {
    if (!plan) return ECT_E_INVALID;
    delete[] plan->h_desc;
    delete[] plan->h_list_off;
    delete plan;
    return ECT_OK;
}

ect_status ect_plan_set_tuning(ect_plan plan, int64_t hybrid_chunk, int64_t hybrid_target_items,
                               int32_t ect_dirs_per_group, int32_t ect_chunks) {
    if (!plan) return ECT_E_INVALID;
    if (hybrid_chunk < 0 || (hybrid_chunk > 0 && hybrid_chunk < 16) || hybrid_chunk > (int64_t(1) << 40) ||
        hybrid_target_items < 1 || hybrid_target_items > (int64_t(1) << 24) || ect_dirs_per_group < 0 ||
        ect_dirs_per_group > kEctMaxDirs || ect_chunks < 0 || ect_chunks > 4096)
        return ECT_E_INVALID;
    ++plan->lists_epoch;
    plan->tune_hybrid_chunk = hybrid_chunk;
    plan->tune_hybrid_target_items = hybrid_target_items;
    plan->tune_ect_dirs_per_group = ect_dirs_per_group;
    plan->tune_ect_chunks = ect_chunks;
    return ECT_OK;
}

ect_status ect_set_stage_events(int32_t stage, hipEvent_t before, hipEvent_t after) {
    if (stage < 0 || stage > 3) return ECT_E_INVALID;
    g_stage_events[stage].before = before;
    g_stage_events[stage].after = after;
    return ECT_OK;
}

}  // extern "C"
