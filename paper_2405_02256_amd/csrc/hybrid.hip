// Hybrid transforms HT(xi) = sum over ordinary points of Delta^ord(eps,x) kbar_s(<xi,x>)
// and their vector-Jacobian products (gfx950).
//
// The hybrid transform is the integral of kappa against the Radon transform
// (Sec. 2.2); by Lemma 3.1 it only needs the ordinary critical points of the
// query's sign vector and the primitive kbar of the kernel.  The sign used
// here is the one the definition gives (a closed square yields
// kbar(max) - kbar(min)).
//
// Several kernels can be evaluated in one pass (a bit mask of Fourier,
// Laplace, Bessel): they share the staged points and the projection <xi, x>.
//
// Work decomposition: queries are bucketed by orthant pair; a work item is
// (image, pair, tile of 64 queries, chunk of points).  One workgroup of four
// waves runs an item: every lane owns one query held in registers, the chunk's
// points are staged through LDS and the four waves take every fourth point.
// Per pair of (query, point):
//   FP32 precision: FP64 phase, FP64 argument reduction to [0, 1) revolutions
//                   (or to a split exponent for Laplace), FP32 kernel value
//                   (hardware sin/cos/exp2 on reduced arguments, polynomial
//                   Ji0), FP64 accumulation;
//   FP64 precision: every step in FP64.
// Items of a tile split over several chunks write per-query partial sums,
// which a second kernel adds in chunk order, so results are bitwise
// reproducible (a kernel boundary is the cheap synchronisation point between
// the chip's non-coherent L2 slices).
#include "ect_body.h"
#include "eval_internal.h"
#include "ji0_coeffs.h"

namespace ect {

namespace {

constexpr double kInv2Pi = 0.15915494309189535;
constexpr double kLog2E = 1.4426950408889634;
constexpr double kLn2 = 0.6931471805599453;
constexpr int kAccSlots = 5;      // doubles per lane in a partial record (slot 4: Laplace shift)
constexpr int kSlotShift = 4;

// Laplace terms exp(-s u) are summed relative to 2^m2 (an integer shift per
// query): term = exp(-s u - m2 ln 2).  The shift follows the running maximum
// of the exponents lazily: it starts at the first point of the item's chunk,
// and a term more than 2^kShiftSlack above it moves it up to that term (the
// sums so far are scaled by an exact power of two).  So no term overflows,
// the largest term of the list is at least 1/2, and partial sums with
// different shifts combine exactly.
constexpr double kShiftSlack = 256.0;   // log2 units
constexpr double kShiftClamp = 1.0e9;   // keeps shifts finite (NaN and huge exponents)

// x * 2^e for an integer-valued e <= 0 or > 0, saturating (|e| beyond the
// FP64 exponent range gives 0 or inf as the product would).
__device__ __forceinline__ double scale2(double x, double e) {
    return ldexp(x, (int)fmin(fmax(e, -4096.0), 4096.0));
}

__device__ __forceinline__ double clamp_shift(double m) { return fmin(fmax(m, -kShiftClamp), kShiftClamp); }

template <int D, typename T>
__device__ __forceinline__ T horner(const double (&c)[D], T x) {
    T r = (T)c[D - 1];
#pragma unroll
    for (int k = D - 2; k >= 0; --k) r = r * x + (T)c[k];
    return r;
}

// sin(2 pi r), cos(2 pi r) for r in [0, 1] (hardware units take revolutions)
__device__ __forceinline__ void sincos_rev_f32(float r, float* sn, float* cs) {
    *sn = __builtin_amdgcn_sinf(r);
    *cs = __builtin_amdgcn_cosf(r);
}

static_assert(JI0_F32_SMALL_DEG + 1 == kJi0SmallCoeffs, "kernel-argument copy of the Ji0 coefficients");

// Horner on coefficients held in scalar registers (the kernel-argument copy):
// FP64 FMAs take them directly as their addend, where literal coefficients
// would be copied into a vector register before every FMA.
template <int D>
__device__ __forceinline__ double horner_sgpr(const double* c, double x) {
    double r = c[D - 1];
#pragma unroll
    for (int k = D - 2; k >= 0; --k) r = fma(r, x, c[k]);
    return r;
}

// Ji0(z) = integral_0^z J0 in FP32 (coefficients fitted against mpmath).
__device__ __forceinline__ float ji0_f32(double z, const double* small_coeffs) {
    const double az = fabs(z);
    float r;
    if (az < JI0_Z0) {
        // the monomial coefficients alternate in sign up to ~16 in size, so the
        // polynomial is evaluated in FP64 (same issue rate as FP32 on this chip)
        const double v = az * az * (1.0 / (JI0_Z0 * JI0_Z0));
        r = (float)(az * horner_sgpr<JI0_F32_SMALL_DEG + 1>(small_coeffs, v));
    } else {
        const float zf = (float)az;
        const float rs = __builtin_amdgcn_rsqf(zf);   // z^-1/2; z^-1 = rs^2
        const float rz = rs * rs;
        const float w = (float)(JI0_Z0 * JI0_Z0) * rz * rz;
        const float A = horner<JI0_F32_TAILA_DEG + 1, float>(JI0_F32_TAILA, w);
        const float Bv = horner<JI0_F32_TAILB_DEG + 1, float>(JI0_F32_TAILB, w);
        const float rf = (float)__builtin_amdgcn_fract(fma(az, kInv2Pi, -0.125));
        float sn, cs;
        sincos_rev_f32(rf, &sn, &cs);
        const float amp = 0.79788456080286536f * rs;
        r = 1.0f - amp * (A * rz * cs + Bv * sn);
    }
    return z < 0.0 ? -r : r;
}

__device__ __forceinline__ double ji0_f64(double z) {
    const double az = fabs(z);
    double r;
    if (az < JI0_Z0) {
        const double v = az * az * (1.0 / (JI0_Z0 * JI0_Z0));
        r = az * horner<JI0_F64_SMALL_DEG + 1, double>(JI0_F64_SMALL, v);
    } else {
        const double rz = 1.0 / az;
        const double w = JI0_Z0 * JI0_Z0 * rz * rz;
        const double A = horner<JI0_F64_TAILA_DEG + 1, double>(JI0_F64_TAILA, w);
        const double Bv = horner<JI0_F64_TAILB_DEG + 1, double>(JI0_F64_TAILB, w);
        const double rev = az * kInv2Pi - 0.125;
        const double fr = rev - rint(rev);
        double sn, cs;
        sincospi(2.0 * fr, &sn, &cs);
        r = 1.0 - sqrt(2.0 / (M_PI * az)) * (A * rz * cs + Bv * sn);
    }
    return z < 0.0 ? -r : r;
}

// FP32 value of exp2(a) for a <= 0 as a double: a = n + f with f in [0, 1),
// exp2(f) in FP32, then an exact scaling by 2^n in FP64.
__device__ __forceinline__ double exp2_split(double a) {
    const double n = floor(a);
    const float f = (float)(a - n);
    const double e = (double)__builtin_amdgcn_exp2f(f);
    // v_cvt_i32_f64 saturates (NaN gives 0), and ldexp of INT_MIN underflows
    // to 0, so exponents below the int range need no clamp
    return ldexp(e, (int)n);
}

// Per-thread query state.
template <int N>
struct Query {
    double xi[N];     // direction
    double cF;        // Fourier: revolutions per unit of <xi,x>, s / (2 pi)
    double cL, mL;    // Laplace: exponent = cL <xi,x> - mL (FP32: log2 units, mL = m2; FP64: mL = m2 ln 2)
    double m2;        // Laplace: current shift, an integer in log2 units
    double cB;        // Bessel: z = s <xi,x>
    double gr, gi;    // backward: output cotangent
    double sigma;     // +1, or -1 when the query's list is the pair's mirror
};

constexpr int kF = 1 << ECT_FOURIER, kL = 1 << ECT_LAPLACE, kB = 1 << ECT_BESSEL, kLin = (int)kHybridLinear;
// accumulator slots: Fourier 0-1, Laplace 2, Bessel 3; backward: 0..n-1
constexpr int kSlotF = 0, kSlotL = 2, kSlotB = 3;

// Contribution of one point.  Forward: per requested kernel, sum of D kbar(s u)
// (without the 1/s); backward (one kernel): acc[a] = sum of D x_a g(kappa).
// Whether accumulator slot k holds a Laplace sum (scaled by 2^-m2).
template <int MASK, bool BWD, int N>
__host__ __device__ constexpr bool lap_slot(int k) {
    if (BWD) return MASK == kL && k < N;
    return (MASK & kL) && k == kSlotL;
}

// Shift of the Laplace exponent in the kernel's units.
template <int PREC>
__device__ __forceinline__ double shift_units(double m2) { return PREC == ECT_FP32 ? m2 : m2 * kLn2; }

// Move the Laplace shift up to exponent `ex` (kernel units, ex > 0 relative
// to the current shift): the sums so far are scaled by an exact power of two.
template <int N, int MASK, int PREC, bool BWD>
__device__ __forceinline__ void raise_shift(Query<N>& q, double* acc, double ex) {
    const double d = ceil(PREC == ECT_FP32 ? ex : ex * kLog2E);
    q.m2 = clamp_shift(q.m2 + d);
    q.mL = shift_units<PREC>(q.m2);
#pragma unroll
    for (int k = 0; k < kAccSlots; ++k)
        if (lap_slot<MASK, BWD, N>(k)) acc[k] = scale2(acc[k], -d);
}

// Start the Laplace shift of a work item at its chunk's first point.
template <int N, int PREC>
__device__ __forceinline__ void init_shift(Query<N>& q, const PointT<N>& pt) {
    double u = q.xi[0] * pt.x[0];
#pragma unroll
    for (int a = 1; a < N; ++a) u = fma(q.xi[a], pt.x[a], u);
    const double c2 = PREC == ECT_FP32 ? q.cL : q.cL * kLog2E;   // log2 units
    q.m2 = clamp_shift(ceil(u * c2));
    q.mL = shift_units<PREC>(q.m2);
}

template <int N, int MASK, int PREC, bool BWD>
__device__ __forceinline__ void accumulate_point(const PointT<N>& pt, Query<N>& q, double* acc,
                                                 const double* ji0c) {
    double u = q.xi[0] * pt.x[0];
#pragma unroll
    for (int a = 1; a < N; ++a) u = fma(q.xi[a], pt.x[a], u);
    if constexpr (MASK == kLin) acc[0] = fma(pt.val, u, acc[0]);
    if constexpr ((MASK & kF) != 0) {
        const double ph = u * q.cF;
        double sn, cs;
        if constexpr (PREC == ECT_FP32) {
            float s32, c32;
            sincos_rev_f32((float)__builtin_amdgcn_fract(ph), &s32, &c32);   // fract is exact
            sn = (double)s32;
            cs = (double)c32;
        } else {
            sincospi(2.0 * (ph - rint(ph)), &sn, &cs);
        }
        if constexpr (!BWD) {
            acc[kSlotF] = fma(pt.val, sn, acc[kSlotF]);
            acc[kSlotF + 1] = fma(pt.val, cs, acc[kSlotF + 1]);
        } else {
            // kappa(s u) = exp(-i s u): d Re/d xi_a = x cos, d Im/d xi_a = -x sin
            const double g = pt.val * (q.gr * cs - q.gi * sn);
#pragma unroll
            for (int a = 0; a < N; ++a) acc[a] = fma(g, pt.x[a], acc[a]);
        }
    }
    if constexpr ((MASK & kL) != 0) {
        constexpr double slack = PREC == ECT_FP32 ? kShiftSlack : kShiftSlack * kLn2;
        double ex = fma(u, q.cL, -q.mL);
        // one compare per pair; the wave branches only when some lane's shift
        // must move (rarely: at most once per factor 2^256 of its terms)
        const uint64_t over = __builtin_amdgcn_ballot_w64(ex > slack);
        if (over != 0) {
            if ((over >> __lane_id()) & 1) {
                raise_shift<N, MASK, PREC, BWD>(q, acc, ex);
                ex = fma(u, q.cL, -q.mL);
            }
        }
        const double term = (PREC == ECT_FP32) ? exp2_split(ex) : exp(ex);
        if constexpr (!BWD) {
            acc[kSlotL] = fma(pt.val, term, acc[kSlotL]);
        } else {
            const double g = pt.val * term;
#pragma unroll
            for (int a = 0; a < N; ++a) acc[a] = fma(g, pt.x[a], acc[a]);
        }
    }
    if constexpr ((MASK & kB) != 0) {
        const double z = u * q.cB;
        if constexpr (!BWD) {
            const double ji = (PREC == ECT_FP32) ? (double)ji0_f32(z, ji0c) : ji0_f64(z);
            acc[kSlotB] = fma(pt.val, ji, acc[kSlotB]);
        } else {
            const double j = (PREC == ECT_FP32) ? (double)j0f((float)z) : j0(z);
            const double g = pt.val * j;
#pragma unroll
            for (int a = 0; a < N; ++a) acc[a] = fma(g, pt.x[a], acc[a]);
        }
    }
}

template <int MASK, bool BWD, int N>
__host__ __device__ constexpr bool slot_used(int k) {
    if (k == kSlotShift) return BWD ? MASK == kL : (MASK & kL) != 0 && MASK != kLin;
    if (BWD) return k < N;
    if (MASK == kLin) return k == 0;
    return ((MASK & kF) && (k == 0 || k == 1)) || ((MASK & kL) && k == 2) || ((MASK & kB) && k == 3);
}

// Add the sums of another part (its own Laplace shift m2o) into acc (shift
// q.m2): both are brought to the larger shift by exact powers of two.
template <int N, int MASK, int PREC, bool BWD>
__device__ __forceinline__ void add_part(Query<N>& q, double* acc, const double* other, double m2o) {
    if constexpr (slot_used<MASK, BWD, N>(kSlotShift)) {
        const double m = fmax(q.m2, m2o);
#pragma unroll
        for (int k = 0; k < kAccSlots; ++k)
            if (lap_slot<MASK, BWD, N>(k)) acc[k] = scale2(acc[k], q.m2 - m) + scale2(other[k], m2o - m);
        q.m2 = m;
        q.mL = shift_units<PREC>(m);
    }
#pragma unroll
    for (int k = 0; k < kAccSlots; ++k)
        if (slot_used<MASK, BWD, N>(k) && k != kSlotShift && !lap_slot<MASK, BWD, N>(k)) acc[k] += other[k];
}

// The kernel scale: the call's argument, or read from device memory (a
// learnable scale in a captured graph); a device scale that is zero or not
// finite raises ECT_DEVERR_SCALE (the outputs are then not finite).
__device__ __forceinline__ double scale_of(const HybridArgs& a) {
    if (!a.s_dev) return a.s;
    const double s = *a.s_dev;
    if (!(isfinite(s) && s != 0.0) && threadIdx.x == 0) raise_error(a.err, ECT_DEVERR_SCALE);
    return s;
}

// Laplace alone, FP32 forward: the exponent of a pair is <c xi, x> - mL with
// the direction pre-scaled by the kernel factor c (one fma per axis), and
// the points of one wave are taken G at a time: when no lane's group needs
// the shift raised (the common case, one compare per group) the G terms are
// summed without a branch, else one point after another as accumulate_point
// does.  The sums take each lane's points in the same order either way.
template <int N>
__device__ __forceinline__ double lap_exponent(const PointT<N>& pt, const double (&cx)[N], double mL) {
    double e = fma(pt.x[0], cx[0], -mL);
#pragma unroll
    for (int a = 1; a < N; ++a) e = fma(pt.x[a], cx[a], e);
    return e;
}

template <int N>
__device__ __forceinline__ void lap_point_slow(const PointT<N>& pt, const double (&cx)[N], Query<N>& q, double* acc) {
    double ex = lap_exponent<N>(pt, cx, q.mL);
    if (ex > kShiftSlack) {
        raise_shift<N, kL, ECT_FP32, false>(q, acc, ex);
        ex = lap_exponent<N>(pt, cx, q.mL);
    }
    acc[kSlotL] = fma(pt.val, exp2_split(ex), acc[kSlotL]);
}

template <int N>
__device__ __forceinline__ void laplace_stage_f32(const PointT<N>* s_pts, int k0, int cnt, const double (&cx)[N],
                                                  Query<N>& q, double* acc) {
    constexpr int G = 4;
    int k = k0;
    for (; k + (G - 1) * kHybridSplit < cnt; k += G * kHybridSplit) {
        double ex[G], v[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const PointT<N>& pt = s_pts[k + g * kHybridSplit];
            ex[g] = lap_exponent<N>(pt, cx, q.mL);
            v[g] = pt.val;
        }
        const double mx = fmax(fmax(ex[0], ex[1]), fmax(ex[2], ex[3]));
        if (__builtin_amdgcn_ballot_w64(mx > kShiftSlack) == 0) {
#pragma unroll
            for (int g = 0; g < G; ++g) acc[kSlotL] = fma(v[g], exp2_split(ex[g]), acc[kSlotL]);
        } else {
            for (int g = 0; g < G; ++g) lap_point_slow<N>(s_pts[k + g * kHybridSplit], cx, q, acc);
        }
    }
    for (; k < cnt; k += kHybridSplit) lap_point_slow<N>(s_pts[k], cx, q, acc);
}

// Per-query set-up shared by the evaluation and reduction kernels.
template <int N, int MASK, int PREC, bool BWD>
__device__ __forceinline__ void setup_query(const HybridArgs& a, int64_t img, int b, int64_t qi, bool active,
                                            Query<N>& q, int64_t& row) {
    constexpr int P = 1 << (N - 1);
    const bool shared_q = a.offsets == nullptr;
    const int64_t row_base = shared_q ? img * a.count : a.offsets[img];
    row = 0;
    q.sigma = 1.0;
    q.gr = q.gi = 0.0;
    const double s = scale_of(a);
    if (active) {
        const QRecT<N> r = ((const QRecT<N>*)a.recs)[bucket_start(a.offsets, a.count, img, P, b) + qi];
        row = row_base + (r.code >> 1);
        q.sigma = (r.code & 1) ? -1.0 : 1.0;
#pragma unroll
        for (int k = 0; k < N; ++k) q.xi[k] = r.v[k];
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) q.xi[k] = 0.0;
    }
    q.cF = s * kInv2Pi;
    q.cB = s;
    q.cL = (PREC == ECT_FP32) ? -s * kLog2E : -s;
    q.mL = 0.0;
    q.m2 = 0.0;
    if constexpr (BWD) {
        if (active) {
            if (MASK == kF) {
                q.gr = a.grad_out[row * 2];
                q.gi = a.grad_out[row * 2 + 1];
            } else {
                q.gr = a.grad_out[row];
            }
        }
    }
}

// Scale the point sums of one query into its outputs.
template <int N, int MASK, int PREC, bool BWD>
__device__ __forceinline__ void finalize(const HybridArgs& a, const Query<N>& q, int64_t row, const double* acc) {
    const double s = scale_of(a);
    if constexpr (MASK == kLin) {
        const double v = q.sigma * acc[0];
        if (a.out_f) {
            a.out_f[row * 2] = v;
            a.out_f[row * 2 + 1] = 0.0;
        }
        if (a.out_l) {
            a.out_l[row] = v;
            if (a.log_scale) a.log_scale[row] = 0.0;
        }
        if (a.out_b) a.out_b[row] = v;
    } else if constexpr (!BWD) {
        if constexpr ((MASK & kF) != 0) {
            a.out_f[row * 2] = q.sigma * acc[kSlotF] / s;
            a.out_f[row * 2 + 1] = q.sigma * acc[kSlotF + 1] / s;
        }
        if constexpr ((MASK & kL) != 0) {
            const double shifted = -q.sigma * acc[kSlotL] / s;
            if (a.log_scale) {
                a.out_l[row] = shifted;
                a.log_scale[row] = q.m2 * kLn2;
            } else {
                const double v = scale2(shifted, q.m2);   // exact; inf only when HT itself overflows
                if (!isfinite(v)) raise_error(a.err, ECT_DEVERR_OVERFLOW);
                a.out_l[row] = v;
            }
        }
        if constexpr ((MASK & kB) != 0) a.out_b[row] = q.sigma * acc[kSlotB] / s;
    } else {
        // G_a = sigma * sum D x_a (weighted kappa); Laplace sums carry 2^-m2
        double scale = q.sigma;
        if constexpr (MASK == kL || MASK == kB) scale *= q.gr;
        double dots = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const double G = (MASK == kL) ? scale2(scale * acc[k], q.m2) : scale * acc[k];
            a.grad_xi[row * N + k] = G;
            dots = fma(q.xi[k], G, dots);
        }
        double gy;
        if constexpr (MASK == kF) gy = q.gr * a.fwd_out[row * 2] + q.gi * a.fwd_out[row * 2 + 1];
        else gy = q.gr * a.fwd_out[row];
        a.grad_s_part[row] = (dots - gy) / s;
    }
}

// Locate the entry (image, pair) of a work item or query tile by binary search
// over a non-decreasing prefix array (the last entry whose start is <= idx).
__device__ __forceinline__ int64_t find_entry(const int64_t* __restrict__ off, int64_t E, int64_t idx) {
    int64_t lo = 0, hi = E - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= idx) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Partial sums are stored slot-major inside an item so that consecutive
// threads touch consecutive doubles.
__device__ __forceinline__ int64_t partial_index(int64_t item, int slot, int q) {
    return (item * kAccSlots + slot) * kHybridTile + q;
}

// One workgroup per work item (image, orthant pair, tile of 64 queries, chunk
// of points).  The chunk's points are staged in LDS kHybridStage at a time with
// one coalesced load per thread; wave w of the four then reads the staged
// points w, w+4, ... (the same address across the wave: a broadcast) for the
// tile's 64 queries, one query per lane.  The four wave sums of a query are
// added in wave order.  A tile split into several chunks writes per-query
// partial sums, which hybrid_reduce adds in chunk order after the kernel; a
// single-chunk tile writes its outputs here.
template <int N, int MASK, int PREC, bool BWD>
__device__ __forceinline__ void hybrid_block(const HybridArgs& a, int64_t item) {
    constexpr int P = 1 << (N - 1);
    __shared__ PointT<N> s_pts[kHybridStage];
    __shared__ double s_acc[kHybridSplit - 1][kAccSlots][kHybridTile];
    const int tid = threadIdx.x;
    const int lane = tid & (kHybridTile - 1);
    const int wave = tid / kHybridTile;
    if (item >= a.params[0]) return;
    const int64_t C = a.params[2];
    const int64_t e = find_entry(a.item_off, (int64_t)a.num_images * P, item);
    const int64_t img = e / P;
    const int b = (int)(e % P);
    const int64_t local = item - a.item_off[e];
    const int l = a.list_base + b;
    const int64_t p0 = a.list_off[img * a.NL + l], p1 = a.list_off[(img + 1) * a.NL + l];
    const int64_t np = p1 - p0;
    const int64_t chunks = np > 0 ? (np + C - 1) / C : 1;
    const int64_t t = local / chunks, c = local % chunks;
    const int64_t qn = a.bcnt[a.offsets == nullptr ? b : e];
    const int64_t qi = t * kHybridTile + lane;
    const bool active = qi < qn;
    // the tile's first chunk tells the reduction which entry the tile belongs to
    const int64_t tslot = (c == 0 && tid == 0) ? a.tile_off[e] + t : -1;
    const ListEntry* __restrict__ pts = list_entries(a.points, a.capacity, l);
    const ImageDesc& d = a.desc[img];
    const int64_t c0 = p0 + c * C, c1 = min(p1, c0 + C);

    Query<N> q;
    int64_t row;
    setup_query<N, MASK, PREC, BWD>(a, img, b, qi, active, q, row);
    if constexpr (slot_used<MASK, BWD, N>(kSlotShift)) {
        if (c0 < c1) init_shift<N, PREC>(q, decode_entry<N>(pts[c0], d));
    }

    double acc[kAccSlots] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double cx[N];
#pragma unroll
    for (int k = 0; k < N; ++k) cx[k] = q.cL * q.xi[k];
    // each stage's entries are loaded during the previous stage's work
    ListEntry nx{0u, 0};
    if (c0 + tid < c1) nx = pts[c0 + tid];
    for (int64_t base = c0; base < c1; base += kHybridStage) {
        const int cnt = (int)min<int64_t>(kHybridStage, c1 - base);
        __syncthreads();
        if (tid < cnt) s_pts[tid] = decode_entry<N>(nx, d);
        __syncthreads();
        if (base + kHybridStage + tid < c1) nx = pts[base + kHybridStage + tid];
        // wave-uniform loop bounds (scalar counter)
        const int k0 = __builtin_amdgcn_readfirstlane(wave);
        if constexpr (BWD && PREC == ECT_FP32) {
            // one kernel's short chain per point: two points per iteration give
            // the wave independent work between the dependent steps (the sums
            // still take the points in order)
#pragma unroll 2
            for (int k = k0; k < cnt; k += kHybridSplit)
                accumulate_point<N, MASK, PREC, BWD>(s_pts[k], q, acc, a.ji0c);
        } else if constexpr (MASK == kL && PREC == ECT_FP32 && !BWD) {
            laplace_stage_f32<N>(s_pts, k0, cnt, cx, q, acc);
        } else {
            for (int k = k0; k < cnt; k += kHybridSplit)
                accumulate_point<N, MASK, PREC, BWD>(s_pts[k], q, acc, a.ji0c);
        }
    }
    acc[kSlotShift] = q.m2;
    if (wave > 0) {
#pragma unroll
        for (int k = 0; k < kAccSlots; ++k)
            if (slot_used<MASK, BWD, N>(k)) s_acc[wave - 1][k][lane] = acc[k];
    }
    __syncthreads();
    if (wave > 0) return;
#pragma unroll
    for (int w = 0; w < kHybridSplit - 1; ++w) {
        double other[kAccSlots];
#pragma unroll
        for (int k = 0; k < kAccSlots; ++k) other[k] = slot_used<MASK, BWD, N>(k) ? s_acc[w][k][lane] : 0.0;
        add_part<N, MASK, PREC, BWD>(q, acc, other, other[kSlotShift]);
    }
    acc[kSlotShift] = q.m2;

    if (chunks > 1) {
#pragma unroll
        for (int k = 0; k < kAccSlots; ++k)
            if (slot_used<MASK, BWD, N>(k)) a.partials[partial_index(item, k, lane)] = acc[k];
        if (tslot >= 0) a.tile_ent[tslot] = (int32_t)e;
        return;
    }
    if (tslot >= 0) a.tile_ent[tslot] = -1;
    if (active) finalize<N, MASK, PREC, BWD>(a, q, row, acc);
}

template <int N, int MASK, int PREC, bool BWD>
__global__ void __launch_bounds__(kHybridThreads) hybrid_kernel(HybridArgs a) {
    hybrid_block<N, MASK, PREC, BWD>(a, blockIdx.x);
}

// The shared-set ECT and a forward hybrid pass in one launch: the first
// ect_blocks workgroups evaluate the ECT (ect_direct_block), the others are the
// hybrid work items.  The two read different lists and write different
// outputs; in one launch the short ECT workgroups run beside the long hybrid
// ones instead of before them.
static_assert(kEctThreads == kHybridThreads, "the combined launch runs both bodies with one workgroup size");

template <int N, int MASK, int PREC>
__global__ void __launch_bounds__(kHybridThreads) ect_hybrid_kernel(HybridArgs h, EctArgs e, int64_t ect_blocks,
                                                                    int64_t ect_groups) {
    const int64_t b = blockIdx.x;
    if (b < ect_blocks) {
        ect_direct_block<N, false, kComboEctDirs>(e, ect_groups, b);
        return;
    }
    hybrid_block<N, MASK, PREC, false>(h, b - ect_blocks);
}

// One workgroup of four waves per query tile: add the partial sums of a
// multi-chunk tile and write the outputs (single-chunk tiles were written
// already).  Wave w adds the w-th quarter of the chunks in chunk order, with
// kReduceBatch chunks' loads in flight per lane; the four quarter sums are then
// added in wave order, so the result is fixed by the chunk count alone.
constexpr int kReduceBatch = 8;

template <int N, int MASK, int PREC, bool BWD>
__global__ void __launch_bounds__(kHybridThreads) hybrid_reduce_kernel(HybridArgs a) {
    constexpr int P = 1 << (N - 1);
    __shared__ double s_acc[kHybridSplit - 1][kAccSlots][kHybridTile];
    const int tid = threadIdx.x;
    const int lane = tid & (kHybridTile - 1);
    const int wave = tid / kHybridTile;
    const int64_t tile = blockIdx.x;
    if (tile >= a.params[1]) return;
    // written by the tile's first chunk in the evaluation launch (-1: one chunk)
    const int32_t ent = a.tile_ent[tile];
    if (ent < 0) return;
    const int64_t C = a.params[2];
    const int64_t e = ent;
    const int64_t img = e / P;
    const int b = (int)(e % P);
    const int64_t t = tile - a.tile_off[e];
    const int l = a.list_base + b;
    const int64_t np = a.list_off[(img + 1) * a.NL + l] - a.list_off[img * a.NL + l];
    const int64_t chunks = np > 0 ? (np + C - 1) / C : 1;
    if (chunks == 1) return;
    const int64_t qn = a.bcnt[a.offsets == nullptr ? b : e];
    const int64_t qi = t * kHybridTile + lane;
    const bool active = qi < qn;
    Query<N> q;
    int64_t row = 0;
    if (wave == 0) setup_query<N, MASK, PREC, BWD>(a, img, b, qi, active, q, row);
    const int64_t first = a.item_off[e] + t * chunks;
    const int64_t per = (chunks + kHybridSplit - 1) / kHybridSplit;
    const int64_t lo = min<int64_t>(chunks, wave * per), hi = min<int64_t>(chunks, lo + per);
    // running Laplace shift of this wave's chunks (below every real shift until the first)
    q.m2 = -kShiftClamp;
    double acc[kAccSlots] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t cc = lo; cc < hi; cc += kReduceBatch) {
        double v[kReduceBatch][kAccSlots];
#pragma unroll
        for (int j = 0; j < kReduceBatch; ++j)
#pragma unroll
            for (int k = 0; k < kAccSlots; ++k)
                v[j][k] = (slot_used<MASK, BWD, N>(k) && cc + j < hi)
                              ? a.partials[partial_index(first + cc + j, k, lane)]
                              : (k == kSlotShift ? -kShiftClamp : 0.0);
#pragma unroll
        for (int j = 0; j < kReduceBatch; ++j) add_part<N, MASK, PREC, BWD>(q, acc, v[j], v[j][kSlotShift]);
    }
    acc[kSlotShift] = q.m2;
    if (wave > 0) {
#pragma unroll
        for (int k = 0; k < kAccSlots; ++k)
            if (slot_used<MASK, BWD, N>(k)) s_acc[wave - 1][k][lane] = acc[k];
    }
    __syncthreads();
    if (wave > 0 || !active) return;
#pragma unroll
    for (int w = 0; w < kHybridSplit - 1; ++w) {
        double other[kAccSlots];
#pragma unroll
        for (int k = 0; k < kAccSlots; ++k) other[k] = slot_used<MASK, BWD, N>(k) ? s_acc[w][k][lane] : 0.0;
        add_part<N, MASK, PREC, BWD>(q, acc, other, other[kSlotShift]);
    }
    finalize<N, MASK, PREC, BWD>(a, q, row, acc);
}

// Sum per-image gradient rows of a shared query set in image order, and the
// per-row d/ds contributions in a fixed tree order.
template <int N>
__global__ void __launch_bounds__(256)
grad_reduce_kernel(const double* __restrict__ part, int num_images, int64_t count, int shared,
                   double* __restrict__ grad_xi, const double* __restrict__ gs_part, int64_t rows,
                   double* __restrict__ grad_s) {
    constexpr int R = 8;   // loads in flight per thread
    if (blockIdx.x < gridDim.x - 1) {
        if (!shared) return;
        const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (k >= count * N) return;
        double acc = 0.0;
        for (int i0 = 0; i0 < num_images; i0 += R) {
            double v[R];
#pragma unroll
            for (int j = 0; j < R; ++j) v[j] = i0 + j < num_images ? part[(int64_t)(i0 + j) * count * N + k] : 0.0;
#pragma unroll
            for (int j = 0; j < R; ++j) acc += v[j];
        }
        grad_xi[k] = acc;
        return;
    }
    if (!grad_s) return;
    __shared__ double s_red[256];
    double acc = 0.0;
    for (int64_t r0 = threadIdx.x; r0 < rows; r0 += (int64_t)R * blockDim.x) {
        double v[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int64_t r = r0 + (int64_t)j * blockDim.x;
            v[j] = r < rows ? gs_part[r] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < R; ++j) acc += v[j];
    }
    s_red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s_red[threadIdx.x] += s_red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *grad_s = s_red[0];
}

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <int N, int MASK, bool BWD>
hipError_t launch_mask(int precision, const HybridArgs& a0, int64_t grid, bool reduce, hipStream_t stream) {
    HybridArgs a = a0;
    for (int k = 0; k < kJi0SmallCoeffs; ++k) a.ji0c[k] = JI0_F32_SMALL[k];
    dim3 g((unsigned)grid), blk(kHybridThreads), rblk(kHybridThreads);
    if (precision == ECT_FP32) {
        if (reduce) hipLaunchKernelGGL((hybrid_reduce_kernel<N, MASK, ECT_FP32, BWD>), g, rblk, 0, stream, a);
        else hipLaunchKernelGGL((hybrid_kernel<N, MASK, ECT_FP32, BWD>), g, blk, 0, stream, a);
    } else {
        if (reduce) hipLaunchKernelGGL((hybrid_reduce_kernel<N, MASK, ECT_FP64, BWD>), g, rblk, 0, stream, a);
        else hipLaunchKernelGGL((hybrid_kernel<N, MASK, ECT_FP64, BWD>), g, blk, 0, stream, a);
    }
    return hipGetLastError();
}

template <int N>
hipError_t launch_dispatch(unsigned mask, int precision, bool backward, const HybridArgs& a, int64_t grid,
                           bool reduce, hipStream_t stream) {
    if (backward) {
        switch (mask) {
            case kF: return launch_mask<N, kF, true>(precision, a, grid, reduce, stream);
            case kL: return launch_mask<N, kL, true>(precision, a, grid, reduce, stream);
            default: return launch_mask<N, kB, true>(precision, a, grid, reduce, stream);
        }
    }
    switch (mask) {
        case 1: return launch_mask<N, 1, false>(precision, a, grid, reduce, stream);
        case 2: return launch_mask<N, 2, false>(precision, a, grid, reduce, stream);
        case 3: return launch_mask<N, 3, false>(precision, a, grid, reduce, stream);
        case 4: return launch_mask<N, 4, false>(precision, a, grid, reduce, stream);
        case 5: return launch_mask<N, 5, false>(precision, a, grid, reduce, stream);
        case 6: return launch_mask<N, 6, false>(precision, a, grid, reduce, stream);
        case kLin: return launch_mask<N, kLin, false>(ECT_FP64, a, grid, reduce, stream);
        default: return launch_mask<N, 7, false>(precision, a, grid, reduce, stream);
    }
}

}  // namespace

hipError_t launch_hybrid(int ndim, unsigned mask, int precision, bool backward, const HybridArgs& a,
                         int64_t grid, int64_t tiles, hipStream_t stream) {
    const int stage = backward ? ECT_STAGE_HYBRID_BWD : ECT_STAGE_HYBRID;
    hipError_t e = hipSuccess;
    if (grid > 0) {
        e = stage_mark(stage, false, stream);
        if (e != hipSuccess) return e;
        e = ndim == 2   ? launch_dispatch<2>(mask, precision, backward, a, grid, false, stream)
            : ndim == 3 ? launch_dispatch<3>(mask, precision, backward, a, grid, false, stream)
                        : launch_dispatch<4>(mask, precision, backward, a, grid, false, stream);
        if (e != hipSuccess) return e;
        e = stage_mark(stage, true, stream);
        if (e != hipSuccess) return e;
    }
    if (tiles > 0)
        e = ndim == 2   ? launch_dispatch<2>(mask, precision, backward, a, tiles, true, stream)
            : ndim == 3 ? launch_dispatch<3>(mask, precision, backward, a, tiles, true, stream)
                        : launch_dispatch<4>(mask, precision, backward, a, tiles, true, stream);
    return e;
}

hipError_t launch_grad_reduce(int ndim, const double* part, int num_images, int64_t count, bool shared,
                              double* grad_xi, const double* gs_part, int64_t rows, double* grad_s,
                              hipStream_t stream) {
    const int64_t n = shared ? count * ndim : 0;
    const unsigned blocks = (unsigned)((n + 255) / 256) + 1;
    if (ndim == 2)
        hipLaunchKernelGGL(grad_reduce_kernel<2>, dim3(blocks), dim3(256), 0, stream, part, num_images, count,
                           shared ? 1 : 0, grad_xi, gs_part, rows, grad_s);
    else if (ndim == 3)
        hipLaunchKernelGGL(grad_reduce_kernel<3>, dim3(blocks), dim3(256), 0, stream, part, num_images, count,
                           shared ? 1 : 0, grad_xi, gs_part, rows, grad_s);
    else
        hipLaunchKernelGGL(grad_reduce_kernel<4>, dim3(blocks), dim3(256), 0, stream, part, num_images, count,
                           shared ? 1 : 0, grad_xi, gs_part, rows, grad_s);
    return hipGetLastError();
}

namespace {

template <int N, int MASK>
hipError_t launch_ect_hybrid_mask(int precision, const HybridArgs& h0, const EctArgs& e, int64_t grid,
                                  int64_t ect_blocks, int64_t ect_groups, size_t shmem, hipStream_t stream) {
    HybridArgs h = h0;
    for (int k = 0; k < kJi0SmallCoeffs; ++k) h.ji0c[k] = JI0_F32_SMALL[k];
    const dim3 g((unsigned)(grid + ect_blocks)), blk(kHybridThreads);
    if (precision == ECT_FP32)
        hipLaunchKernelGGL((ect_hybrid_kernel<N, MASK, ECT_FP32>), g, blk, shmem, stream, h, e, ect_blocks, ect_groups);
    else
        hipLaunchKernelGGL((ect_hybrid_kernel<N, MASK, ECT_FP64>), g, blk, shmem, stream, h, e, ect_blocks, ect_groups);
    return hipGetLastError();
}

template <int N>
hipError_t launch_ect_hybrid_n(unsigned mask, int precision, const HybridArgs& h, const EctArgs& e, int64_t grid,
                               int64_t ect_blocks, int64_t ect_groups, size_t shmem, hipStream_t stream) {
    switch (mask) {
        case 1: return launch_ect_hybrid_mask<N, 1>(precision, h, e, grid, ect_blocks, ect_groups, shmem, stream);
        case 2: return launch_ect_hybrid_mask<N, 2>(precision, h, e, grid, ect_blocks, ect_groups, shmem, stream);
        case 3: return launch_ect_hybrid_mask<N, 3>(precision, h, e, grid, ect_blocks, ect_groups, shmem, stream);
        case 4: return launch_ect_hybrid_mask<N, 4>(precision, h, e, grid, ect_blocks, ect_groups, shmem, stream);
        case 5: return launch_ect_hybrid_mask<N, 5>(precision, h, e, grid, ect_blocks, ect_groups, shmem, stream);
        case 6: return launch_ect_hybrid_mask<N, 6>(precision, h, e, grid, ect_blocks, ect_groups, shmem, stream);
        default: return launch_ect_hybrid_mask<N, 7>(precision, h, e, grid, ect_blocks, ect_groups, shmem, stream);
    }
}

}  // namespace

hipError_t launch_ect_hybrid(int ndim, unsigned mask, int precision, const HybridArgs& h, const EctArgs& e,
                             int64_t grid, int64_t ect_blocks, int64_t ect_groups, hipStream_t stream) {
    // the ECT block keeps at most kComboEctDirs directions; the constant-kernel
    // limit has no combined instantiation (the caller makes two launches)
    if (e.dirs_per_group < 1 || e.dirs_per_group > kComboEctDirs || mask < 1 || mask > 7 || e.chunks < 1)
        return hipErrorInvalidValue;
    const size_t shmem = sizeof(double) * e.M + sizeof(int32_t) * e.dirs_per_group * e.M;
    hipError_t err = stage_mark(ECT_STAGE_HYBRID, false, stream);
    if (err != hipSuccess) return err;
    if (ndim == 2) err = launch_ect_hybrid_n<2>(mask, precision, h, e, grid, ect_blocks, ect_groups, shmem, stream);
    else if (ndim == 3) err = launch_ect_hybrid_n<3>(mask, precision, h, e, grid, ect_blocks, ect_groups, shmem, stream);
    else err = launch_ect_hybrid_n<4>(mask, precision, h, e, grid, ect_blocks, ect_groups, shmem, stream);
    if (err != hipSuccess) return err;
    return stage_mark(ECT_STAGE_HYBRID, true, stream);
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

}  // namespace ect
