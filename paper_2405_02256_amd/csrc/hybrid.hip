// Hybrid transforms HT(xi) = sum over ordinary points of Delta^ord(eps,x) kbar_s(<xi,x>)
// and their vector-Jacobian products (gfx950).
//
// The hybrid transform is the integral of kappa against the Radon transform
// (Sec. 2.2); by Lemma 3.1 it only needs the ordinary critical points of the
// query's sign vector and the primitive kbar of the kernel.  The sign used
// here is the one the definition gives (a closed square yields
// kbar(max) - kbar(min)).
//
// Work decomposition: queries are bucketed by orthant pair; a work item is
// (image, pair, tile of 64 queries, chunk of points).  One wave runs an item:
// every lane owns one query held in registers, and the wave walks the chunk's
// points in lockstep, so each point is fetched once per wave with a scalar
// load.  Per pair of (query, point):
//   FP32 precision: FP64 phase, FP64 argument reduction to [0, 1) revolutions
//                   (or to a split exponent for Laplace), FP32 kernel value
//                   (hardware sin/cos/exp2 on reduced arguments, polynomial
//                   Ji0), FP64 accumulation;
//   FP64 precision: every step in FP64.
// Items of one query tile write per-lane partial sums; the last item of the
// tile to finish (counted with an atomic) adds the partials in chunk order, so
// results are bitwise reproducible.
#include "eval_internal.h"
#include "ji0_coeffs.h"

namespace ect {

namespace {

constexpr double kInv2Pi = 0.15915494309189535;
constexpr double kLog2E = 1.4426950408889634;
constexpr int kAccSlots = 4;      // doubles per lane in a partial record

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

// Ji0(z) = integral_0^z J0 in FP32 (coefficients fitted against mpmath).
__device__ __forceinline__ float ji0_f32(double z) {
    const double az = fabs(z);
    float r;
    if (az < JI0_Z0) {
        // the monomial coefficients alternate in sign up to ~16 in size, so the
        // polynomial is evaluated in FP64 (same issue rate as FP32 on this chip)
        const double v = az * az * (1.0 / (JI0_Z0 * JI0_Z0));
        r = (float)(az * horner<JI0_F32_SMALL_DEG + 1, double>(JI0_F32_SMALL, v));
    } else {
        const float zf = (float)az;
        const float rz = __builtin_amdgcn_rcpf(zf);
        const float w = (float)(JI0_Z0 * JI0_Z0) * rz * rz;
        const float A = horner<JI0_F32_TAILA_DEG + 1, float>(JI0_F32_TAILA, w);
        const float Bv = horner<JI0_F32_TAILB_DEG + 1, float>(JI0_F32_TAILB, w);
        const double rev = az * kInv2Pi - 0.125;
        const float rf = (float)(rev - floor(rev));
        float sn, cs;
        sincos_rev_f32(rf, &sn, &cs);
        const float amp = 0.79788456080286536f * __builtin_amdgcn_rsqf(zf);
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
    return ldexp(e, (int)fmax(n, -2000.0));
}

// Per-lane query state.
template <int N>
struct Query {
    double xi[N];     // raw direction
    double w[N];      // scaled direction used for the phase
    double m;         // Laplace shift (natural log units)
    double gr, gi;    // backward: output cotangent
    double sigma;     // +1, or -1 when the query's list is the pair's mirror
};

// Accumulate the contributions of points [c0, c1) of `pts`.
//   forward: acc[0] (Fourier: acc[0], acc[1] = sums of D sin, D cos)
//   backward: acc[a] = sum of D x_a kappa-part (weighted by the cotangent)
template <int N, int KER, int PREC, bool BWD>
__device__ __forceinline__ void accumulate(const Point* __restrict__ pts, int64_t c0, int64_t c1,
                                           const Query<N>& q, double* acc) {
#pragma unroll 2
    for (int64_t p = c0; p < c1; ++p) {
        const Point pt = pts[p];
        if constexpr (KER == ECT_FOURIER) {
            // phase in revolutions: s <xi, x> / (2 pi)
            double ph = q.w[0] * pt.x[0];
#pragma unroll
            for (int a = 1; a < N; ++a) ph = fma(q.w[a], pt.x[a], ph);
            double sn, cs;
            if constexpr (PREC == ECT_FP32) {
                float s32, c32;
                sincos_rev_f32((float)(ph - floor(ph)), &s32, &c32);
                sn = (double)s32;
                cs = (double)c32;
            } else {
                sincospi(2.0 * (ph - rint(ph)), &sn, &cs);
            }
            if constexpr (!BWD) {
                acc[0] = fma(pt.val, sn, acc[0]);
                acc[1] = fma(pt.val, cs, acc[1]);
            } else {
                // kappa(s u) = exp(-i s u): d Re/d xi_a = x cos, d Im/d xi_a = -x sin
                const double g = pt.val * (q.gr * cs - q.gi * sn);
#pragma unroll
                for (int a = 0; a < N; ++a) acc[a] = fma(g, pt.x[a], acc[a]);
            }
        } else if constexpr (KER == ECT_LAPLACE) {
            // exponent -s u - m <= 0 (FP32: in log2 units)
            double ex = fma(q.w[0], pt.x[0], -q.m);
#pragma unroll
            for (int a = 1; a < N; ++a) ex = fma(q.w[a], pt.x[a], ex);
            const double term = (PREC == ECT_FP32) ? exp2_split(ex) : exp(ex);
            if constexpr (!BWD) {
                acc[0] = fma(pt.val, term, acc[0]);
            } else {
                const double g = pt.val * term;
#pragma unroll
                for (int a = 0; a < N; ++a) acc[a] = fma(g, pt.x[a], acc[a]);
            }
        } else {
            double z = q.w[0] * pt.x[0];
#pragma unroll
            for (int a = 1; a < N; ++a) z = fma(q.w[a], pt.x[a], z);
            if constexpr (!BWD) {
                const double ji = (PREC == ECT_FP32) ? (double)ji0_f32(z) : ji0_f64(z);
                acc[0] = fma(pt.val, ji, acc[0]);
            } else {
                const double j = (PREC == ECT_FP32) ? (double)j0f((float)z) : j0(z);
                const double g = pt.val * j;
#pragma unroll
                for (int a = 0; a < N; ++a) acc[a] = fma(g, pt.x[a], acc[a]);
            }
        }
    }
}

template <int N, int KER, int PREC, bool BWD>
__global__ void __launch_bounds__(kHybridLanes) hybrid_kernel(HybridArgs a) {
    constexpr int P = 1 << (N - 1);
    constexpr int NACC = BWD ? N : (KER == ECT_FOURIER ? 2 : 1);
    const int lane = threadIdx.x;
    const int64_t item = blockIdx.x;
    const int64_t total = a.params[0];
    if (item >= total) return;
    const int64_t C = a.params[2];
    const int64_t E = (int64_t)a.num_images * P;
    int64_t lo = 0, hi = E - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (a.item_off[mid] <= item) lo = mid; else hi = mid - 1;
    }
    const int64_t e = lo;
    const int64_t img = e / P;
    const int b = (int)(e % P);
    const int64_t local = item - a.item_off[e];
    const int l = a.list_base + b;
    const int64_t p0 = a.list_off[img * a.NL + l], p1 = a.list_off[(img + 1) * a.NL + l];
    const int64_t np = p1 - p0;
    const int64_t chunks = np > 0 ? (np + C - 1) / C : 1;
    const int64_t t = local / chunks, c = local % chunks;
    const bool shared_q = a.offsets == nullptr;
    const int64_t bidx = shared_q ? b : e;
    const int64_t qn = a.bcnt[bidx];
    const int64_t qi = t * kHybridLanes + lane;
    const bool active = qi < qn;
    const int64_t row_base = shared_q ? img * a.count : a.offsets[img];
    int64_t row = 0;
    Query<N> q;
    q.sigma = 1.0;
    q.m = 0.0;
    q.gr = q.gi = 0.0;
    const double s = a.s;
    if (active) {
        const int64_t code = a.perm[a.bstart[bidx] + qi];
        row = row_base + (code >> 1);                       // output row
        const int64_t vrow = shared_q ? (code >> 1) : row;  // row of the query vector
        q.sigma = (code & 1) ? -1.0 : 1.0;
#pragma unroll
        for (int k = 0; k < N; ++k) q.xi[k] = a.vecs[vrow * N + k];
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) q.xi[k] = 0.0;
    }
    const ImageDesc& dsc = a.desc[img];
    if constexpr (KER == ECT_FOURIER) {
#pragma unroll
        for (int k = 0; k < N; ++k) q.w[k] = q.xi[k] * (s * kInv2Pi);
    } else if constexpr (KER == ECT_LAPLACE) {
        // m = max over the image's vertex box of -s <xi, x> (an upper bound of every exponent)
        double m = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) m += fmax(-s * q.xi[k] * dsc.lo[k], -s * q.xi[k] * dsc.hi[k]);
        q.m = (PREC == ECT_FP32) ? m * kLog2E : m;
#pragma unroll
        for (int k = 0; k < N; ++k) q.w[k] = (PREC == ECT_FP32) ? -s * kLog2E * q.xi[k] : -s * q.xi[k];
        q.m = active ? q.m : 0.0;
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) q.w[k] = s * q.xi[k];
    }
    if constexpr (BWD) {
        if (active) {
            if (KER == ECT_FOURIER) {
                q.gr = a.grad_out[row * 2];
                q.gi = a.grad_out[row * 2 + 1];
            } else {
                q.gr = a.grad_out[row];
            }
        }
    }

    double acc[kAccSlots] = {0.0, 0.0, 0.0, 0.0};
    const Point* __restrict__ pts = a.points + (int64_t)l * a.capacity;
    const int64_t c0 = p0 + c * C, c1 = min(p1, c0 + C);
    if (np > 0) accumulate<N, KER, PREC, BWD>(pts, c0, c1, q, acc);

    if (chunks > 1) {
        double* part = a.partials + (item * kHybridLanes + lane) * kAccSlots;
#pragma unroll
        for (int k = 0; k < NACC; ++k) part[k] = acc[k];
        __threadfence();
        uint32_t old = 0;
        if (lane == 0)
            old = __hip_atomic_fetch_add(a.counters + a.tile_off[e] + t, 1u, __ATOMIC_ACQ_REL,
                                         __HIP_MEMORY_SCOPE_AGENT);
        old = __shfl(old, 0, 64);
        if (old != (uint32_t)(chunks - 1)) return;
        __threadfence();
#pragma unroll
        for (int k = 0; k < NACC; ++k) acc[k] = 0.0;
        const int64_t first = a.item_off[e] + t * chunks;
        for (int64_t cc = 0; cc < chunks; ++cc) {
            const double* pp = a.partials + ((first + cc) * kHybridLanes + lane) * kAccSlots;
#pragma unroll
            for (int k = 0; k < NACC; ++k) acc[k] += __builtin_nontemporal_load(pp + k);
        }
        if (lane == 0) a.counters[a.tile_off[e] + t] = 0u;
    }
    if (!active) return;

    if constexpr (!BWD) {
        if constexpr (KER == ECT_FOURIER) {
            a.out[row * 2] = q.sigma * acc[0] / s;
            a.out[row * 2 + 1] = q.sigma * acc[1] / s;
            if (a.log_scale) a.log_scale[row] = 0.0;
        } else if constexpr (KER == ECT_LAPLACE) {
            const double mnat = (PREC == ECT_FP32) ? q.m / kLog2E : q.m;
            const double shifted = -q.sigma * acc[0] / s;
            if (a.log_scale) {
                a.out[row] = shifted;
                a.log_scale[row] = mnat;
            } else {
                const double v = shifted * exp(mnat);
                if (!isfinite(v)) raise_error(a.err, ECT_DEVERR_OVERFLOW);
                a.out[row] = v;
            }
        } else {
            a.out[row] = q.sigma * acc[0] / s;
            if (a.log_scale) a.log_scale[row] = 0.0;
        }
    } else {
        // G_a = sigma * sum D x_a (weighted kappa); Laplace sums carry exp(-m)
        double scale = q.sigma;
        if constexpr (KER == ECT_LAPLACE) scale *= q.gr * exp((PREC == ECT_FP32) ? q.m / kLog2E : q.m);
        if constexpr (KER == ECT_BESSEL) scale *= q.gr;
        double dots = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const double G = scale * acc[k];
            a.grad_xi[row * N + k] = G;
            dots = fma(q.xi[k], G, dots);
        }
        double gy;
        if constexpr (KER == ECT_FOURIER) gy = q.gr * a.fwd_out[row * 2] + q.gi * a.fwd_out[row * 2 + 1];
        else gy = q.gr * a.fwd_out[row];
        a.grad_s_part[row] = (dots - gy) / s;
    }
}

// Sum per-image gradient rows of a shared query set in image order, and the
// per-row d/ds contributions in a fixed tree order.
template <int N>
__global__ void __launch_bounds__(256)
grad_reduce_kernel(const double* __restrict__ part, int num_images, int64_t count, int shared,
                   double* __restrict__ grad_xi, const double* __restrict__ gs_part, int64_t rows,
                   double* __restrict__ grad_s) {
    if (blockIdx.x < gridDim.x - 1) {
        if (!shared) return;
        const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (k >= count * N) return;
        double acc = 0.0;
        for (int i = 0; i < num_images; ++i) acc += part[(int64_t)i * count * N + k];
        grad_xi[k] = acc;
        return;
    }
    if (!grad_s) return;
    __shared__ double s_red[256];
    double acc = 0.0;
    for (int64_t r = threadIdx.x; r < rows; r += blockDim.x) acc += gs_part[r];
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

template <int N, bool BWD>
hipError_t launch_n(int kernel, int precision, const HybridArgs& a, int64_t grid, hipStream_t stream) {
    dim3 g((unsigned)grid), blk(kHybridLanes);
#define ECT_HYB(K, PR) hipLaunchKernelGGL((hybrid_kernel<N, K, PR, BWD>), g, blk, 0, stream, a)
    if (precision == ECT_FP32) {
        if (kernel == ECT_FOURIER) ECT_HYB(ECT_FOURIER, ECT_FP32);
        else if (kernel == ECT_LAPLACE) ECT_HYB(ECT_LAPLACE, ECT_FP32);
        else ECT_HYB(ECT_BESSEL, ECT_FP32);
    } else {
        if (kernel == ECT_FOURIER) ECT_HYB(ECT_FOURIER, ECT_FP64);
        else if (kernel == ECT_LAPLACE) ECT_HYB(ECT_LAPLACE, ECT_FP64);
        else ECT_HYB(ECT_BESSEL, ECT_FP64);
    }
#undef ECT_HYB
    return hipGetLastError();
}

}  // namespace

hipError_t launch_hybrid_fwd(int ndim, int kernel, int precision, const HybridArgs& a, int64_t grid,
                             hipStream_t stream) {
    if (grid <= 0) return hipSuccess;
    hipError_t e = stage_mark(ECT_STAGE_HYBRID, false, stream);
    if (e != hipSuccess) return e;
    e = ndim == 2 ? launch_n<2, false>(kernel, precision, a, grid, stream)
                  : launch_n<3, false>(kernel, precision, a, grid, stream);
    if (e != hipSuccess) return e;
    return stage_mark(ECT_STAGE_HYBRID, true, stream);
}

hipError_t launch_hybrid_bwd(int ndim, int kernel, int precision, const HybridArgs& a, int64_t grid,
                             hipStream_t stream) {
    if (grid <= 0) return hipSuccess;
    hipError_t e = stage_mark(ECT_STAGE_HYBRID_BWD, false, stream);
    if (e != hipSuccess) return e;
    e = ndim == 2 ? launch_n<2, true>(kernel, precision, a, grid, stream)
                  : launch_n<3, true>(kernel, precision, a, grid, stream);
    if (e != hipSuccess) return e;
    return stage_mark(ECT_STAGE_HYBRID_BWD, true, stream);
}

hipError_t launch_grad_reduce(int ndim, const double* part, int num_images, int64_t count, bool shared,
                              double* grad_xi, const double* gs_part, int64_t rows, double* grad_s,
                              hipStream_t stream) {
    const int64_t n = shared ? count * ndim : 0;
    const unsigned blocks = (unsigned)((n + 255) / 256) + 1;
    if (ndim == 2)
        hipLaunchKernelGGL(grad_reduce_kernel<2>, dim3(blocks), dim3(256), 0, stream, part, num_images, count,
                           shared ? 1 : 0, grad_xi, gs_part, rows, grad_s);
    else
        hipLaunchKernelGGL(grad_reduce_kernel<3>, dim3(blocks), dim3(256), 0, stream, part, num_images, count,
                           shared ? 1 : 0, grad_xi, gs_part, rows, grad_s);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

}  // namespace ect
