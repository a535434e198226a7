/*
 * Plain FP64 CPU oracle for topological integral transforms of weighted cubical
 * complexes.  TEST INFRASTRUCTURE ONLY: nothing on the product path may link or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the GPU library.
 *
 * Every routine evaluates a plain definition over ALL cells of the complex, so
 * that a reader can check it against the paper by eye:
 *
 *   cells      weighted cubical complex built from an image: "primal" gives one
 *              top cell per pixel and every lower cell the min over its coface
 *              top cells (Sec. 4.1, implementation of cubical complexes);
 *              "dual" puts pixel values on vertices and gives every other cell
 *              the min over its vertices (Sec. 5, experimental setup).
 *   chi        chi(phi) = sum over cells of (-1)^dim * phi (Sec. 2.1).
 *   ect        ECT(xi,t) = chi of phi restricted to {xi <= t} (Sec. 2.2).  A cell
 *              cut by the hyperplane contributes phi*((-1)^d + (-1)^(d-1)) = 0,
 *              so ECT(xi,t) = sum of (-1)^dim phi(c) over cells whose highest
 *              vertex satisfies <xi,v> <= t (Lemma 2.1 with its sign factors
 *              and with the max of xi over the cell).
 *   hybrid     HT(xi) = integral of kappa(t) R(xi,t) dt (Sec. 2.2).  With Lemma A.1,
 *              a cell of positive dimension contributes (-1)^(dim-1) phi on the
 *              open interval (min_c xi, max_c xi) and a vertex only on a single
 *              point, so HT = sum over cells of dim >= 1 of
 *              (-1)^(dim-1) phi(c) [kbar(max_c xi) - kbar(min_c xi)].
 *   gradient   derivative of the previous sum in xi and in the kernel scale s.
 *   critical   lower-star and upper-star Euler characteristics at each vertex
 *              for each sign vector (Sec. 3, definitions of the critical values;
 *              Sec. 4.2 and Appendix A for the star enumeration).
 *
 * Conventions:
 *   - GUDHI-style cell grid: cell coordinate c_a in [0, 2 N_a], dim c = number of
 *     odd coordinates, N_a top cells along axis a; axis 0 varies fastest.
 *   - Vertex k (c = 2k) sits at x_a = fma(h_a, k_a, o_a).
 *   - Canonical projection u = fma(xi_{n-1}, x_{n-1}, ... fma(xi_1, x_1, xi_0*x_0)).
 *   - Thresholds are a non-decreasing FP64 array; the sublevel set is closed (u <= t).
 *   - Kernels with scale s: kappa_s(t) = kappa(s t), kbar_s(t) = kbar(s t)/s with
 *       Fourier  kappa = exp(-i t),  kbar = i exp(-i t) = (sin t, cos t)
 *       Laplace  kappa = exp(-t),    kbar = -exp(-t)
 *       Bessel   kappa = J0,         kbar = Ji0(t) = integral_0^t J0
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no fused multiply-add
 * except where fma() is written out).
 */
#define _DEFAULT_SOURCE 1 /* j0 from the XSI extensions of libm */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXD 4
#define MAXV (1 << MAXD)   /* vertices of a cell, at most */

enum { OR_PRIMAL = 0, OR_DUAL = 1 };
enum { OR_FOURIER = 0, OR_LAPLACE = 1, OR_BESSEL = 2 };

typedef struct {
    int n;
    int dims[MAXD];   /* pixels along axis a */
    int N[MAXD];      /* top cells along axis a */
    int G[MAXD];      /* cell grid extent 2N+1 */
    int V[MAXD];      /* vertices along axis a: N+1 */
    long long ncell;
    long long nvert;
    double o[MAXD], h[MAXD];
} ogrid;

static int grid_init(ogrid* g, int n, const int32_t* dims, int construction,
                     const double* origin, const double* spacing) {
    if (n < 1 || n > MAXD) return 1;
    g->n = n;
    g->ncell = 1;
    g->nvert = 1;
    for (int a = 0; a < MAXD; ++a) {
        g->dims[a] = 1; g->N[a] = 0; g->G[a] = 1; g->V[a] = 1; g->o[a] = 0.0; g->h[a] = 1.0;
    }
    for (int a = 0; a < n; ++a) {
        if (dims[a] < 1) return 1;
        g->dims[a] = dims[a];
        g->N[a] = construction == OR_PRIMAL ? dims[a] : dims[a] - 1;
        g->G[a] = 2 * g->N[a] + 1;
        g->V[a] = g->N[a] + 1;
        g->ncell *= g->G[a];
        g->nvert *= g->V[a];
        g->o[a] = origin ? origin[a] : -0.5 * (double)g->N[a];
        g->h[a] = spacing ? spacing[a] : 1.0;
    }
    return 0;
}

static void cell_coords(const ogrid* g, long long id, int c[MAXD]) {
    for (int a = 0; a < MAXD; ++a) { c[a] = 0; }
    for (int a = 0; a < g->n; ++a) { c[a] = (int)(id % g->G[a]); id /= g->G[a]; }
}

static int cell_dim(const ogrid* g, const int c[MAXD]) {
    int d = 0;
    for (int a = 0; a < g->n; ++a) d += c[a] & 1;
    return d;
}

static long long pixel_index(const ogrid* g, const int p[MAXD]) {
    long long idx = 0, stride = 1;
    for (int a = 0; a < g->n; ++a) { idx += (long long)p[a] * stride; stride *= g->dims[a]; }
    return idx;
}

static long long vertex_index(const ogrid* g, const int k[MAXD]) {
    long long idx = 0, stride = 1;
    for (int a = 0; a < g->n; ++a) { idx += (long long)k[a] * stride; stride *= g->V[a]; }
    return idx;
}

/* Next point of the box lo..hi (every axis, in steps of `step`, axis 0
 * fastest); returns 0 after the last one. */
static int box_next(int* q, const int* lo, const int* hi, int step) {
    for (int a = 0; a < MAXD; ++a) {
        if (q[a] + step <= hi[a]) { q[a] += step; return 1; }
        q[a] = lo[a];
    }
    return 0;
}

/* Value of one cell.  Primal: min over coface top cells (all-odd coordinates
 * within one step of c and inside the grid).  Dual: min over its vertices. */
static int32_t cell_value(const ogrid* g, const int c[MAXD], const int32_t* px, int construction) {
    int lo[MAXD], hi[MAXD];
    for (int a = 0; a < MAXD; ++a) { lo[a] = 0; hi[a] = 0; }
    for (int a = 0; a < g->n; ++a) {
        if (construction == OR_PRIMAL) {
            if (c[a] & 1) { lo[a] = hi[a] = c[a]; }
            else { lo[a] = c[a] - 1 < 1 ? c[a] + 1 : c[a] - 1;
                   hi[a] = c[a] + 1 > 2 * g->N[a] - 1 ? c[a] - 1 : c[a] + 1; }
        } else {
            if (c[a] & 1) { lo[a] = c[a] - 1; hi[a] = c[a] + 1; }
            else { lo[a] = hi[a] = c[a]; }
        }
    }
    int32_t best = 0;
    int have = 0;
    int q[MAXD];
    for (int a = 0; a < MAXD; ++a) q[a] = lo[a];
    do {
        int p[MAXD];
        for (int a = 0; a < MAXD; ++a)
            p[a] = construction == OR_PRIMAL ? (q[a] - 1) / 2 : q[a] / 2;
        int32_t v = px[pixel_index(g, p)];
        if (!have || v < best) { best = v; have = 1; }
    } while (box_next(q, lo, hi, 2));
    return best;
}

int oracle_cell_values(int n, const int32_t* dims, const int32_t* px, int construction, int32_t* phi) {
    ogrid g;
    if (grid_init(&g, n, dims, construction, NULL, NULL)) return 1;
    for (int a = 0; a < n; ++a) if (g.N[a] < 0) return 1;
    for (long long id = 0; id < g.ncell; ++id) {
        int c[MAXD];
        cell_coords(&g, id, c);
        phi[id] = cell_value(&g, c, px, construction);
    }
    return 0;
}

long long oracle_euler_characteristic(int n, const int32_t* dims, const int32_t* px, int construction) {
    ogrid g;
    if (grid_init(&g, n, dims, construction, NULL, NULL)) return 0;
    long long chi = 0;
    for (long long id = 0; id < g.ncell; ++id) {
        int c[MAXD];
        cell_coords(&g, id, c);
        int32_t v = cell_value(&g, c, px, construction);
        chi += (cell_dim(&g, c) & 1) ? -(long long)v : (long long)v;
    }
    return chi;
}

/* ---- shared per-call preparation: nonzero cells and their vertex lists ---- */

typedef struct {
    long long count;
    int32_t* value;      /* phi */
    int8_t* dim;
    int8_t* nv;          /* number of vertices (2^dim) */
    long long* verts;    /* [count][MAXV] vertex indices */
    long long* vidx;     /* unused slots = -1 */
} cellset;

static void cellset_free(cellset* cs) {
    free(cs->value); free(cs->dim); free(cs->nv); free(cs->verts);
    memset(cs, 0, sizeof(*cs));
}

/* Collect every cell with phi != 0 (cells with phi == 0 contribute nothing to
 * any of the sums).  min_dim excludes lower-dimensional cells when asked. */
static int cellset_build(const ogrid* g, const int32_t* px, int construction, int min_dim, cellset* cs) {
    memset(cs, 0, sizeof(*cs));
    long long cap = 0;
    for (long long id = 0; id < g->ncell; ++id) {
        int c[MAXD];
        cell_coords(g, id, c);
        if (cell_dim(g, c) >= min_dim && cell_value(g, c, px, construction) != 0) ++cap;
    }
    cs->value = (int32_t*)malloc(sizeof(int32_t) * (cap ? cap : 1));
    cs->dim = (int8_t*)malloc(cap ? cap : 1);
    cs->nv = (int8_t*)malloc(cap ? cap : 1);
    cs->verts = (long long*)malloc(sizeof(long long) * MAXV * (cap ? cap : 1));
    if (!cs->value || !cs->dim || !cs->nv || !cs->verts) { cellset_free(cs); return 1; }
    long long m = 0;
    for (long long id = 0; id < g->ncell; ++id) {
        int c[MAXD];
        cell_coords(g, id, c);
        int d = cell_dim(g, c);
        if (d < min_dim) continue;
        int32_t v = cell_value(g, c, px, construction);
        if (v == 0) continue;
        cs->value[m] = v;
        cs->dim[m] = (int8_t)d;
        int lo[MAXD], hi[MAXD];
        for (int a = 0; a < MAXD; ++a) {
            if (a < g->n && (c[a] & 1)) { lo[a] = c[a] - 1; hi[a] = c[a] + 1; }
            else { lo[a] = hi[a] = c[a]; }
        }
        int nv = 0;
        int q[MAXD];
        for (int a = 0; a < MAXD; ++a) q[a] = lo[a];
        do {
            int k[MAXD];
            for (int a = 0; a < MAXD; ++a) k[a] = q[a] / 2;
            cs->verts[m * MAXV + nv++] = vertex_index(g, k);
        } while (box_next(q, lo, hi, 2));
        cs->nv[m] = (int8_t)nv;
        ++m;
    }
    cs->count = m;
    return 0;
}

/* Vertex coordinates x[v][a] = fma(h_a, k_a, o_a). */
static double* vertex_coords(const ogrid* g) {
    double* x = (double*)malloc(sizeof(double) * MAXD * (g->nvert ? g->nvert : 1));
    if (!x) return NULL;
    for (long long v = 0; v < g->nvert; ++v) {
        long long r = v;
        for (int a = 0; a < MAXD; ++a) {
            int k = 0;
            if (a < g->n) { k = (int)(r % g->V[a]); r /= g->V[a]; }
            x[v * MAXD + a] = a < g->n ? fma(g->h[a], (double)k, g->o[a]) : 0.0;
        }
    }
    return x;
}

static double project(int n, const double* xi, const double* x) {
    double u = xi[0] * x[0];
    for (int a = 1; a < n; ++a) u = fma(xi[a], x[a], u);
    return u;
}

/* smallest j with t[j] >= u, or M if none */
static int first_threshold_at_or_above(const double* t, int M, double u) {
    int lo = 0, hi = M;
    while (lo < hi) {
        int mid = lo + (hi - lo) / 2;
        if (t[mid] >= u) hi = mid; else lo = mid + 1;
    }
    return lo;
}

/* ECT(xi_d, t_j) for every direction d and threshold j (int32 out[d][j]). */
int oracle_ect(int n, const int32_t* dims, const int32_t* px, int construction,
               const double* origin, const double* spacing,
               int ndirs, const double* dirs, int M, const double* thr, int32_t* out) {
    ogrid g;
    if (grid_init(&g, n, dims, construction, origin, spacing) || M < 1) return 1;
    for (int j = 1; j < M; ++j) if (!(thr[j] >= thr[j - 1])) return 2;
    cellset cs;
    if (cellset_build(&g, px, construction, 0, &cs)) return 3;
    double* x = vertex_coords(&g);
    if (!x) { cellset_free(&cs); return 3; }
    int err = 0;
#pragma omp parallel
    {
        double* u = (double*)malloc(sizeof(double) * g.nvert);
        long long* hist = (long long*)malloc(sizeof(long long) * (M + 1));
        if (!u || !hist) {
#pragma omp atomic write
            err = 3;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int d = 0; d < ndirs; ++d) {
                const double* xi = dirs + (long long)d * n;
                for (long long v = 0; v < g.nvert; ++v) u[v] = project(n, xi, x + v * MAXD);
                memset(hist, 0, sizeof(long long) * (M + 1));
                for (long long i = 0; i < cs.count; ++i) {
                    double top = u[cs.verts[i * MAXV]];
                    for (int q = 1; q < cs.nv[i]; ++q) {
                        double w = u[cs.verts[i * MAXV + q]];
                        if (w > top) top = w;
                    }
                    long long contrib = (cs.dim[i] & 1) ? -(long long)cs.value[i] : (long long)cs.value[i];
                    hist[first_threshold_at_or_above(thr, M, top)] += contrib;
                }
                long long run = 0;
                for (int j = 0; j < M; ++j) { run += hist[j]; out[(long long)d * M + j] = (int32_t)run; }
            }
        }
        free(u); free(hist);
    }
    free(x);
    cellset_free(&cs);
    return err;
}


/* ---- compensated accumulation ----
 * The cell form sums, per cell, kbar at its top vertex minus kbar at its
 * bottom vertex.  At a vertex that is not critical these contributions cancel
 * exactly in exact arithmetic, but in plain FP64 they leave rounding residues
 * of the size of the largest term, which can exceed the value of the
 * transform itself (Laplace kernel at large phases).  Every product is split
 * with TwoProduct (fma) and every addition with TwoSum (Knuth), so that the
 * sum is evaluated as in doubled precision (Ogita, Rump, Oishi, "Accurate sum
 * and dot product", SIAM J. Sci. Comput. 2005, algorithms Sum2 / Dot2). */
typedef struct { double hi, lo; } csum;

static void csum_add(csum* a, double x) {
    double t = a->hi + x;
    double bp = t - a->hi;
    double err = (a->hi - (t - bp)) + (x - bp);
    a->hi = t;
    a->lo += err;
}

/* a += w * v with w an integer weight (exactly representable) */
static void csum_axpy(csum* a, double w, double v) {
    double p = w * v;
    double e = fma(w, v, -p);
    csum_add(a, p);
    csum_add(a, e);
}

/* a += w * x * v */
static void csum_axpy3(csum* a, double w, double x, double v) {
    double p = x * v;
    double e = fma(x, v, -p);
    csum_axpy(a, w, p);
    csum_axpy(a, w, e);
}

static double csum_value(const csum* a) { return a->hi + a->lo; }

/* ---- kernels ---- */

/* Ji0(z) = integral_0^z J0(t) dt by composite 10-point Gauss-Legendre over unit
 * panels of glibc's j0.  The integral up to each integer is memoised in a
 * per-thread table, which only avoids recomputing identical panel sums. */
static const double GL_X[10] = {
    -0.9739065285171717, -0.8650633666889845, -0.6794095682990244, -0.4333953941292472,
    -0.1488743389816312,  0.1488743389816312,  0.4333953941292472,  0.6794095682990244,
     0.8650633666889845,  0.9739065285171717};
static const double GL_W[10] = {
    0.0666713443086881, 0.1494513491505806, 0.2190863625159820, 0.2692667193099963,
    0.2955242247147529, 0.2955242247147529, 0.2692667193099963, 0.2190863625159820,
    0.1494513491505806, 0.0666713443086881};

static double gl_panel(double a, double b) {
    double mid = 0.5 * (a + b), half = 0.5 * (b - a), s = 0.0;
    for (int i = 0; i < 10; ++i) s += GL_W[i] * j0(mid + half * GL_X[i]);
    return s * half;
}

typedef struct { double* cum; int len; } ji0_table;

static double ji0_eval(ji0_table* tb, double z) {
    double az = fabs(z);
    int k = (int)floor(az);
    if (k + 1 > tb->len) {
        int nl = k + 64;
        double* nc = (double*)realloc(tb->cum, sizeof(double) * nl);
        if (!nc) return NAN;
        if (tb->len == 0) { nc[0] = 0.0; tb->len = 1; }
        for (int i = tb->len; i < nl; ++i) nc[i] = nc[i - 1] + gl_panel((double)(i - 1), (double)i);
        tb->cum = nc;
        tb->len = nl;
    }
    double r = tb->cum[k] + (az > k ? gl_panel((double)k, az) : 0.0);
    return z < 0 ? -r : r;
}

double oracle_ji0(double z) {
    ji0_table tb = {NULL, 0};
    double r = ji0_eval(&tb, z);
    free(tb.cum);
    return r;
}

/* Hybrid transform at each query vector, by the cell form of the defining
 * integral.  out: Fourier [q][2] = (Re, Im); others [q].  For Laplace a per-query
 * shift m = max over the vertices of the contributing cells of (-s u) is
 * applied when shift != NULL: out = HT * exp(-m), shift[q] = m.  For the other
 * kernels shift (if given) is set to 0. */
int oracle_hybrid(int n, const int32_t* dims, const int32_t* px, int construction,
                  const double* origin, const double* spacing,
                  int nq, const double* xi_all, int kernel, double s,
                  double* out, double* shift) {
    ogrid g;
    if (grid_init(&g, n, dims, construction, origin, spacing)) return 1;
    if (!(s == s)) return 1;
    cellset cs;
    if (cellset_build(&g, px, construction, 1, &cs)) return 3;
    double* x = vertex_coords(&g);
    if (!x) { cellset_free(&cs); return 3; }
    /* vertices touched by contributing cells */
    unsigned char* used = (unsigned char*)calloc(g.nvert ? g.nvert : 1, 1);
    for (long long i = 0; i < cs.count; ++i)
        for (int q = 0; q < cs.nv[i]; ++q) used[cs.verts[i * MAXV + q]] = 1;
    int err = 0;
#pragma omp parallel
    {
        double* u = (double*)malloc(sizeof(double) * g.nvert);
        double* kr = (double*)malloc(sizeof(double) * g.nvert);
        double* ki = (double*)malloc(sizeof(double) * g.nvert);
        ji0_table tb = {NULL, 0};
        if (!u || !kr || !ki) {
#pragma omp atomic write
            err = 3;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int qi = 0; qi < nq; ++qi) {
                const double* xi = xi_all + (long long)qi * n;
                double m = 0.0;
                int have_m = 0;
                for (long long v = 0; v < g.nvert; ++v) {
                    if (!used[v]) continue;
                    u[v] = project(n, xi, x + v * MAXD);
                    double e = -s * u[v];
                    if (!have_m || e > m) { m = e; have_m = 1; }
                }
                if (kernel != OR_LAPLACE || !shift || s == 0.0) m = 0.0;
                for (long long v = 0; v < g.nvert; ++v) {
                    if (!used[v]) continue;
                    double z = s * u[v];
                    /* s = 0: kappa_0 is the constant kappa(0) = 1 for every kernel, with primitive t */
                    if (s == 0.0) { kr[v] = u[v]; ki[v] = 0.0; }
                    else if (kernel == OR_FOURIER) { kr[v] = sin(z) / s; ki[v] = cos(z) / s; }
                    else if (kernel == OR_LAPLACE) { kr[v] = -exp(-z - m) / s; ki[v] = 0.0; }
                    else { kr[v] = ji0_eval(&tb, z) / s; ki[v] = 0.0; }
                }
                csum ar = {0.0, 0.0}, ai = {0.0, 0.0};
                for (long long i = 0; i < cs.count; ++i) {
                    long long top = cs.verts[i * MAXV], bot = top;
                    for (int q = 1; q < cs.nv[i]; ++q) {
                        long long w = cs.verts[i * MAXV + q];
                        if (u[w] > u[top]) top = w;
                        if (u[w] < u[bot]) bot = w;
                    }
                    double sg = (cs.dim[i] & 1) ? (double)cs.value[i] : -(double)cs.value[i];
                    csum_axpy(&ar, sg, kr[top]);
                    csum_axpy(&ar, -sg, kr[bot]);
                    csum_axpy(&ai, sg, ki[top]);
                    csum_axpy(&ai, -sg, ki[bot]);
                }
                if (kernel == OR_FOURIER) { out[2LL * qi] = csum_value(&ar); out[2LL * qi + 1] = csum_value(&ai); }
                else out[qi] = csum_value(&ar);
                if (shift) shift[qi] = m;
            }
        }
        free(u); free(kr); free(ki); free(tb.cum);
    }
    free(used);
    free(x);
    cellset_free(&cs);
    return err;
}

/* Vector-Jacobian product of the unshifted hybrid transform.
 * gout: Fourier [q][2], others [q].  gxi[q][a] = sum_c gout_c dHT_c/dxi_a;
 * gs (if not NULL) = sum over q and c of gout_c dHT_c/ds.
 * d kbar_s(u)/d xi_a = kappa(s u) x_a;  dHT/ds = (1/s)[sum sg phi (u kappa(su))|_bot^top - HT]. */
int oracle_hybrid_grad(int n, const int32_t* dims, const int32_t* px, int construction,
                       const double* origin, const double* spacing,
                       int nq, const double* xi_all, int kernel, double s,
                       const double* gout, double* gxi, double* gs) {
    ogrid g;
    if (grid_init(&g, n, dims, construction, origin, spacing)) return 1;
    if (!(s == s) || (s == 0.0)) return 1;
    cellset cs;
    if (cellset_build(&g, px, construction, 1, &cs)) return 3;
    double* x = vertex_coords(&g);
    if (!x) { cellset_free(&cs); return 3; }
    unsigned char* used = (unsigned char*)calloc(g.nvert ? g.nvert : 1, 1);
    for (long long i = 0; i < cs.count; ++i)
        for (int q = 0; q < cs.nv[i]; ++q) used[cs.verts[i * MAXV + q]] = 1;
    double* gs_part = (double*)calloc(nq > 0 ? nq : 1, sizeof(double));
    int err = 0;
#pragma omp parallel
    {
        double* u = (double*)malloc(sizeof(double) * g.nvert);
        double* kb = (double*)malloc(sizeof(double) * 2 * g.nvert);  /* g-weighted kbar_s */
        double* kp = (double*)malloc(sizeof(double) * g.nvert);      /* g-weighted kappa(su) */
        ji0_table tb = {NULL, 0};
        if (!u || !kb || !kp) {
#pragma omp atomic write
            err = 3;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int qi = 0; qi < nq; ++qi) {
                const double* xi = xi_all + (long long)qi * n;
                double gr = kernel == OR_FOURIER ? gout[2LL * qi] : gout[qi];
                double gi = kernel == OR_FOURIER ? gout[2LL * qi + 1] : 0.0;
                for (long long v = 0; v < g.nvert; ++v) {
                    if (!used[v]) continue;
                    u[v] = project(n, xi, x + v * MAXD);
                    double z = s * u[v];
                    if (kernel == OR_FOURIER) {
                        kb[v] = (gr * sin(z) + gi * cos(z)) / s;
                        kp[v] = gr * cos(z) - gi * sin(z);
                    } else if (kernel == OR_LAPLACE) {
                        kb[v] = -gr * exp(-z) / s;
                        kp[v] = gr * exp(-z);
                    } else {
                        kb[v] = gr * ji0_eval(&tb, z) / s;
                        kp[v] = gr * j0(z);
                    }
                }
                csum acc[MAXD];
                for (int a = 0; a < MAXD; ++a) acc[a].hi = acc[a].lo = 0.0;
                csum du = {0.0, 0.0}, y = {0.0, 0.0};
                for (long long i = 0; i < cs.count; ++i) {
                    long long top = cs.verts[i * MAXV], bot = top;
                    for (int q = 1; q < cs.nv[i]; ++q) {
                        long long w = cs.verts[i * MAXV + q];
                        if (u[w] > u[top]) top = w;
                        if (u[w] < u[bot]) bot = w;
                    }
                    double sg = (cs.dim[i] & 1) ? (double)cs.value[i] : -(double)cs.value[i];
                    for (int a = 0; a < n; ++a) {
                        csum_axpy3(&acc[a], sg, x[top * MAXD + a], kp[top]);
                        csum_axpy3(&acc[a], -sg, x[bot * MAXD + a], kp[bot]);
                    }
                    csum_axpy3(&du, sg, u[top], kp[top]);
                    csum_axpy3(&du, -sg, u[bot], kp[bot]);
                    csum_axpy(&y, sg, kb[top]);
                    csum_axpy(&y, -sg, kb[bot]);
                }
                for (int a = 0; a < n; ++a) gxi[(long long)qi * n + a] = csum_value(&acc[a]);
                gs_part[qi] = (csum_value(&du) - csum_value(&y)) / s;
            }
        }
        free(u); free(kb); free(kp); free(tb.cum);
    }
    if (gs) {
        double t = 0.0;
        for (int qi = 0; qi < nq; ++qi) t += gs_part[qi];
        *gs = t;
    }
    free(gs_part);
    free(used);
    free(x);
    cellset_free(&cs);
    return err;
}

/* Critical values at every vertex for every sign vector eps (index e: bit a set
 * means eps_a = -1).  The lower star of vertex x for eps is the set of cells of
 * its star on which x is the highest vertex for any xi of sign eps: along every
 * axis where the cell extends, it extends towards -eps_a.  The upper star is
 * the mirror image.  lower[v][e] = chi(phi | LwSt), ordinary[v][e] =
 * chi(phi | UpSt) - chi(phi | LwSt). */
int oracle_critical_values(int n, const int32_t* dims, const int32_t* px, int construction,
                           int32_t* lower, int32_t* ordinary) {
    ogrid g;
    if (grid_init(&g, n, dims, construction, NULL, NULL)) return 1;
    const int ne = 1 << n;
#pragma omp parallel for schedule(static)
    for (long long v = 0; v < g.nvert; ++v) {
        int k[MAXD] = {0};
        long long r = v;
        for (int a = 0; a < n; ++a) { k[a] = (int)(r % g.V[a]); r /= g.V[a]; }
        /* the star of the vertex: offsets in {-1, 0, 1} along the image's axes */
        int olo[MAXD], ohi[MAXD];
        for (int a = 0; a < MAXD; ++a) { olo[a] = a < n ? -1 : 0; ohi[a] = a < n ? 1 : 0; }
        for (int e = 0; e < ne; ++e) {
            long long lw = 0, up = 0;
            int off[MAXD];
            for (int a = 0; a < MAXD; ++a) off[a] = olo[a];
            do {
                int c[MAXD] = {0};
                int inside = 1, is_low = 1, is_up = 1;
                for (int a = 0; a < n; ++a) {
                    c[a] = 2 * k[a] + off[a];
                    if (c[a] < 0 || c[a] > 2 * g.N[a]) inside = 0;
                    int eps = (e >> a) & 1 ? -1 : 1;
                    if (off[a] != 0 && off[a] != -eps) is_low = 0;
                    if (off[a] != 0 && off[a] != eps) is_up = 0;
                }
                if (!inside || (!is_low && !is_up)) continue;
                long long val = cell_value(&g, c, px, construction);
                if (cell_dim(&g, c) & 1) val = -val;
                if (is_low) lw += val;
                if (is_up) up += val;
            } while (box_next(off, olo, ohi, 1));
            lower[v * ne + e] = (int32_t)lw;
            ordinary[v * ne + e] = (int32_t)(up - lw);
        }
    }
    return 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* Ji0 at many arguments (one shared memo table). */
void oracle_ji0_array(long long n, const double* z, double* out) {
    ji0_table tb = {NULL, 0};
    for (long long i = 0; i < n; ++i) out[i] = ji0_eval(&tb, z[i]);
    free(tb.cum);
}

/* Radon transform R(xi_d, t_j) = chi of the slice {<xi_d, .> = t_j} (Sec. 2.2),
 * for every direction d and threshold j (int32 out[d][j]).  Written out from
 * the cells: a cell whose vertices all project to t lies in the slice and
 * contributes (-1)^dim phi (every vertex does at its projection, and so does a
 * cell of positive dimension when xi is not generic); a cell of dimension >= 1
 * with min < t < max over its vertices' projections is cut through its
 * relative interior, the cut has one dimension less, and it contributes
 * (-1)^(dim-1) phi.  (At t = min or t = max of a cell with min < max the slice
 * meets only a proper face, which is a cell of its own.)  Thresholds must be
 * non-decreasing; the open-interval contributions go through a difference
 * array over threshold indices. */
int oracle_radon(int n, const int32_t* dims, const int32_t* px, int construction,
                 const double* origin, const double* spacing,
                 int ndirs, const double* dirs, int M, const double* thr, int32_t* out) {
    ogrid g;
    if (grid_init(&g, n, dims, construction, origin, spacing) || M < 1) return 1;
    for (int j = 1; j < M; ++j) if (!(thr[j] >= thr[j - 1])) return 2;
    cellset cs;
    if (cellset_build(&g, px, construction, 0, &cs)) return 3;
    double* x = vertex_coords(&g);
    if (!x) { cellset_free(&cs); return 3; }
    int err = 0;
#pragma omp parallel
    {
        double* u = (double*)malloc(sizeof(double) * g.nvert);
        long long* diff = (long long*)malloc(sizeof(long long) * (M + 1));
        long long* point = (long long*)malloc(sizeof(long long) * M);
        if (!u || !diff || !point) {
#pragma omp atomic write
            err = 3;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int d = 0; d < ndirs; ++d) {
                const double* xi = dirs + (long long)d * n;
                for (long long v = 0; v < g.nvert; ++v) u[v] = project(n, xi, x + v * MAXD);
                memset(diff, 0, sizeof(long long) * (M + 1));
                memset(point, 0, sizeof(long long) * M);
                for (long long i = 0; i < cs.count; ++i) {
                    double lo = u[cs.verts[i * MAXV]], hi = lo;
                    for (int q = 1; q < cs.nv[i]; ++q) {
                        const double w = u[cs.verts[i * MAXV + q]];
                        if (w < lo) lo = w;
                        if (w > hi) hi = w;
                    }
                    if (lo == hi) {   /* the whole cell lies in the slice at t = lo */
                        const long long c = (cs.dim[i] & 1) ? -(long long)cs.value[i] : (long long)cs.value[i];
                        for (int j = first_threshold_at_or_above(thr, M, lo); j < M && thr[j] == lo; ++j)
                            point[j] += c;
                        continue;
                    }
                    /* thresholds with lo < t < hi: indices [j0, j1) */
                    int j0 = first_threshold_at_or_above(thr, M, lo);
                    while (j0 < M && thr[j0] == lo) ++j0;
                    const int j1 = first_threshold_at_or_above(thr, M, hi);
                    if (j0 >= j1) continue;
                    const long long s = (cs.dim[i] & 1) ? (long long)cs.value[i] : -(long long)cs.value[i];
                    diff[j0] += s;
                    diff[j1] -= s;
                }
                long long run = 0;
                for (int j = 0; j < M; ++j) {
                    run += diff[j];
                    out[(long long)d * M + j] = (int32_t)(run + point[j]);
                }
            }
        }
        free(u); free(diff); free(point);
    }
    free(x);
    cellset_free(&cs);
    return err;
}

/* Canonical FP64 projections <xi, x_v> of every vertex (the expression the
 * ECT is defined with), in linear vertex order. */
int oracle_vertex_projections(int n, const int32_t* dims, int construction, const double* origin,
                              const double* spacing, const double* xi, double* out) {
    ogrid g;
    if (grid_init(&g, n, dims, construction, origin, spacing)) return 1;
    double* x = vertex_coords(&g);
    if (!x) return 3;
    for (long long v = 0; v < g.nvert; ++v) out[v] = project(n, xi, x + v * MAXD);
    free(x);
    return 0;
}
