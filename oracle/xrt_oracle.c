/*
 * Plain FP64 CPU reference of the discrete X-ray transform -- TEST INFRASTRUCTURE.
 * The definition it implements is stated in xrt_oracle.h.  Pinned by
 * tests/test_oracle_*.py against the paper's worked examples (Sec. 5, Tables
 * test_2D_parallel .. test_helical_cone), the ambiguity examples of Sec. 4.1,
 * a per-unit brute force, chord lengths and the adjoint identity.
 */
#include "xrt_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Geometry in "unit coordinates": u_a = (x_a - c_a) / d_a.  In these the unit boxes
 * are the paper's unit-scale supports (Sec. 2.1: Omega_ji; Sec. 3.2.1: Omega_kji):
 *   x planes u_x = i - nx/2,  y planes u_y = ny/2 - j,  z planes u_z = nz/2 - k. */
typedef struct {
    int dim;
    int n[3];
    double d[3];
    double c[3];
} ogrid;

static void make_grid(const ora_grid* g, ogrid* o)
{
    o->dim = g->nz > 0 ? 3 : 2;
    o->n[0] = g->nx; o->n[1] = g->ny; o->n[2] = g->nz > 0 ? g->nz : 1;
    o->d[0] = g->dx; o->d[1] = g->dy; o->d[2] = g->nz > 0 ? g->dz : 1.0;
    o->c[0] = g->cx; o->c[1] = g->cy; o->c[2] = g->nz > 0 ? g->cz : 0.0;
}

/* Ray in unit coordinates: pu + t*wu, with t the physical arc length along the ray. */
static void to_unit(const ogrid* o, const double* p, const double* th, double* pu, double* wu)
{
    for (int a = 0; a < 3; ++a) { pu[a] = 0.0; wu[a] = 0.0; }
    for (int a = 0; a < o->dim; ++a) {
        pu[a] = (p[a] - o->c[a]) / o->d[a];
        wu[a] = th[a] / o->d[a];
    }
}

/* Continuous index coordinate along axis a: its floor is the unit index
 * (i = floor(u_x + nx/2), j = floor(ny/2 - u_y), k = floor(nz/2 - u_z)). */
static double index_coord(const ogrid* o, int a, double u)
{
    double half = 0.5 * o->n[a];
    return a == 0 ? u + half : half - u;
}

/* Clip the line to the image box.  Axes along which the ray does not move use the
 * half-open membership test (the ray belongs to the unit with the bigger index).
 * Returns 0 when the chord is empty. */
static int clip(const ogrid* o, const double* pu, const double* wu, double* tin, double* tout)
{
    double lo = -INFINITY, hi = INFINITY;
    for (int a = 0; a < o->dim; ++a) {
        double half = 0.5 * o->n[a];
        if (wu[a] != 0.0) {
            double t0 = (-half - pu[a]) / wu[a];
            double t1 = (half - pu[a]) / wu[a];
            lo = fmax(lo, fmin(t0, t1));
            hi = fmin(hi, fmax(t0, t1));
        } else {
            double q = index_coord(o, a, pu[a]);
            if (!(q >= 0.0 && q < (double)o->n[a])) return 0;
        }
    }
    if (!(lo < hi)) return 0;
    *tin = lo;
    *tout = hi;
    return 1;
}

static int cmp_double(const void* a, const void* b)
{
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

/* All grid-plane crossings strictly inside (tin, tout), sorted increasingly. */
static long crossings(const ogrid* o, const double* pu, const double* wu,
                      double tin, double tout, double* buf)
{
    long m = 0;
    for (int a = 0; a < o->dim; ++a) {
        if (wu[a] == 0.0) continue;
        double half = 0.5 * o->n[a];
        for (int q = 1; q < o->n[a]; ++q) {
            double plane = a == 0 ? (double)q - half : half - (double)q;
            double t = (plane - pu[a]) / wu[a];
            if (t > tin && t < tout) buf[m++] = t;
        }
    }
    qsort(buf, (size_t)m, sizeof(double), cmp_double);
    return m;
}

/* Visit every piece of the chord: calls fn(I, length) for pieces of positive length. */
typedef void (*visit_fn)(void* ctx, long I, double len);

static void walk(const ogrid* o, const double* p, const double* th, double* buf,
                 visit_fn fn, void* ctx)
{
    double pu[3], wu[3], tin, tout;
    to_unit(o, p, th, pu, wu);
    if (!clip(o, pu, wu, &tin, &tout)) return;
    long m = crossings(o, pu, wu, tin, tout, buf);
    double prev = tin;
    for (long s = 0; s <= m; ++s) {
        double next = s < m ? buf[s] : tout;
        if (next > prev) {
            double mid = 0.5 * (prev + next);
            long idx[3] = {0, 0, 0};
            int ok = 1;
            for (int a = 0; a < o->dim; ++a) {
                double q = index_coord(o, a, pu[a] + mid * wu[a]);
                double f = floor(q);
                if (f < 0.0 || f >= (double)o->n[a]) { ok = 0; break; }
                idx[a] = (long)f;
            }
            if (ok) {
                long I = (idx[2] * o->n[1] + idx[1]) * (long)o->n[0] + idx[0];
                fn(ctx, I, next - prev);
            }
        }
        prev = next;
    }
}

static long max_crossings(const ogrid* o)
{
    return (long)o->n[0] + o->n[1] + o->n[2] + 8;
}

static long n_units(const ogrid* o)
{
    return (long)o->n[0] * o->n[1] * o->n[2];
}

/* ---------------------------------------------------------------- forward */

typedef struct { const double* img; double acc; } fwd_ctx;

static void fwd_visit(void* c, long I, double len)
{
    fwd_ctx* f = (fwd_ctx*)c;
    f->acc += f->img[I] * len;
}

void ora_forward(const ora_grid* g, long nrays, const double* p, const double* th,
                 const double* img, double* out, int nthreads)
{
    ogrid o;
    make_grid(g, &o);
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
    {
        double* buf = (double*)malloc(sizeof(double) * (size_t)max_crossings(&o));
#pragma omp for schedule(dynamic, 64)
        for (long r = 0; r < nrays; ++r) {
            fwd_ctx c = {img, 0.0};
            walk(&o, p + 3 * r, th + 3 * r, buf, fwd_visit, &c);
            out[r] = c.acc;
        }
        free(buf);
    }
}

/* ---------------------------------------------------------------- adjoint */

typedef struct { double* img; double w; } adj_ctx;

static void adj_visit(void* c, long I, double len)
{
    adj_ctx* a = (adj_ctx*)c;
    a->img[I] += a->w * len;
}

void ora_adjoint(const ora_grid* g, long nrays, const double* p, const double* th,
                 const double* sino, double* img, int nthreads)
{
    ogrid o;
    make_grid(g, &o);
    long nv = n_units(&o);
    if (nthreads < 1) nthreads = 1;
    double* part = (double*)calloc((size_t)nthreads * (size_t)nv, sizeof(double));
#pragma omp parallel num_threads(nthreads)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* mine = part + (size_t)tid * (size_t)nv;
        double* buf = (double*)malloc(sizeof(double) * (size_t)max_crossings(&o));
#pragma omp for schedule(static)
        for (long r = 0; r < nrays; ++r) {
            if (sino[r] == 0.0) continue;
            adj_ctx c = {mine, sino[r]};
            walk(&o, p + 3 * r, th + 3 * r, buf, adj_visit, &c);
        }
        free(buf);
    }
    /* fixed-order reduction: deterministic for a given thread count */
    memset(img, 0, sizeof(double) * (size_t)nv);
    for (int t = 0; t < nthreads; ++t) {
        const double* src = part + (size_t)t * (size_t)nv;
        for (long I = 0; I < nv; ++I) img[I] += src[I];
    }
    free(part);
}

/* ---------------------------------------------------------------- hit lists */

typedef struct { long* idx; double* len; long n, cap; double eps; } hit_ctx;

static void hit_visit(void* c, long I, double len)
{
    hit_ctx* h = (hit_ctx*)c;
    if (!(len > h->eps)) return;
    if (h->n < h->cap) {
        h->idx[h->n] = I;
        h->len[h->n] = len;
    }
    h->n++;
}

long ora_ray_hits(const ora_grid* g, const double* p, const double* th,
                  long* idx, double* len, long cap, double eps)
{
    ogrid o;
    make_grid(g, &o);
    double* buf = (double*)malloc(sizeof(double) * (size_t)max_crossings(&o));
    hit_ctx h = {idx, len, 0, cap, eps};
    walk(&o, p, th, buf, hit_visit, &h);
    free(buf);
    long n = h.n < cap ? h.n : cap;
    /* sort by 1D index (insertion sort: hit lists are O(N) long) */
    for (long a = 1; a < n; ++a) {
        long ki = idx[a];
        double kl = len[a];
        long b = a - 1;
        while (b >= 0 && idx[b] > ki) {
            idx[b + 1] = idx[b];
            len[b + 1] = len[b];
            --b;
        }
        idx[b + 1] = ki;
        len[b + 1] = kl;
    }
    return h.n;
}

typedef struct { long n; double eps; } cnt_ctx;

static void cnt_visit(void* c, long I, double len)
{
    (void)I;
    cnt_ctx* k = (cnt_ctx*)c;
    if (len > k->eps) k->n++;
}

void ora_hit_counts(const ora_grid* g, long nrays, const double* p, const double* th,
                    double eps, long* counts, int nthreads)
{
    ogrid o;
    make_grid(g, &o);
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
    {
        double* buf = (double*)malloc(sizeof(double) * (size_t)max_crossings(&o));
#pragma omp for schedule(dynamic, 64)
        for (long r = 0; r < nrays; ++r) {
            cnt_ctx c = {0, eps};
            walk(&o, p + 3 * r, th + 3 * r, buf, cnt_visit, &c);
            counts[r] = c.n;
        }
        free(buf);
    }
}

double ora_chord(const ora_grid* g, const double* p, const double* th)
{
    ogrid o;
    make_grid(g, &o);
    double pu[3], wu[3], tin, tout;
    to_unit(&o, p, th, pu, wu);
    if (!clip(&o, pu, wu, &tin, &tout)) return 0.0;
    return tout - tin;
}

/* ---------------------------------------------------------------- attenuated transform */
/*
 * Generalised Radon transform with an exponential attenuation weight (Introduction,
 * eq. generalizedRadontransform, the SPECT case): Phi(t) = exp(-int_t^inf mu(p + s th) ds),
 * i.e. the attenuation between the point and the detector side (+th) of the ray, for a
 * unit-wise constant attenuation map mu.  For the pieces of the chord, in order of
 * increasing t, with lengths len_i, values f_i, mu_i and A_i = sum_{j > i} mu_j len_j:
 *   g = sum_i f_i exp(-A_i) (1 - exp(-mu_i len_i)) / mu_i     (f_i len_i when mu_i = 0),
 * the exact integral of f Phi over each piece.
 */
typedef struct { long* idx; double* len; long n; } piece_ctx;

static void piece_visit(void* c, long I, double len)
{
    piece_ctx* p = (piece_ctx*)c;
    p->idx[p->n] = I;
    p->len[p->n] = len;
    ++p->n;
}

static double piece_weight(double mu, double len)
{
    double x = mu * len;
    return x != 0.0 ? -expm1(-x) / mu : len;
}

void ora_forward_att(const ora_grid* g, long nrays, const double* p, const double* th,
                     const double* img, const double* mu, double* out, int nthreads)
{
    ogrid o;
    make_grid(g, &o);
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
    {
        long cap = max_crossings(&o) + 1;
        double* buf = (double*)malloc(sizeof(double) * (size_t)max_crossings(&o));
        long* idx = (long*)malloc(sizeof(long) * (size_t)cap);
        double* len = (double*)malloc(sizeof(double) * (size_t)cap);
#pragma omp for schedule(dynamic, 64)
        for (long r = 0; r < nrays; ++r) {
            piece_ctx c = {idx, len, 0};
            walk(&o, p + 3 * r, th + 3 * r, buf, piece_visit, &c);
            double acc = 0.0, A = 0.0;
            for (long i = c.n - 1; i >= 0; --i) {
                double m = mu[idx[i]];
                acc += img[idx[i]] * exp(-A) * piece_weight(m, len[i]);
                A += m * len[i];
            }
            out[r] = acc;
        }
        free(len);
        free(idx);
        free(buf);
    }
}

void ora_adjoint_att(const ora_grid* g, long nrays, const double* p, const double* th,
                     const double* sino, const double* mu, double* img, int nthreads)
{
    ogrid o;
    make_grid(g, &o);
    long nv = n_units(&o);
    if (nthreads < 1) nthreads = 1;
    double* part = (double*)calloc((size_t)nthreads * (size_t)nv, sizeof(double));
#pragma omp parallel num_threads(nthreads)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* mine = part + (size_t)tid * (size_t)nv;
        long cap = max_crossings(&o) + 1;
        double* buf = (double*)malloc(sizeof(double) * (size_t)max_crossings(&o));
        long* idx = (long*)malloc(sizeof(long) * (size_t)cap);
        double* len = (double*)malloc(sizeof(double) * (size_t)cap);
#pragma omp for schedule(static)
        for (long r = 0; r < nrays; ++r) {
            if (sino[r] == 0.0) continue;
            piece_ctx c = {idx, len, 0};
            walk(&o, p + 3 * r, th + 3 * r, buf, piece_visit, &c);
            double A = 0.0;
            for (long i = c.n - 1; i >= 0; --i) {
                double m = mu[idx[i]];
                mine[idx[i]] += sino[r] * exp(-A) * piece_weight(m, len[i]);
                A += m * len[i];
            }
        }
        free(len);
        free(idx);
        free(buf);
    }
    memset(img, 0, sizeof(double) * (size_t)nv);
    for (int t = 0; t < nthreads; ++t) {
        const double* src = part + (size_t)t * (size_t)nv;
        for (long I = 0; I < nv; ++I) img[I] += src[I];
    }
    free(part);
}


/* ---------------------------------------------------------------- simplex basis
 * The image on the simplices of a structured triangulation (the paper's polygonal /
 * polyhedral extension, Introduction "Contributions" and Sec. 4.2): in index
 * coordinates xi (xi_a = its floor is the unit index along axis a) every pixel is cut
 * into 2 triangles by the plane xi_x - xi_y = const, every voxel into 6 tetrahedra by the
 * planes xi_x - xi_y, xi_y - xi_z, xi_x - xi_z = const (Kuhn's triangulation).  Simplex
 * s of unit I is the set of points whose local coordinates l_a = xi_a - floor(xi_a),
 * sorted from largest to smallest, come in the s-th order of the axes in lexicographic
 * order: 2D (x,y) = 0, (y,x) = 1; 3D (x,y,z) = 0, (x,z,y) = 1, (y,x,z) = 2,
 * (y,z,x) = 3, (z,x,y) = 4, (z,y,x) = 5.  Equal coordinates (within SIMPLEX_TIE) rank the
 * later axis first, which gives a point on a diagonal plane to the simplex with the
 * bigger index (the resolution of Sec. 4.1 carried to the new faces).  Simplex index =
 * I * S + s, S = 2 (2D) or 6 (3D).
 *
 * Method: the chord partition again, with the crossings of the diagonal plane families
 * xi_a - xi_b = integer added to those of the grid planes; each piece goes to the
 * simplex containing its midpoint. */

static long simplex_count(const ogrid* o) { return o->dim == 3 ? 6 : 2; }

static long max_crossings_simplex(const ogrid* o)
{
    return 3L * ((long)o->n[0] + o->n[1] + o->n[2]) + 16;
}

/* index coordinate of axis a along the ray: xi_a(t) = x0[a] + t * om[a] */
static void index_line(const ogrid* o, const double* pu, const double* wu, double* x0, double* om)
{
    for (int a = 0; a < 3; ++a) { x0[a] = 0.0; om[a] = 0.0; }
    for (int a = 0; a < o->dim; ++a) {
        x0[a] = index_coord(o, a, pu[a]);
        om[a] = a == 0 ? wu[a] : -wu[a];
    }
}

/* Local coordinates closer than this (index units) count as equal: a ray placed in a
 * diagonal face in exact arithmetic has coordinates that differ by rounding only (the
 * faces' counterpart of snapping tiny direction components to zero). */
#define SIMPLEX_TIE 1e-9

/* axis a ranks before axis b: larger coordinate, or equal and a the later axis */
static int ranks_before(const double* l, int a, int b)
{
    if (fabs(l[a] - l[b]) <= SIMPLEX_TIE) return a > b;
    return l[a] > l[b];
}

/* rank of the permutation that sorts the local coordinates (largest first, ties: the
 * later axis first), lexicographic over permutations */
static int simplex_of(int dim, const double* l)
{
    if (dim == 2) return ranks_before(l, 1, 0) ? 1 : 0;
    int ord[3] = {0, 1, 2};
    for (int i = 1; i < 3; ++i) {
        int k = ord[i], j = i - 1;
        while (j >= 0 && ranks_before(l, k, ord[j])) {
            ord[j + 1] = ord[j];
            --j;
        }
        ord[j + 1] = k;
    }
    static const int rank[3][3] = {{-1, 0, 1}, {2, -1, 3}, {4, 5, -1}};  /* [first][second] */
    return rank[ord[0]][ord[1]];
}

static void simplex_walk(const ogrid* o, const double* p, const double* th, double* buf,
                         visit_fn fn, void* ctx)
{
    double pu[3], wu[3], tin, tout, x0[3], om[3];
    to_unit(o, p, th, pu, wu);
    if (!clip(o, pu, wu, &tin, &tout)) return;
    index_line(o, pu, wu, x0, om);
    long m = 0;
    /* grid planes xi_a = integer */
    for (int a = 0; a < o->dim; ++a) {
        if (om[a] == 0.0) continue;
        for (int q = 1; q < o->n[a]; ++q) {
            double t = ((double)q - x0[a]) / om[a];
            if (t > tin && t < tout) buf[m++] = t;
        }
    }
    /* diagonal planes xi_a - xi_b = integer */
    static const int pairs[3][2] = {{0, 1}, {1, 2}, {0, 2}};
    int npairs = o->dim == 3 ? 3 : 1;
    for (int k = 0; k < npairs; ++k) {
        int a = pairs[k][0], b = pairs[k][1];
        double d0 = x0[a] - x0[b], dw = om[a] - om[b];
        if (dw == 0.0) continue;
        double e0 = d0 + tin * dw, e1 = d0 + tout * dw;
        double lo = fmin(e0, e1), hi = fmax(e0, e1);
        for (double q = ceil(lo); q <= floor(hi); q += 1.0) {
            double t = (q - d0) / dw;
            if (t > tin && t < tout) buf[m++] = t;
        }
    }
    qsort(buf, (size_t)m, sizeof(double), cmp_double);
    long S = simplex_count(o);
    double prev = tin;
    for (long s = 0; s <= m; ++s) {
        double next = s < m ? buf[s] : tout;
        if (next > prev) {
            double mid = 0.5 * (prev + next);
            long idx[3] = {0, 0, 0};
            double loc[3] = {0.0, 0.0, 0.0};
            int ok = 1;
            for (int a = 0; a < o->dim; ++a) {
                double q = x0[a] + mid * om[a];
                double f = floor(q);
                if (f < 0.0 || f >= (double)o->n[a]) { ok = 0; break; }
                idx[a] = (long)f;
                loc[a] = q - f;
            }
            if (ok) {
                long I = (idx[2] * o->n[1] + idx[1]) * (long)o->n[0] + idx[0];
                fn(ctx, I * S + simplex_of(o->dim, loc), next - prev);
            }
        }
        prev = next;
    }
}

void ora_forward_simplex(const ora_grid* g, long nrays, const double* p, const double* th,
                         const double* img, double* out, int nthreads)
{
    ogrid o;
    make_grid(g, &o);
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
    {
        double* buf = (double*)malloc(sizeof(double) * (size_t)max_crossings_simplex(&o));
#pragma omp for schedule(dynamic, 64)
        for (long r = 0; r < nrays; ++r) {
            fwd_ctx c = {img, 0.0};
            simplex_walk(&o, p + 3 * r, th + 3 * r, buf, fwd_visit, &c);
            out[r] = c.acc;
        }
        free(buf);
    }
}

void ora_adjoint_simplex(const ora_grid* g, long nrays, const double* p, const double* th,
                         const double* sino, double* img, int nthreads)
{
    ogrid o;
    make_grid(g, &o);
    long nv = n_units(&o) * simplex_count(&o);
    if (nthreads < 1) nthreads = 1;
    double* part = (double*)calloc((size_t)nthreads * (size_t)nv, sizeof(double));
#pragma omp parallel num_threads(nthreads)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* mine = part + (size_t)tid * (size_t)nv;
        double* buf = (double*)malloc(sizeof(double) * (size_t)max_crossings_simplex(&o));
#pragma omp for schedule(static)
        for (long r = 0; r < nrays; ++r) {
            if (sino[r] == 0.0) continue;
            adj_ctx c = {mine, sino[r]};
            simplex_walk(&o, p + 3 * r, th + 3 * r, buf, adj_visit, &c);
        }
        free(buf);
    }
    memset(img, 0, sizeof(double) * (size_t)nv);
    for (int t = 0; t < nthreads; ++t) {
        const double* src = part + (size_t)t * (size_t)nv;
        for (long I = 0; I < nv; ++I) img[I] += src[I];
    }
    free(part);
}

/* consecutive pieces of one simplex (split by a crossing that rounding placed inside
 * it) count as one hit */
typedef struct { long* idx; double* len; long n, cap; long last; double run; double eps; } shit_ctx;

static void shit_flush(shit_ctx* h)
{
    if (h->last >= 0 && h->run > h->eps) {
        if (h->n < h->cap) {
            h->idx[h->n] = h->last;
            h->len[h->n] = h->run;
        }
        h->n++;
    }
}

static void shit_visit(void* c, long I, double len)
{
    shit_ctx* h = (shit_ctx*)c;
    if (I == h->last) {
        h->run += len;
        return;
    }
    shit_flush(h);
    h->last = I;
    h->run = len;
}

long ora_ray_hits_simplex(const ora_grid* g, const double* p, const double* th,
                          long* idx, double* len, long cap, double eps)
{
    ogrid o;
    make_grid(g, &o);
    double* buf = (double*)malloc(sizeof(double) * (size_t)max_crossings_simplex(&o));
    shit_ctx h = {idx, len, 0, cap, -1, 0.0, eps};
    simplex_walk(&o, p, th, buf, shit_visit, &h);
    shit_flush(&h);
    free(buf);
    long n = h.n < cap ? h.n : cap;
    for (long a = 1; a < n; ++a) {
        long ki = idx[a];
        double kl = len[a];
        long b = a - 1;
        while (b >= 0 && idx[b] > ki) {
            idx[b + 1] = idx[b];
            len[b + 1] = len[b];
            --b;
        }
        idx[b + 1] = ki;
        len[b + 1] = kl;
    }
    return h.n;
}
