/*
 * Plain FP64 CPU oracle for one SPH hydro step.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or
 * load this file or the library built from it; only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark do. It shares no code,
 * header, table or constant generator with the HIP path.
 *
 * It follows the generic SPH workflow of Algorithm 1 (Sec. 3): find the
 * neighbours of every particle (step 2), evaluate density, pressure,
 * acceleration and rate of change of internal energy (step 3, as listed in
 * the prose after Algorithm 1), compute a new global time-step (step 5) and
 * update velocity and position (step 6). The paper names the ingredients but
 * not their formulas; the readings used (each a textbook choice) are:
 *
 *   kernel    M4 cubic spline (Table 1, ChaNGa), W = w(r/h) / (pi h^3); the
 *             mini-app's other interchangeable kernels (Sec. 4, Table 2)
 *             are selectable: Wendland C2 and the sinc family (orc_set_kernel)
 *   gradient  kernel derivatives, standard volume elements m/rho (Table 1);
 *             or the integral approach to derivatives (IAD, Table 1 for
 *             SPHYNX; orc_set_gradient), with the same volume elements
 *   volumes   standard (X = m), or SPHYNX's generalised volume elements
 *             (Table 1) with weights X (orc_density_weighted and
 *             orc_momentum_energy_weighted)
 *   density   summation, self term included, gather with h_i
 *   variable h  neighbour iff r^2 < (2 max(h_i, h_j))^2; gradient is the
 *             mean of grad W(r, h_i) and grad W(r, h_j)
 *   momentum  a_i = -sum_j m_j (P_i/rho_i^2 + P_j/rho_j^2 + Pi_ij) gradW_ij
 *   energy    du_i = 1/2 sum_j m_j (...) v_ij . gradW_ij
 *   AV        Monaghan: mu = hbar v.r / (r^2 + eta^2 hbar^2) if v.r < 0,
 *             Pi = (-alpha cbar mu + beta mu^2) / rhobar
 *   EOS       Tait (square patch) or ideal gas gamma = 5/3 (Evrard, Sec. 5.1)
 *   dt        global min over particles of the Courant and force limits
 *   update    kick-drift-kick leapfrog with a global dt
 *
 * Every sum over neighbours runs in ascending neighbour-index order. Built
 * with -O2 -ffp-contract=off so that no multiply-add is fused unless written
 * as fma() below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ---------------------------------------------------------------- kernel */

/* M4 cubic spline shape, q = r/h (Monaghan & Lattanzio 1985). */
static double m4_w(double q)
{
    if (q < 1.0) return 1.0 - 1.5 * q * q + 0.75 * q * q * q;
    if (q < 2.0) { double t = 2.0 - q; return 0.25 * t * t * t; }
    return 0.0;
}

/* dw/dq of the M4 shape. */
static double m4_dw(double q)
{
    if (q < 1.0) return -3.0 * q + 2.25 * q * q;
    if (q < 2.0) { double t = 2.0 - q; return -0.75 * t * t; }
    return 0.0;
}

/*
 * The other kernels of the mini-app's interchangeable set (Sec. 4, Table 2;
 * Table 1 names Wendland for ChaNGa and SPH-flow and the sinc family for
 * SPHYNX). All have support 2h, so the neighbour relation is unchanged.
 *
 * Wendland C2 in 3D (Wendland 1995), written for support H = 2h:
 *   W = 21 / (2 pi H^3) (1 - r/H)^4 (1 + 4 r/H)
 * which with q = r/h is 21 / (16 pi h^3) (1 - q/2)^4 (1 + 2q).
 *
 * Sinc family (Cabezon, Garcia-Senz & Relano 2008): with S(x) = sin(x)/x,
 *   W = B_n / h^3 S(pi q / 2)^n for q < 2,
 * B_n from the normalisation 4 pi int_0^2 q^2 S(pi q/2)^n dq = 1.
 */
static int32_t g_kernel = 0;     /* 0 M4, 1 Wendland C2, 2 sinc */
static int32_t g_sinc_n = 5;
static double g_sinc_b = 0.0;    /* B_n of the current exponent */

static double sinc_s(double x)
{
    if (x == 0.0) return 1.0;
    return sin(x) / x;
}

/* dS/dx = (x cos x - sin x) / x^2, with its series near 0 */
static double sinc_ds(double x)
{
    if (fabs(x) < 1e-4) return -x / 3.0 + x * x * x / 30.0;
    return (x * cos(x) - sin(x)) / (x * x);
}

static double sinc_shape(double q)
{
    if (q >= 2.0) return 0.0;
    return pow(sinc_s(0.5 * ORC_PI * q), (double)g_sinc_n);
}

/* B_n by composite Simpson's rule on [0, 2] */
static double sinc_norm(void)
{
    const int k = 20000;
    const double dq = 2.0 / k;
    double acc = 0.0;
    for (int i = 0; i <= k; ++i) {
        double q = i * dq;
        double f = q * q * sinc_shape(q);
        double wgt = (i == 0 || i == k) ? 1.0 : ((i & 1) ? 4.0 : 2.0);
        acc += wgt * f;
    }
    return 1.0 / (4.0 * ORC_PI * acc * dq / 3.0);
}

/* Select the kernel of orc_kernel_w/dwdr, orc_density and
 * orc_momentum_energy: 0 M4 (default), 1 Wendland C2, 2 sinc of exponent n
 * (3 <= n <= 12). Returns 0, or -1 for an unknown choice. Not thread-safe:
 * call it between evaluations. */
int32_t orc_set_kernel(int32_t family, int32_t n)
{
    if (family < 0 || family > 2) return -1;
    if (family == 2 && (n < 3 || n > 12)) return -1;
    g_kernel = family;
    if (family == 2) {
        g_sinc_n = n;
        g_sinc_b = sinc_norm();
    }
    return 0;
}

/* The normalisation constant of the current kernel: W(0, h) h^3. */
double orc_kernel_sigma(void)
{
    if (g_kernel == 1) return 21.0 / (16.0 * ORC_PI);
    if (g_kernel == 2) return g_sinc_b;
    return 1.0 / ORC_PI;
}

/* W(r, h) in 3D. */
double orc_kernel_w(double r, double h)
{
    double q = r / h;
    if (g_kernel == 1) {
        if (q >= 2.0) return 0.0;
        double t = 1.0 - 0.5 * q;
        return 21.0 / (16.0 * ORC_PI * h * h * h) * t * t * t * t * (1.0 + 2.0 * q);
    }
    if (g_kernel == 2) return g_sinc_b / (h * h * h) * sinc_shape(q);
    return m4_w(q) / (ORC_PI * h * h * h);
}

/* dW/dr (r, h) in 3D. */
double orc_kernel_dwdr(double r, double h)
{
    double q = r / h;
    if (g_kernel == 1) {
        if (q >= 2.0) return 0.0;
        double t = 1.0 - 0.5 * q;
        return -105.0 / (16.0 * ORC_PI * h * h * h * h) * q * t * t * t;
    }
    if (g_kernel == 2) {
        if (q >= 2.0) return 0.0;
        double x = 0.5 * ORC_PI * q;
        return g_sinc_b / (h * h * h * h) * (double)g_sinc_n *
               pow(sinc_s(x), (double)(g_sinc_n - 1)) * sinc_ds(x) * 0.5 * ORC_PI;
    }
    return m4_dw(q) / (ORC_PI * h * h * h * h);
}

/* ------------------------------------------------------------ geometry */

typedef struct {
    double lo[3], hi[3];
    int32_t periodic[3];
} orc_box;

/* Minimum image along one periodic axis of length len. */
static double min_image(double d, double len)
{
    double half = 0.5 * len;
    if (d > half) return d - len;
    if (d < -half) return d + len;
    return d;
}

/* Separation x_i - x_j with the minimum image on periodic axes. */
static void separation(const double *x, const double *y, const double *z,
                       int64_t i, int64_t j, const orc_box *b,
                       double *dx, double *dy, double *dz)
{
    double ex = x[i] - x[j], ey = y[i] - y[j], ez = z[i] - z[j];
    if (b->periodic[0]) ex = min_image(ex, b->hi[0] - b->lo[0]);
    if (b->periodic[1]) ey = min_image(ey, b->hi[1] - b->lo[1]);
    if (b->periodic[2]) ez = min_image(ez, b->hi[2] - b->lo[2]);
    *dx = ex; *dy = ey; *dz = ez;
}

/* Squared distance, evaluated in one fixed order:
 * r^2 = fma(dz, dz, fma(dy, dy, dx*dx)). */
static double dist2(double dx, double dy, double dz)
{
    return fma(dz, dz, fma(dy, dy, dx * dx));
}

/* The neighbour relation: j != i and r^2 < (2 max(h_i, h_j))^2, strict. */
static int is_neighbor(const double *x, const double *y, const double *z,
                       const double *h, int64_t i, int64_t j, const orc_box *b)
{
    double dx, dy, dz;
    if (i == j) return 0;
    separation(x, y, z, i, j, b, &dx, &dy, &dz);
    double s = 2.0 * fmax(h[i], h[j]);
    return dist2(dx, dy, dz) < s * s;
}

/* Gather-only relation used for smoothing-length counting: r^2 < 4 h_i^2. */
static int in_gather_sphere(const double *x, const double *y, const double *z,
                            const double *h, int64_t i, int64_t j,
                            const orc_box *b)
{
    double dx, dy, dz;
    if (i == j) return 0;
    separation(x, y, z, i, j, b, &dx, &dy, &dz);
    double s = 2.0 * h[i];
    return dist2(dx, dy, dz) < s * s;
}

static orc_box make_box(const double *lo, const double *hi, const int32_t *per)
{
    orc_box b;
    for (int a = 0; a < 3; ++a) {
        b.lo[a] = lo[a]; b.hi[a] = hi[a]; b.periodic[a] = per[a];
    }
    return b;
}

/* ------------------------------------------------- brute-force neighbours */

/*
 * O(N^2) neighbour sets, the definition written out. offsets has n+1
 * entries. If the total exceeds cap, ids is left partially written and the
 * needed total is returned; otherwise the total is returned.
 */
int64_t orc_neighbors_brute(int64_t n, const double *x, const double *y,
                            const double *z, const double *h,
                            const double *lo, const double *hi,
                            const int32_t *per, int64_t cap,
                            int64_t *offsets, int32_t *ids)
{
    orc_box b = make_box(lo, hi, per);
    int64_t *cnt = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j) c += is_neighbor(x, y, z, h, i, j, &b);
        cnt[i] = c;
    }
    offsets[0] = 0;
    for (int64_t i = 0; i < n; ++i) offsets[i + 1] = offsets[i] + cnt[i];
    int64_t total = offsets[n];
    free(cnt);
    if (total > cap) return total;
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        int64_t o = offsets[i];
        for (int64_t j = 0; j < n; ++j)
            if (is_neighbor(x, y, z, h, i, j, &b)) ids[o++] = (int32_t)j;
    }
    return total;
}

/* ------------------------------------------------- uniform-grid neighbours */

typedef struct {
    int64_t nc[3];        /* cells per axis */
    double inv_s[3];      /* 1 / cell side */
    int64_t *start;       /* first sorted slot of each linear cell */
    int64_t *order;       /* particle index of each sorted slot */
    int64_t ncell;
} orc_grid;

typedef struct { int64_t cell, idx; } cell_rec;

static int cmp_cell_rec(const void *a, const void *b)
{
    const cell_rec *p = (const cell_rec *)a, *q = (const cell_rec *)b;
    if (p->cell != q->cell) return p->cell < q->cell ? -1 : 1;
    return p->idx < q->idx ? -1 : (p->idx > q->idx);
}

static int64_t cell_coord(double v, double lo, double inv_s, int64_t nc)
{
    double f = floor((v - lo) * inv_s);
    if (f < 0.0) return 0;
    if (f > (double)(nc - 1)) return nc - 1;
    return (int64_t)f;
}

/* Cells of side >= reach * (1 + 1e-9); particles outside the box are
 * clamped into the border cells, which keeps every pair within reach in
 * adjacent cells. */
static void grid_build(orc_grid *g, int64_t n, const double *x, const double *y,
                       const double *z, const orc_box *b, double reach)
{
    const double *p[3] = {x, y, z};
    g->ncell = 1;
    for (int a = 0; a < 3; ++a) {
        double len = b->hi[a] - b->lo[a];
        double want = reach * (1.0 + 1e-9);
        int64_t nc = (int64_t)floor(len / want);
        if (nc < 1) nc = 1;
        if (nc > 1024) nc = 1024;
        g->nc[a] = nc;
        g->inv_s[a] = (double)nc / len;
        g->ncell *= nc;
    }
    cell_rec *rec = (cell_rec *)malloc(sizeof(cell_rec) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        for (int a = 0; a < 3; ++a)
            c[a] = cell_coord(p[a][i], b->lo[a], g->inv_s[a], g->nc[a]);
        rec[i].cell = (c[2] * g->nc[1] + c[1]) * g->nc[0] + c[0];
        rec[i].idx = i;
    }
    qsort(rec, (size_t)n, sizeof(cell_rec), cmp_cell_rec);
    g->start = (int64_t *)calloc((size_t)(g->ncell + 1), sizeof(int64_t));
    g->order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t s = 0; s < n; ++s) {
        g->order[s] = rec[s].idx;
        g->start[rec[s].cell + 1]++;
    }
    for (int64_t c = 0; c < g->ncell; ++c) g->start[c + 1] += g->start[c];
    free(rec);
}

static void grid_free(orc_grid *g)
{
    free(g->start);
    free(g->order);
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t p = *(const int32_t *)a, q = *(const int32_t *)b;
    return (p > q) - (p < q);
}

/* Distinct neighbouring cell coordinates of c along one axis. */
static int axis_cells(int64_t c, int64_t nc, int periodic, int64_t out[3])
{
    int k = 0;
    for (int64_t d = -1; d <= 1; ++d) {
        int64_t v = c + d;
        if (periodic) {
            v = ((v % nc) + nc) % nc;
        } else if (v < 0 || v >= nc) {
            continue;
        }
        int dup = 0;
        for (int t = 0; t < k; ++t) dup |= (out[t] == v);
        if (!dup) out[k++] = v;
    }
    return k;
}

/* All candidates j of particle i whose relation rel(i, j) holds, sorted
 * ascending; returns the count (writes at most cap entries to buf). */
typedef int (*relation_fn)(const double *, const double *, const double *,
                           const double *, int64_t, int64_t, const orc_box *);

static int64_t grid_query(const orc_grid *g, int64_t i, const double *x,
                          const double *y, const double *z, const double *h,
                          const orc_box *b, relation_fn rel, int32_t *buf,
                          int64_t cap)
{
    const double *p[3] = {x, y, z};
    int64_t c[3], nb[3][3];
    int k[3];
    for (int a = 0; a < 3; ++a) {
        c[a] = cell_coord(p[a][i], b->lo[a], g->inv_s[a], g->nc[a]);
        k[a] = axis_cells(c[a], g->nc[a], b->periodic[a], nb[a]);
    }
    int64_t cnt = 0;
    for (int iz = 0; iz < k[2]; ++iz)
        for (int iy = 0; iy < k[1]; ++iy)
            for (int ix = 0; ix < k[0]; ++ix) {
                int64_t cell = (nb[2][iz] * g->nc[1] + nb[1][iy]) * g->nc[0] + nb[0][ix];
                for (int64_t s = g->start[cell]; s < g->start[cell + 1]; ++s) {
                    int64_t j = g->order[s];
                    if (rel(x, y, z, h, i, j, b)) {
                        if (cnt < cap) buf[cnt] = (int32_t)j;
                        ++cnt;
                    }
                }
            }
    if (cnt <= cap) qsort(buf, (size_t)cnt, sizeof(int32_t), cmp_i32);
    return cnt;
}

static double max_of(const double *v, int64_t n)
{
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i) m = fmax(m, v[i]);
    return m;
}

/*
 * Neighbour sets by a plain uniform grid (cells of side >= 2 h_max, sorted
 * by linear cell index). Same contract as orc_neighbors_brute; each set is
 * sorted ascending. Returns -1 if one set exceeds 2^22 entries.
 */
int64_t orc_neighbors_grid(int64_t n, const double *x, const double *y,
                           const double *z, const double *h,
                           const double *lo, const double *hi,
                           const int32_t *per, int64_t cap,
                           int64_t *offsets, int32_t *ids)
{
    orc_box b = make_box(lo, hi, per);
    orc_grid g;
    offsets[0] = 0;
    if (n == 0) return 0;
    grid_build(&g, n, x, y, z, &b, 2.0 * max_of(h, n));
    int64_t *cnt = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    int64_t bufcap = n < ((int64_t)1 << 22) ? n : ((int64_t)1 << 22);
    #pragma omp parallel
    {
        int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)bufcap);
        #pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i)
            cnt[i] = grid_query(&g, i, x, y, z, h, &b, is_neighbor, buf, 0);
        free(buf);
    }
    for (int64_t i = 0; i < n; ++i) {
        if (cnt[i] > bufcap) { free(cnt); grid_free(&g); return -1; }
        offsets[i + 1] = offsets[i] + cnt[i];
    }
    int64_t total = offsets[n];
    free(cnt);
    if (total <= cap) {
        #pragma omp parallel
        {
            int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)bufcap);
            #pragma omp for schedule(dynamic, 256)
            for (int64_t i = 0; i < n; ++i) {
                int64_t c = grid_query(&g, i, x, y, z, h, &b, is_neighbor, buf, bufcap);
                memcpy(ids + offsets[i], buf, sizeof(int32_t) * (size_t)c);
            }
            free(buf);
        }
    }
    grid_free(&g);
    return total;
}

/*
 * Neighbour sets of the particles sel[0..k) only, by the same grid over all
 * n particles: offsets[q] .. offsets[q + 1] in ids holds particle sel[q]'s
 * set, ascending. Returns the total (ids written only if it fits cap), or -1
 * if one set exceeds 2^22 entries.
 */
int64_t orc_neighbors_subset(int64_t n, const double *x, const double *y,
                             const double *z, const double *h,
                             const double *lo, const double *hi,
                             const int32_t *per, int64_t k, const int64_t *sel,
                             int64_t cap, int64_t *offsets, int32_t *ids)
{
    orc_box b = make_box(lo, hi, per);
    orc_grid g;
    offsets[0] = 0;
    if (n == 0 || k == 0) {
        for (int64_t q = 0; q < k; ++q) offsets[q + 1] = 0;
        return 0;
    }
    grid_build(&g, n, x, y, z, &b, 2.0 * max_of(h, n));
    int64_t *cnt = (int64_t *)calloc((size_t)k, sizeof(int64_t));
    int64_t bufcap = n < ((int64_t)1 << 22) ? n : ((int64_t)1 << 22);
    #pragma omp parallel
    {
        int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)bufcap);
        #pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < k; ++q)
            cnt[q] = grid_query(&g, sel[q], x, y, z, h, &b, is_neighbor, buf, 0);
        free(buf);
    }
    for (int64_t q = 0; q < k; ++q) {
        if (cnt[q] > bufcap) { free(cnt); grid_free(&g); return -1; }
        offsets[q + 1] = offsets[q] + cnt[q];
    }
    int64_t total = offsets[k];
    free(cnt);
    if (total <= cap) {
        #pragma omp parallel
        {
            int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)bufcap);
            #pragma omp for schedule(dynamic, 16)
            for (int64_t q = 0; q < k; ++q) {
                int64_t c = grid_query(&g, sel[q], x, y, z, h, &b, is_neighbor, buf, bufcap);
                memcpy(ids + offsets[q], buf, sizeof(int32_t) * (size_t)c);
            }
            free(buf);
        }
    }
    grid_free(&g);
    return total;
}

/*
 * Cube root of a > 0 for the h update, by a rule both implementations
 * follow so that their h agree bit for bit (a library cbrt is not correctly
 * rounded and differs between libraries): Newton's iteration for y^3 = a,
 * y <- (2 y + a / y^2) / 3, seven steps from y = 3/2 after bringing a into
 * [1, 8) by exact factors of 8 (the start's relative error, at most 1/2,
 * squares at every step), then scaled back by the matching power of 2.
 * Only correctly rounded IEEE operations, no fused multiply-add.
 */
static double cbrt_newton(double a)
{
    int k = 0;
    while (a >= 8.0) { a *= 0.125; ++k; }
    while (a < 1.0) { a *= 8.0; --k; }
    double y = 1.5;
    for (int t = 0; t < 7; ++t) y = (2.0 * y + a / (y * y)) / 3.0;
    return ldexp(y, k);
}

/*
 * Smoothing-length iteration toward a target neighbour count (Algorithm 1
 * step 2 and its footnote: the code aims at a given number of neighbours and
 * h follows from it). Gather count N_i = |{j != i : r^2 < 4 h_i^2}|; every
 * particle outside [lo_count, hi_count] is updated with
 * h <- h * (1 + (n_target / N_i)^(1/3)) / 2 (h doubles when N_i = 0; the
 * cube root by cbrt_newton); at most max_iter sweeps. Returns the index of
 * the last sweep.
 */
int32_t orc_smoothing_length(int64_t n, const double *x, const double *y,
                             const double *z, double *h,
                             const double *lo, const double *hi,
                             const int32_t *per, double n_target,
                             int32_t lo_count, int32_t hi_count,
                             int32_t max_iter, int32_t *count_out)
{
    orc_box b = make_box(lo, hi, per);
    int32_t it;
    int32_t *cnt = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (it = 0; it <= max_iter; ++it) {
        orc_grid g;
        grid_build(&g, n, x, y, z, &b, 2.0 * max_of(h, n));
        #pragma omp parallel for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i)
            cnt[i] = (int32_t)grid_query(&g, i, x, y, z, h, &b, in_gather_sphere, NULL, 0);
        grid_free(&g);
        int64_t bad = 0;
        for (int64_t i = 0; i < n; ++i) bad += (cnt[i] < lo_count || cnt[i] > hi_count);
        if (bad == 0 || it == max_iter) break;
        #pragma omp parallel for
        for (int64_t i = 0; i < n; ++i) {
            if (cnt[i] >= lo_count && cnt[i] <= hi_count) continue;
            if (cnt[i] == 0) h[i] = 2.0 * h[i];
            else h[i] = h[i] * 0.5 * (1.0 + cbrt_newton(n_target / (double)cnt[i]));
        }
    }
    if (count_out) memcpy(count_out, cnt, sizeof(int32_t) * (size_t)n);
    free(cnt);
    return it;
}

/* ------------------------------------------------------------- density */

/* rho_i = m_i W(0, h_i) + sum_{j in N_i} m_j W(r_ij, h_i), over the set
 * nb[0..len) of particle i (ascending). */
static double density_of(int64_t i, const double *x, const double *y, const double *z,
                         const double *h, const double *m, const orc_box *b,
                         const int32_t *nb, int64_t len)
{
    double s = m[i] * orc_kernel_w(0.0, h[i]);
    for (int64_t k = 0; k < len; ++k) {
        int64_t j = nb[k];
        double dx, dy, dz;
        separation(x, y, z, i, j, b, &dx, &dy, &dz);
        double r = sqrt(dist2(dx, dy, dz));
        s += m[j] * orc_kernel_w(r, h[i]);
    }
    return s;
}

void orc_density(int64_t n, const double *x, const double *y, const double *z,
                 const double *h, const double *m,
                 const double *lo, const double *hi, const int32_t *per,
                 const int64_t *offsets, const int32_t *ids, double *rho)
{
    orc_box b = make_box(lo, hi, per);
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i)
        rho[i] = density_of(i, x, y, z, h, m, &b, ids + offsets[i], offsets[i + 1] - offsets[i]);
}

/* The same for the particles sel[0..k) only (their sets in CSR by q, as
 * orc_neighbors_subset gives them); rho[q] is particle sel[q]'s. */
void orc_density_subset(int64_t n, const double *x, const double *y, const double *z,
                        const double *h, const double *m,
                        const double *lo, const double *hi, const int32_t *per,
                        int64_t k, const int64_t *sel, const int64_t *offsets,
                        const int32_t *ids, double *rho)
{
    (void)n;
    orc_box b = make_box(lo, hi, per);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < k; ++q)
        rho[q] = density_of(sel[q], x, y, z, h, m, &b, ids + offsets[q],
                            offsets[q + 1] - offsets[q]);
}

/* ------------------------------------------ generalised volume elements */

/*
 * Generalised volume elements (Table 1, SPHYNX; Cabezon, Garcia-Senz &
 * Figueira 2017, in the general form of Hopkins 2013). With weights X_j:
 *   k_i   = X_i W(0, h_i) + sum_{j in N_i} X_j W(r_ij, h_i),
 *   V_i   = X_i / k_i,   rho_i = m_i / V_i = k_i (m_i / X_i),
 * and X_i = (m_i / rho~_i)^p from a previous density estimate rho~. X = m
 * gives the standard elements (m_i / X_i = 1 exactly).
 */
void orc_volume_weights(int64_t n, const double *m, const double *rho_prev, double p,
                        double *X)
{
    for (int64_t i = 0; i < n; ++i) X[i] = pow(m[i] / rho_prev[i], p);
}

void orc_density_weighted(int64_t n, const double *x, const double *y, const double *z,
                          const double *h, const double *m, const double *X,
                          const double *lo, const double *hi, const int32_t *per,
                          const int64_t *offsets, const int32_t *ids, double *rho)
{
    orc_box b = make_box(lo, hi, per);
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double k = X[i] * orc_kernel_w(0.0, h[i]);
        for (int64_t q = offsets[i]; q < offsets[i + 1]; ++q) {
            int64_t j = ids[q];
            double dx, dy, dz;
            separation(x, y, z, i, j, &b, &dx, &dy, &dz);
            double r = sqrt(dist2(dx, dy, dz));
            k += X[j] * orc_kernel_w(r, h[i]);
        }
        rho[i] = k * (m[i] / X[i]);
    }
}

/* ------------------------------------------------------------------ EOS */

/*
 * eos = 0, Tait: x = rho/rho_ref, P = p_bg + B (x^7 - 1), c = c0 x^3 with
 *       B = rho0 c0^2 / gamma_tait (gamma_tait = 7 assumed by the powers).
 * eos = 1, ideal gas: P = (gamma - 1) rho u, c = sqrt(gamma (gamma - 1) u).
 * Also pr2 = P / rho^2.
 */
void orc_eos(int64_t n, int32_t eos, double rho0, double c0, double gamma_tait,
             double gamma_gas, const double *rho, const double *u,
             const double *rho_ref, const double *p_bg,
             double *p, double *c, double *pr2)
{
    #pragma omp parallel for
    for (int64_t i = 0; i < n; ++i) {
        double P, C;
        if (eos == 0) {
            double B = rho0 * c0 * c0 / gamma_tait;
            double xr = rho[i] / rho_ref[i];
            double x2 = xr * xr, x4 = x2 * x2, x6 = x4 * x2, x7 = x6 * xr;
            double x3 = x2 * xr;
            P = p_bg[i] + B * (x7 - 1.0);
            C = c0 * x3;
        } else {
            P = (gamma_gas - 1.0) * rho[i] * u[i];
            C = sqrt(gamma_gas * (gamma_gas - 1.0) * u[i]);
        }
        p[i] = P;
        c[i] = C;
        pr2[i] = P / (rho[i] * rho[i]);
    }
}

/* ------------------------------------------------------------------ IAD */

/*
 * Integral approach to derivatives (Garcia-Senz, Cabezon & Escartin 2012),
 * with standard volume elements V_j = m_j / rho_j:
 *   tau_i = sum_{j in N_i} V_j (x_j - x_i)(x_j - x_i)^T W(r_ij, h_i),
 *   c_i   = tau_i^{-1}  when det tau_i >= k_c (tr tau_i / 3)^3,
 * with k_c = 1e-2 (a reading: the paper gives no rule for the degenerate
 * case). For a symmetric positive semi-definite tau the ratio
 * det / (tr / 3)^3 lies in [0, 1] (the arithmetic-geometric mean inequality
 * on the eigenvalues), equals 1 for an isotropic neighbourhood and tends to
 * 0 when the neighbours no longer span three dimensions; there the inverse
 * is set by rounding alone. Below the threshold c_i takes the isotropic form
 * (tr tau_i / 3)^{-1} I, which the full inverse also reduces to for an
 * isotropic tau; c_i = 0 when tr tau_i = 0 (no neighbour inside 2 h_i).
 *   A_ij  = c_i (x_j - x_i) W(r_ij, h_i),
 * so that sum_j V_j (f_j - f_i) A_ij is exact for linear f. A_ij takes the
 * place of grad_i W_ij; the pair forces use the antisymmetric mean
 * Abar_ij = (A_ij - A_ji) / 2 = -(W(r, h_i) c_i + W(r, h_j) c_j) r_ij / 2.
 * c6 holds c_i as xx, xy, xz, yy, yz, zz (6 doubles per particle).
 */
static int32_t g_gradient = 0;   /* 0 kernel derivatives, 1 IAD */
#define ORC_IAD_COND 1e-2        /* k_c of the conditioning rule above */

int32_t orc_set_gradient(int32_t mode)
{
    if (mode != 0 && mode != 1) return -1;
    g_gradient = mode;
    return 0;
}

void orc_iad_matrices(int64_t n, const double *x, const double *y, const double *z,
                      const double *h, const double *m, const double *rho,
                      const double *lo, const double *hi, const int32_t *per,
                      const int64_t *offsets, const int32_t *ids, double *c6)
{
    orc_box b = make_box(lo, hi, per);
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double a = 0.0, bb = 0.0, c = 0.0, d = 0.0, e = 0.0, f = 0.0;
        for (int64_t k = offsets[i]; k < offsets[i + 1]; ++k) {
            int64_t j = ids[k];
            double dx, dy, dz;
            separation(x, y, z, i, j, &b, &dx, &dy, &dz);  /* x_i - x_j */
            double r = sqrt(dist2(dx, dy, dz));
            double vw = m[j] / rho[j] * orc_kernel_w(r, h[i]);
            a += vw * dx * dx;
            bb += vw * dx * dy;
            c += vw * dx * dz;
            d += vw * dy * dy;
            e += vw * dy * dz;
            f += vw * dz * dz;
        }
        double cof_a = d * f - e * e, cof_b = c * e - bb * f, cof_c = bb * e - c * d;
        double det = a * cof_a + bb * cof_b + c * cof_c;
        double tr = a + d + f;
        double *o = c6 + 6 * i;
        for (int t = 0; t < 6; ++t) o[t] = 0.0;
        if (!(tr > 0.0) || !isfinite(tr) || !isfinite(det))
            continue;                       /* no neighbour inside 2 h_i */
        double tm = tr / 3.0;
        if (!(det >= ORC_IAD_COND * (tm * tm * tm))) {
            o[0] = o[3] = o[5] = 3.0 / tr;  /* isotropic form */
            continue;
        }
        o[0] = cof_a / det;
        o[1] = cof_b / det;
        o[2] = cof_c / det;
        o[3] = (a * f - c * c) / det;
        o[4] = (bb * c - a * e) / det;
        o[5] = (a * d - bb * bb) / det;
    }
}

/* ------------------------------------------------- momentum and energy */

/*
 * Without weights (standard volume elements), for each j in N_i (ascending):
 *   gradW = 1/2 [dW/dr(r, h_i) + dW/dr(r, h_j)] r_ij / r  (zero when r = 0)
 *   mu    = hbar (v_ij . r_ij) / (r^2 + eta2 hbar^2) if v_ij . r_ij < 0 else 0
 *   Pi    = (-alpha cbar mu + beta mu^2) / rhobar
 *   G     = pr2_i + pr2_j + Pi
 *   a_i  -= m_j G gradW ;  du_i += 1/2 m_j G v_ij . gradW ; mumax_i = max |mu|
 * Also the error scales S^a_i = sum m_j |G| |gradW| and
 * S^u_i = 1/2 sum m_j |G| |v_ij| |gradW| (either output may be NULL).
 *
 * With generalised volume elements of weights X, the pair weight m_j G
 * becomes (the same form with X = m)
 *   F_ij = (X_j Q_i + X_i Q_j) / m_i + m_j Pi_ij,  Q_i = m_i^2 pr2_i / X_i,
 * from m_i a_i = -sum_j X_i X_j (P_i / k_i^2 + P_j / k_j^2) gradW_ij with
 * k = rho X / m; F_ij m_i is symmetric in i and j, so momentum and energy
 * stay conserved. IAD keeps V_j = m_j / rho_j, which equals X_j / k_j.
 */
/* The pair sums of particle i over its set nb[0..len) (ascending), into
 * out = {a_x, a_y, a_z, du/dt, max |mu|, S^a, S^u}; c6 (IAD matrices) and X
 * (weights) may be NULL. */
static void momentum_of(int64_t i, const int32_t *nb, int64_t len, const double *x,
                        const double *y, const double *z, const double *vx,
                        const double *vy, const double *vz, const double *h,
                        const double *m, const double *X, const double *rho,
                        const double *c, const double *pr2, const orc_box *b,
                        const double *c6, double alpha, double beta, double eta2,
                        double out[7])
{
    double axi = 0.0, ayi = 0.0, azi = 0.0, dui = 0.0, mum = 0.0;
    double sai = 0.0, sui = 0.0;
    for (int64_t k = 0; k < len; ++k) {
        int64_t j = nb[k];
        double dx, dy, dz;
        separation(x, y, z, i, j, b, &dx, &dy, &dz);
        double r2 = dist2(dx, dy, dz);
        double r = sqrt(r2);
        double gx = 0.0, gy = 0.0, gz = 0.0;
        if (c6) {
            const double *ci = c6 + 6 * i, *cj = c6 + 6 * j;
            double wi = orc_kernel_w(r, h[i]), wj = orc_kernel_w(r, h[j]);
            gx = -0.5 * (wi * (ci[0] * dx + ci[1] * dy + ci[2] * dz) +
                         wj * (cj[0] * dx + cj[1] * dy + cj[2] * dz));
            gy = -0.5 * (wi * (ci[1] * dx + ci[3] * dy + ci[4] * dz) +
                         wj * (cj[1] * dx + cj[3] * dy + cj[4] * dz));
            gz = -0.5 * (wi * (ci[2] * dx + ci[4] * dy + ci[5] * dz) +
                         wj * (cj[2] * dx + cj[4] * dy + cj[5] * dz));
        } else if (r > 0.0) {
            double dwbar = 0.5 * (orc_kernel_dwdr(r, h[i]) + orc_kernel_dwdr(r, h[j]));
            gx = dwbar * dx / r;
            gy = dwbar * dy / r;
            gz = dwbar * dz / r;
        }
        double wx = vx[i] - vx[j], wy = vy[i] - vy[j], wz = vz[i] - vz[j];
        double vdotr = wx * dx + wy * dy + wz * dz;
        double hbar = 0.5 * (h[i] + h[j]);
        double cbar = 0.5 * (c[i] + c[j]);
        double rhobar = 0.5 * (rho[i] + rho[j]);
        double mu = 0.0;
        if (vdotr < 0.0) mu = hbar * vdotr / (r2 + eta2 * hbar * hbar);
        double Pi = (-alpha * cbar * mu + beta * mu * mu) / rhobar;
        double G = pr2[i] + pr2[j] + Pi;
        double F = m[j] * G;
        if (X) {
            double Qi = m[i] * m[i] * pr2[i] / X[i], Qj = m[j] * m[j] * pr2[j] / X[j];
            F = (X[j] * Qi + X[i] * Qj) / m[i] + m[j] * Pi;
        }
        axi -= F * gx;
        ayi -= F * gy;
        azi -= F * gz;
        dui += 0.5 * F * (wx * gx + wy * gy + wz * gz);
        if (fabs(mu) > mum) mum = fabs(mu);
        double gn = sqrt(gx * gx + gy * gy + gz * gz);
        sai += fabs(F) * gn;
        sui += 0.5 * fabs(F) * sqrt(wx * wx + wy * wy + wz * wz) * gn;
    }
    out[0] = axi; out[1] = ayi; out[2] = azi; out[3] = dui;
    out[4] = mum; out[5] = sai; out[6] = sui;
}

static void momentum_energy_impl(int64_t n, const double *x, const double *y,
                                 const double *z, const double *vx, const double *vy,
                                 const double *vz, const double *h, const double *m,
                                 const double *X, const double *rho, const double *c,
                                 const double *pr2, const double *lo, const double *hi,
                                 const int32_t *per, const int64_t *offsets,
                                 const int32_t *ids, double alpha, double beta, double eta2,
                                 double *ax, double *ay, double *az, double *dudt,
                                 double *mumax, double *sa, double *su)
{
    orc_box b = make_box(lo, hi, per);
    double *c6 = NULL;
    if (g_gradient == 1) {
        c6 = (double *)malloc(sizeof(double) * 6 * (size_t)(n > 0 ? n : 1));
        orc_iad_matrices(n, x, y, z, h, m, rho, lo, hi, per, offsets, ids, c6);
    }
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double o[7];
        momentum_of(i, ids + offsets[i], offsets[i + 1] - offsets[i], x, y, z, vx, vy, vz,
                    h, m, X, rho, c, pr2, &b, c6, alpha, beta, eta2, o);
        ax[i] = o[0]; ay[i] = o[1]; az[i] = o[2]; dudt[i] = o[3];
        if (mumax) mumax[i] = o[4];
        if (sa) sa[i] = o[5];
        if (su) su[i] = o[6];
    }
    free(c6);
}

/* Momentum and energy (kernel derivatives, standard volume elements) for
 * the particles sel[0..k) only, with their sets in CSR by q (as
 * orc_neighbors_subset gives them); every other array covers all n
 * particles. Outputs are indexed by q; mumax, sa, su may be NULL. Returns -1
 * (and computes nothing) when IAD gradients are selected. */
int32_t orc_momentum_energy_subset(int64_t n, const double *x, const double *y,
                                   const double *z, const double *vx, const double *vy,
                                   const double *vz, const double *h, const double *m,
                                   const double *rho, const double *c, const double *pr2,
                                   const double *lo, const double *hi, const int32_t *per,
                                   int64_t k, const int64_t *sel, const int64_t *offsets,
                                   const int32_t *ids, double alpha, double beta,
                                   double eta2, double *ax, double *ay, double *az,
                                   double *dudt, double *mumax, double *sa, double *su)
{
    (void)n;
    if (g_gradient != 0) return -1;
    orc_box b = make_box(lo, hi, per);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < k; ++q) {
        double o[7];
        momentum_of(sel[q], ids + offsets[q], offsets[q + 1] - offsets[q], x, y, z, vx, vy,
                    vz, h, m, NULL, rho, c, pr2, &b, NULL, alpha, beta, eta2, o);
        ax[q] = o[0]; ay[q] = o[1]; az[q] = o[2]; dudt[q] = o[3];
        if (mumax) mumax[q] = o[4];
        if (sa) sa[q] = o[5];
        if (su) su[q] = o[6];
    }
    return 0;
}

void orc_momentum_energy(int64_t n, const double *x, const double *y,
                         const double *z, const double *vx, const double *vy,
                         const double *vz, const double *h, const double *m,
                         const double *rho, const double *c, const double *pr2,
                         const double *lo, const double *hi, const int32_t *per,
                         const int64_t *offsets, const int32_t *ids,
                         double alpha, double beta, double eta2,
                         double *ax, double *ay, double *az, double *dudt,
                         double *mumax, double *sa, double *su)
{
    momentum_energy_impl(n, x, y, z, vx, vy, vz, h, m, NULL, rho, c, pr2, lo, hi, per,
                         offsets, ids, alpha, beta, eta2, ax, ay, az, dudt, mumax, sa, su);
}

void orc_momentum_energy_weighted(int64_t n, const double *x, const double *y,
                                  const double *z, const double *vx, const double *vy,
                                  const double *vz, const double *h, const double *m,
                                  const double *X, const double *rho, const double *c,
                                  const double *pr2, const double *lo, const double *hi,
                                  const int32_t *per, const int64_t *offsets,
                                  const int32_t *ids, double alpha, double beta,
                                  double eta2, double *ax, double *ay, double *az,
                                  double *dudt, double *mumax, double *sa, double *su)
{
    momentum_energy_impl(n, x, y, z, vx, vy, vz, h, m, X, rho, c, pr2, lo, hi, per, offsets,
                         ids, alpha, beta, eta2, ax, ay, az, dudt, mumax, sa, su);
}

/* ------------------------------------------------------------ time-step */

/*
 * Global dt = min_i min( c_cfl h_i / (c_i + 1.2 (alpha c_i + beta mumax_i)),
 *                        c_force sqrt(h_i / |a_i + g_i|) ),
 * the force limit skipped where |a + g| = 0 (Monaghan 1989). g may be NULL.
 */
double orc_timestep(int64_t n, const double *h, const double *c,
                    const double *mumax, const double *ax, const double *ay,
                    const double *az, const double *gx, const double *gy,
                    const double *gz, double alpha, double beta, double c_cfl,
                    double c_force)
{
    double dt = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        double d = c_cfl * h[i] / (c[i] + 1.2 * (alpha * c[i] + beta * mumax[i]));
        double tx = ax[i], ty = ay[i], tz = az[i];
        if (gx) { tx += gx[i]; ty += gy[i]; tz += gz[i]; }
        double amag = sqrt(tx * tx + ty * ty + tz * tz);
        if (amag > 0.0) d = fmin(d, c_force * sqrt(h[i] / amag));
        dt = fmin(dt, d);
    }
    return dt;
}

/* The same criterion per particle (individual time steps): dtc[i] is the
 * smaller of the Courant and force limits of particle i. */
void orc_timestep_each(int64_t n, const double *h, const double *c, const double *mumax,
                       const double *ax, const double *ay, const double *az,
                       const double *gx, const double *gy, const double *gz, double alpha,
                       double beta, double c_cfl, double c_force, double *dtc)
{
    for (int64_t i = 0; i < n; ++i) {
        double d = c_cfl * h[i] / (c[i] + 1.2 * (alpha * c[i] + beta * mumax[i]));
        double tx = ax[i], ty = ay[i], tz = az[i];
        if (gx) { tx += gx[i]; ty += gy[i]; tz += gz[i]; }
        double amag = sqrt(tx * tx + ty * ty + tz * tz);
        if (amag > 0.0) d = fmin(d, c_force * sqrt(h[i] / amag));
        dtc[i] = d;
    }
}

/* ---------------------------------------------------------- integration */

/*
 * Kick-drift-kick leapfrog with a global dt.
 * stage 0 (kick + drift): v += dt/2 (a + g); u += dt/2 du; x += dt v; each
 *         periodic coordinate is wrapped back into [lo, hi).
 * stage 1 (kick):         v += dt/2 (a + g); u += dt/2 du.
 * g may be NULL.
 */
void orc_integrate(int64_t n, int32_t stage, double dt, double *x, double *y,
                   double *z, double *vx, double *vy, double *vz, double *u,
                   const double *ax, const double *ay, const double *az,
                   const double *dudt, const double *gx, const double *gy,
                   const double *gz, const double *lo, const double *hi,
                   const int32_t *per)
{
    double half = 0.5 * dt;
    double *p[3] = {x, y, z};
    #pragma omp parallel for
    for (int64_t i = 0; i < n; ++i) {
        double tx = ax[i], ty = ay[i], tz = az[i];
        if (gx) { tx += gx[i]; ty += gy[i]; tz += gz[i]; }
        vx[i] += half * tx;
        vy[i] += half * ty;
        vz[i] += half * tz;
        u[i] += half * dudt[i];
        if (stage == 0) {
            x[i] += dt * vx[i];
            y[i] += dt * vy[i];
            z[i] += dt * vz[i];
            for (int a = 0; a < 3; ++a) {
                if (!per[a]) continue;
                double len = hi[a] - lo[a];
                if (p[a][i] >= hi[a]) p[a][i] -= len;
                else if (p[a][i] < lo[a]) p[a][i] += len;
            }
        }
    }
}

/* ---------------------------------------------------------- diagnostics */

/* Neumaier-compensated running sum. */
typedef struct { double s, c; } nsum;

static void nsum_add(nsum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}

/*
 * out[8] = M, Px, Py, Pz, Lx, Ly, Lz, E with P = sum m v, L = sum m x cross v,
 * E = sum m (v^2/2 + u).
 */
void orc_diagnostics(int64_t n, const double *x, const double *y,
                     const double *z, const double *vx, const double *vy,
                     const double *vz, const double *u, const double *m,
                     double *out)
{
    nsum acc[8];
    memset(acc, 0, sizeof(acc));
    for (int64_t i = 0; i < n; ++i) {
        double mi = m[i];
        nsum_add(&acc[0], mi);
        nsum_add(&acc[1], mi * vx[i]);
        nsum_add(&acc[2], mi * vy[i]);
        nsum_add(&acc[3], mi * vz[i]);
        nsum_add(&acc[4], mi * (y[i] * vz[i] - z[i] * vy[i]));
        nsum_add(&acc[5], mi * (z[i] * vx[i] - x[i] * vz[i]));
        nsum_add(&acc[6], mi * (x[i] * vy[i] - y[i] * vx[i]));
        nsum_add(&acc[7], mi * (0.5 * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]) + u[i]));
    }
    for (int k = 0; k < 8; ++k) out[k] = acc[k].s + acc[k].c;
}

/* -------------------------------------------------------- self-gravity */

/* Plummer-softened direct sum, G = 1: g_i = -sum_{j != i} m_j r_ij /
 * (r^2 + eps^2)^{3/2}. Supplies the fixed external field of the Evrard
 * inputs; it is not part of the hydro step. */
void orc_gravity_direct(int64_t n, const double *x, const double *y,
                        const double *z, const double *m, double eps,
                        double *gx, double *gy, double *gz)
{
    double e2 = eps * eps;
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double sx = 0.0, sy = 0.0, sz = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            double d2 = dx * dx + dy * dy + dz * dz + e2;
            double inv = 1.0 / (d2 * sqrt(d2));
            sx -= m[j] * dx * inv;
            sy -= m[j] * dy * inv;
            sz -= m[j] * dz * inv;
        }
        gx[i] = sx; gy[i] = sy; gz[i] = sz;
    }
}

/*
 * The same direct sum for the particles listed in sel only (nsel of them),
 * plus its error scale sg_k = sum_{j != i} m_j |x_i - x_j| / (r^2 + eps^2)^{3/2}
 * (sg may be NULL). Every j in index order, as orc_gravity_direct.
 */
void orc_gravity_direct_subset(int64_t n, const double *x, const double *y,
                               const double *z, const double *m, double eps,
                               int64_t nsel, const int64_t *sel, double *gx,
                               double *gy, double *gz, double *sg)
{
    double e2 = eps * eps;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < nsel; ++k) {
        int64_t i = sel[k];
        double sx = 0.0, sy = 0.0, sz = 0.0, ss = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            double d2 = dx * dx + dy * dy + dz * dz + e2;
            double inv = 1.0 / (d2 * sqrt(d2));
            sx -= m[j] * dx * inv;
            sy -= m[j] * dy * inv;
            sz -= m[j] * dz * inv;
            ss += m[j] * sqrt(dx * dx + dy * dy + dz * dz) * inv;
        }
        gx[k] = sx; gy[k] = sy; gz[k] = sz;
        if (sg) sg[k] = ss;
    }
}

/* ----------------------------------------------------------- threading */

int32_t orc_num_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int32_t t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* ------------------------------------------------- tree self-gravity */

/*
 * Self-gravity by a Morton octree with multipoles to quadrupole order (the
 * parent codes' approach, Alg. 1 step 4, Sec. 5.2.5 phase I; SPHYNX keeps
 * quadrupoles). G = 1. The tree, the moments and the acceptance test are
 * fixed here so that they are reproducible:
 *
 *   cube   lo_a = min_i x_a, L = max_a (max_i x_a - lo_a) (1 if zero);
 *   keys   k_a = min(1023, floor((x_a - lo_a) / L * 1024)), interleaved as
 *          Morton code k_x | k_y << 1 | k_z << 2 per bit (30 bits);
 *   order  particles sorted by (key, index);
 *   nodes  the root holds all particles; a node of level l < 10 with more
 *          than leaf_size particles gets one child per non-empty octant
 *          (next three key bits), in octant order; the others are leaves.
 *          Node side s = L / 2^l, geometric centre lo + (k + 1/2) s;
 *   moments M = sum m, centre of mass c, traceless quadrupole
 *          Q_ab = sum m (3 d_a d_b - |d|^2 delta_ab), d = x - c; a leaf sums
 *          its particles in sorted order, an internal node its children in
 *          octant order with the parallel-axis shift
 *          Q += Q_k + M_k (3 e_a e_b - |e|^2 delta_ab), e = c_k - c;
 *   groups the root if it holds at most 64 particles; else, for every node
 *          with more than 64 particles, its children with at most 64 taken
 *          in octant order and merged while the merged run holds at most 64
 *          (a child with more than 64 ends a run), and a leaf with more than
 *          64 (finest level only) cut into runs of 64. Each group is a run of
 *          the sorted order within one node of more than 64 particles, so
 *          its box stays compact. A node N is accepted for every particle of a group
 *          G when dist(c_N, box_G) > s_N / theta + |c_N - centre_N|, box_G
 *          the bounding box of G's particles; otherwise a leaf N is summed
 *          directly and an internal N is opened (its children are visited
 *          next). Visiting is breadth-first from the root, children in
 *          octant order;
 *   terms  direct: -m_j d / (|d|^2 + eps^2)^{3/2}, d = x_i - x_j, j != i;
 *          node: -M d / r^3 + Q d / r^5 - 5/2 (d.Q d) d / r^7, d = x_i - c
 *          (unsoftened), the gradient of the expansion of the potential
 *          -M/r - d.Q d / (2 r^5).
 * scale (optional): per particle, the sum of the magnitudes of the terms.
 * stats (optional): [nodes, leaves, node terms, direct terms, largest frontier,
 * groups].
 * group_work (optional): per group, accepted nodes plus directly summed
 * particles.
 */
#define ORC_GROUP 64
typedef struct {
    int64_t start, end, child0;
    int32_t level, nchild;
    uint32_t prefix;
    double M, c[3], Q[6], blo[3], bhi[3], s, delta;
} orc_gnode;

static uint32_t spread10(uint32_t v)
{
    uint32_t r = 0;
    for (int b = 0; b < 10; ++b) r |= ((v >> b) & 1u) << (3 * b);
    return r;
}

typedef struct { uint32_t key; int64_t idx; } orc_kidx;

static int kidx_cmp(const void *a, const void *b)
{
    const orc_kidx *p = (const orc_kidx *)a, *q = (const orc_kidx *)b;
    if (p->key != q->key) return p->key < q->key ? -1 : 1;
    return p->idx < q->idx ? -1 : (p->idx > q->idx);
}

/* first position in [lo, hi) of the sorted keys with key >= k */
static int64_t lower_key(const orc_kidx *s, int64_t lo, int64_t hi, uint32_t k)
{
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (s[mid].key < k) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* The tree of the definition above: sorted particles, nodes (breadth-first,
 * children contiguous) with their moments. The caller frees both. */
static orc_gnode *gtree_build(int64_t n, const double **P, const double *m,
                              int32_t leaf_size, orc_kidx **srt_out, int64_t *nn_out)
{
    double lo[3], L = 0.0;
    for (int a = 0; a < 3; ++a) {
        double mn = P[a][0], mx = P[a][0];
        for (int64_t i = 1; i < n; ++i) {
            if (P[a][i] < mn) mn = P[a][i];
            if (P[a][i] > mx) mx = P[a][i];
        }
        lo[a] = mn;
        if (mx - mn > L) L = mx - mn;
    }
    if (!(L > 0.0)) L = 1.0;
    orc_kidx *srt = (orc_kidx *)malloc(sizeof(orc_kidx) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        uint32_t k[3];
        for (int a = 0; a < 3; ++a) {
            double q = floor((P[a][i] - lo[a]) / L * 1024.0);
            k[a] = q >= 1023.0 ? 1023u : (uint32_t)q;
        }
        srt[i].key = spread10(k[0]) | (spread10(k[1]) << 1) | (spread10(k[2]) << 2);
        srt[i].idx = i;
    }
    qsort(srt, (size_t)n, sizeof(orc_kidx), kidx_cmp);

    /* nodes, breadth-first */
    int64_t cap = 1024, nn = 1;
    orc_gnode *T = (orc_gnode *)calloc((size_t)cap, sizeof(orc_gnode));
    T[0].start = 0; T[0].end = n; T[0].level = 0; T[0].prefix = 0;
    for (int64_t t = 0; t < nn; ++t) {
        T[t].child0 = -1; T[t].nchild = 0;
        if (T[t].level >= 10 || T[t].end - T[t].start <= leaf_size) continue;
        int shift = 3 * (9 - T[t].level);
        int64_t first = nn;
        for (uint32_t o = 0; o < 8; ++o) {
            uint32_t pre = (T[t].prefix << 3) | o;
            int64_t a = lower_key(srt, T[t].start, T[t].end, pre << shift);
            int64_t b = lower_key(srt, T[t].start, T[t].end, (pre + 1) << shift);
            if (a == b) continue;
            if (nn == cap) {
                cap *= 2;
                T = (orc_gnode *)realloc(T, sizeof(orc_gnode) * (size_t)cap);
            }
            memset(&T[nn], 0, sizeof(orc_gnode));
            T[nn].start = a; T[nn].end = b; T[nn].level = T[t].level + 1; T[nn].prefix = pre;
            ++nn;
        }
        T[t].child0 = first;
        T[t].nchild = (int32_t)(nn - first);
    }

    /* moments, children before parents */
    for (int64_t t = nn - 1; t >= 0; --t) {
        orc_gnode *N = &T[t];
        double M = 0.0, sc[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < 6; ++q) N->Q[q] = 0.0;
        if (N->nchild == 0) {
            for (int a = 0; a < 3; ++a) { N->blo[a] = INFINITY; N->bhi[a] = -INFINITY; }
            for (int64_t k = N->start; k < N->end; ++k) {
                int64_t j = srt[k].idx;
                M += m[j];
                for (int a = 0; a < 3; ++a) {
                    sc[a] += m[j] * P[a][j];
                    if (P[a][j] < N->blo[a]) N->blo[a] = P[a][j];
                    if (P[a][j] > N->bhi[a]) N->bhi[a] = P[a][j];
                }
            }
            for (int a = 0; a < 3; ++a) N->c[a] = sc[a] / M;
            for (int64_t k = N->start; k < N->end; ++k) {
                int64_t j = srt[k].idx;
                double d[3] = {P[0][j] - N->c[0], P[1][j] - N->c[1], P[2][j] - N->c[2]};
                double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                N->Q[0] += m[j] * (3.0 * d[0] * d[0] - d2);
                N->Q[1] += m[j] * (3.0 * d[0] * d[1]);
                N->Q[2] += m[j] * (3.0 * d[0] * d[2]);
                N->Q[3] += m[j] * (3.0 * d[1] * d[1] - d2);
                N->Q[4] += m[j] * (3.0 * d[1] * d[2]);
                N->Q[5] += m[j] * (3.0 * d[2] * d[2] - d2);
            }
        } else {
            for (int a = 0; a < 3; ++a) { N->blo[a] = INFINITY; N->bhi[a] = -INFINITY; }
            for (int64_t k = N->child0; k < N->child0 + N->nchild; ++k) {
                M += T[k].M;
                for (int a = 0; a < 3; ++a) {
                    sc[a] += T[k].M * T[k].c[a];
                    if (T[k].blo[a] < N->blo[a]) N->blo[a] = T[k].blo[a];
                    if (T[k].bhi[a] > N->bhi[a]) N->bhi[a] = T[k].bhi[a];
                }
            }
            for (int a = 0; a < 3; ++a) N->c[a] = sc[a] / M;
            for (int64_t k = N->child0; k < N->child0 + N->nchild; ++k) {
                double e[3] = {T[k].c[0] - N->c[0], T[k].c[1] - N->c[1], T[k].c[2] - N->c[2]};
                double e2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
                double Mk = T[k].M;
                N->Q[0] += T[k].Q[0] + Mk * (3.0 * e[0] * e[0] - e2);
                N->Q[1] += T[k].Q[1] + Mk * (3.0 * e[0] * e[1]);
                N->Q[2] += T[k].Q[2] + Mk * (3.0 * e[0] * e[2]);
                N->Q[3] += T[k].Q[3] + Mk * (3.0 * e[1] * e[1] - e2);
                N->Q[4] += T[k].Q[4] + Mk * (3.0 * e[1] * e[2]);
                N->Q[5] += T[k].Q[5] + Mk * (3.0 * e[2] * e[2] - e2);
            }
        }
        N->M = M;
        N->s = L / (double)(1u << N->level);
        uint32_t kk[3] = {0, 0, 0};
        for (int b = 0; b < N->level; ++b)
            for (int a = 0; a < 3; ++a)
                kk[a] |= ((N->prefix >> (3 * b + a)) & 1u) << b;
        double dd = 0.0;
        for (int a = 0; a < 3; ++a) {
            double centre = lo[a] + ((double)kk[a] + 0.5) * N->s;
            double e = N->c[a] - centre;
            dd += e * e;
        }
        N->delta = sqrt(dd);
    }
    *srt_out = srt;
    *nn_out = nn;
    return T;
}

/* The groups of the definition above, as runs [gs[q], ge[q]) of the sorted
 * order (room for 8 nn + n / 64 + 2 entries); returns their number. */
static int64_t gtree_groups(const orc_gnode *T, int64_t nn, int64_t n, int64_t *gs,
                            int64_t *ge)
{
    int64_t n_group = 0;
    if (n <= ORC_GROUP) {
        gs[0] = 0;
        ge[0] = n;
        n_group = 1;
    }
    for (int64_t t = 0; t < nn; ++t) {
        if (T[t].end - T[t].start <= ORC_GROUP) continue;
        if (T[t].nchild == 0) {
            for (int64_t a = T[t].start; a < T[t].end; a += ORC_GROUP) {
                gs[n_group] = a;
                ge[n_group++] = a + ORC_GROUP < T[t].end ? a + ORC_GROUP : T[t].end;
            }
            continue;
        }
        int64_t cs = -1, ce = -1;
        for (int64_t k = T[t].child0; k < T[t].child0 + T[t].nchild; ++k) {
            if (T[k].end - T[k].start > ORC_GROUP) {
                if (cs >= 0) { gs[n_group] = cs; ge[n_group++] = ce; cs = -1; }
                continue;
            }
            if (cs >= 0 && T[k].end - cs <= ORC_GROUP) {
                ce = T[k].end;
                continue;
            }
            if (cs >= 0) { gs[n_group] = cs; ge[n_group++] = ce; }
            cs = T[k].start;
            ce = T[k].end;
        }
        if (cs >= 0) { gs[n_group] = cs; ge[n_group++] = ce; }
    }
    return n_group;
}

/* The groups of the tree of the particles (for the tests): starts and ends
 * in sorted positions (cap entries each) and order[k] = the particle at
 * sorted position k. Returns the number of groups, or -1 if cap is short. */
int64_t orc_gravity_tree_groups(int64_t n, const double *x, const double *y, const double *z,
                                const double *m, int32_t leaf_size, int64_t cap,
                                int64_t *gs_out, int64_t *ge_out, int64_t *order)
{
    if (n <= 0) return 0;
    const double *P[3] = {x, y, z};
    orc_kidx *srt;
    int64_t nn;
    orc_gnode *T = gtree_build(n, P, m, leaf_size, &srt, &nn);
    int64_t room = 8 * nn + n / ORC_GROUP + 2;
    int64_t *gs = (int64_t *)malloc(sizeof(int64_t) * (size_t)room);
    int64_t *ge = (int64_t *)malloc(sizeof(int64_t) * (size_t)room);
    int64_t ng = gtree_groups(T, nn, n, gs, ge);
    if (ng <= cap) {
        memcpy(gs_out, gs, sizeof(int64_t) * (size_t)ng);
        memcpy(ge_out, ge, sizeof(int64_t) * (size_t)ng);
        for (int64_t k = 0; k < n; ++k) order[k] = srt[k].idx;
    }
    free(gs);
    free(ge);
    free(T);
    free(srt);
    return ng <= cap ? ng : -1;
}

int64_t orc_gravity_tree(int64_t n, const double *x, const double *y, const double *z,
                         const double *m, double eps, double theta, int32_t leaf_size,
                         double *gx, double *gy, double *gz, double *scale, int64_t *stats,
                         int64_t *group_work)
{
    if (n <= 0) return 0;
    const double *P[3] = {x, y, z};
    orc_kidx *srt;
    int64_t nn;
    orc_gnode *T = gtree_build(n, P, m, leaf_size, &srt, &nn);

    /* groups, each walked breadth-first from the root */
    int64_t n_leaf = 0, n_node_terms = 0, n_direct_terms = 0, max_front = 1;
    for (int64_t t = 0; t < nn; ++t) n_leaf += T[t].nchild == 0;
    int64_t *gs = (int64_t *)malloc(sizeof(int64_t) * (size_t)(8 * nn + n / ORC_GROUP + 2));
    int64_t *ge = (int64_t *)malloc(sizeof(int64_t) * (size_t)(8 * nn + n / ORC_GROUP + 2));
    int64_t n_group = gtree_groups(T, nn, n, gs, ge);
    const double e2 = eps * eps;
    #pragma omp parallel for schedule(dynamic, 16) reduction(+ : n_node_terms, n_direct_terms) reduction(max : max_front)
    for (int64_t q = 0; q < n_group; ++q) {
        orc_gnode Gs;
        orc_gnode *G = &Gs;
        G->start = gs[q];
        G->end = ge[q];
        for (int a = 0; a < 3; ++a) { G->blo[a] = INFINITY; G->bhi[a] = -INFINITY; }
        for (int64_t k = G->start; k < G->end; ++k)
            for (int a = 0; a < 3; ++a) {
                double v = P[a][srt[k].idx];
                if (v < G->blo[a]) G->blo[a] = v;
                if (v > G->bhi[a]) G->bhi[a] = v;
            }
        int64_t fcap = 64, fn = 1, ncap = 64, nx, work = 0;
        int64_t *front = (int64_t *)malloc(sizeof(int64_t) * (size_t)fcap);
        int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncap);
        front[0] = 0;
        int64_t gn = G->end - G->start;
        double *ax = (double *)calloc((size_t)gn * 4, sizeof(double));
        while (fn > 0) {
            nx = 0;
            for (int64_t f = 0; f < fn; ++f) {
                const orc_gnode *N = &T[front[f]];
                double dd = 0.0;
                for (int a = 0; a < 3; ++a) {
                    double e = 0.0;
                    if (N->c[a] < G->blo[a]) e = G->blo[a] - N->c[a];
                    else if (N->c[a] > G->bhi[a]) e = N->c[a] - G->bhi[a];
                    dd += e * e;
                }
                if (sqrt(dd) > N->s / theta + N->delta) {
                    for (int64_t k = 0; k < gn; ++k) {
                        int64_t i = srt[G->start + k].idx;
                        double d[3] = {x[i] - N->c[0], y[i] - N->c[1], z[i] - N->c[2]};
                        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                        double rinv = 1.0 / sqrt(r2);
                        double rinv2 = rinv * rinv;
                        double rinv3 = rinv * rinv2;
                        double rinv5 = rinv3 * rinv2;
                        double rinv7 = rinv5 * rinv2;
                        double Qd[3] = {N->Q[0] * d[0] + N->Q[1] * d[1] + N->Q[2] * d[2],
                                        N->Q[1] * d[0] + N->Q[3] * d[1] + N->Q[4] * d[2],
                                        N->Q[2] * d[0] + N->Q[4] * d[1] + N->Q[5] * d[2]};
                        double dQd = d[0] * Qd[0] + d[1] * Qd[1] + d[2] * Qd[2];
                        double t[3];
                        for (int a = 0; a < 3; ++a) {
                            t[a] = -N->M * d[a] * rinv3 + Qd[a] * rinv5 - 2.5 * dQd * d[a] * rinv7;
                            ax[4 * k + a] += t[a];
                        }
                        ax[4 * k + 3] += sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
                    }
                    n_node_terms += gn;
                    work += 1;
                } else if (N->nchild == 0) {
                    for (int64_t k = 0; k < gn; ++k) {
                        int64_t i = srt[G->start + k].idx;
                        for (int64_t l = N->start; l < N->end; ++l) {
                            int64_t j = srt[l].idx;
                            if (j == i) continue;
                            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
                            double d2 = dx * dx + dy * dy + dz * dz + e2;
                            double inv = 1.0 / (d2 * sqrt(d2));
                            double t0 = -m[j] * dx * inv, t1 = -m[j] * dy * inv,
                                   t2 = -m[j] * dz * inv;
                            ax[4 * k + 0] += t0;
                            ax[4 * k + 1] += t1;
                            ax[4 * k + 2] += t2;
                            ax[4 * k + 3] += sqrt(t0 * t0 + t1 * t1 + t2 * t2);
                        }
                    }
                    n_direct_terms += gn * (N->end - N->start);
                    work += N->end - N->start;
                } else {
                    for (int64_t k = N->child0; k < N->child0 + N->nchild; ++k) {
                        if (nx == ncap) {
                            ncap *= 2;
                            next = (int64_t *)realloc(next, sizeof(int64_t) * (size_t)ncap);
                        }
                        next[nx++] = k;
                    }
                }
            }
            int64_t *tmp = front; front = next; next = tmp;
            int64_t tc = fcap; fcap = ncap; ncap = tc;
            fn = nx;
            if (fn > max_front) max_front = fn;
        }
        for (int64_t k = 0; k < gn; ++k) {
            int64_t i = srt[G->start + k].idx;
            gx[i] = ax[4 * k + 0];
            gy[i] = ax[4 * k + 1];
            gz[i] = ax[4 * k + 2];
            if (scale) scale[i] = ax[4 * k + 3];
        }
        if (group_work) group_work[q] = work;
        free(ax);
        free(front);
        free(next);
    }
    if (stats) {
        stats[0] = nn;
        stats[1] = n_leaf;
        stats[2] = n_node_terms;
        stats[3] = n_direct_terms;
        stats[4] = max_front;
    }
    if (stats) stats[5] = n_group;
    free(gs);
    free(ge);
    free(T);
    free(srt);
    return nn;
}

/* The tree itself, for the tests: out[16 t + q] = M, c (3), Q (6), s,
 * delta, level, start, end, nchild of node t (start and end are positions in
 * the sorted order, order[k] the particle at position k). Returns the node
 * count; nothing is written when it exceeds cap. */
int64_t orc_gravity_tree_nodes(int64_t n, const double *x, const double *y, const double *z,
                               const double *m, int32_t leaf_size, int64_t cap, double *out,
                               int64_t *order)
{
    if (n <= 0) return 0;
    const double *P[3] = {x, y, z};
    orc_kidx *srt;
    int64_t nn;
    orc_gnode *T = gtree_build(n, P, m, leaf_size, &srt, &nn);
    if (nn <= cap) {
        for (int64_t t = 0; t < nn; ++t) {
            double *o = out + 16 * t;
            o[0] = T[t].M;
            for (int a = 0; a < 3; ++a) o[1 + a] = T[t].c[a];
            for (int q = 0; q < 6; ++q) o[4 + q] = T[t].Q[q];
            o[10] = T[t].s;
            o[11] = T[t].delta;
            o[12] = T[t].level;
            o[13] = (double)T[t].start;
            o[14] = (double)T[t].end;
            o[15] = T[t].nchild;
        }
        for (int64_t k = 0; k < n; ++k) order[k] = srt[k].idx;
    }
    free(T);
    free(srt);
    return nn;
}
