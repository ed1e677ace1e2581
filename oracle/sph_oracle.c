/*
 * sph_oracle.c -- plain, slow, FP64 reference of the SPH neighbour-interaction
 * sweep of "Smoothed Particle Hydrodynamics in pkdgrav3 for Shock Physics
 * Simulations. I. Hydrodynamics" (Meier, Potter, Reinhardt, Stadel).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the GPU path.
 *
 * What it computes, each function citing the passage it follows:
 *   - kernel family W = sigma f(q) / H^3, q = r/H      (Sec. 2.3, kernel list)
 *   - neighbour sets by a uniform cell list            (Sec. 2.3.2)
 *   - density sum, d rho / dH and the grad-h term      (Sec. 2.3.3, eq:Density_estimate)
 *   - smoothing length from the constant-mass rule     (Sec. 2.3.3)
 *   - equation of state                                (Sec. 2.3.1)
 *   - pressure force, PdV du/dt, artificial viscosity  (Sec. 2.3.5, eq:AV_heating)
 *   - acceleration and signal-velocity time-step limits (Sec. 2.3.6, eq:courant_condition)
 *   - entropy-conserving update of u, evolved density  (Sec. 2.3.5, Sec. 2.3.3)
 *   - interface correction: kernel imbalance and averages (Sec. 2.3.4, eq:Kernel_imbalance)
 * The kick-drift-kick sequence is composed in oracle/__init__.py.
 *
 * Conventions (readings of the paper, listed in the design notes):
 *   H  = kernel support radius; h = H/2 is the smoothing length, so the
 *        kernel radius R_kernel(h) = 2h = H.
 *   x_ij = x_i - x_j with the minimum image taken per component:
 *        d = x_j - x_i;  d > L/2 -> d - L;  d < -L/2 -> d + L;  x_ij = -d.
 *   r^2 = (dx*dx + dy*dy) + dz*dz, evaluated left to right, never contracted
 *        into FMA (build with -ffp-contract=off).
 *   Gather set  G_i = { j != i : r_ij^2 < H_i^2 }.
 *   Force set   F_i = { j != i : r_ij^2 < max(H_i, H_j)^2 }.
 *   The density sum includes the particle itself.
 *
 * Every function is plain C, single-threaded in meaning; OpenMP only splits
 * independent particles across threads for timing.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* Layout mirrored by oracle/__init__.py (ctypes). */
typedef struct {
    int32_t kernel;   /* 0 cubic spline (M4), 1 Wendland C2, 2 Wendland C4, 3 Wendland C6 */
    int32_t periodic; /* 1: periodic box [lo, hi); 0: open boundary */
    int32_t eos;      /* 0 ideal gas, 1 stiffened gas */
    int32_t nr_maxit; /* iteration cap of the smoothing-length solve */
    double n_ngb;     /* target neighbour number */
    double lo[3], hi[3];
    double gamma, P0;
    double alpha, beta, eps_av; /* artificial viscosity */
    double eta_c, eta_a, dt_max;/* time-step limits */
    double h_max;     /* cap on the support radius H */
    double nr_tol;    /* relative tolerance on H */
    int32_t flags;    /* ORC_ENTROPY: du/dt without the PdV term (the isentropic
                         change is applied by orc_isentrope); ORC_EVOLVED: the
                         force pass also returns d rho / dt */
    int32_t pad_;
} orc_params;

#define ORC_ENTROPY 1
#define ORC_EVOLVED 2

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the row loops (timing only: rows are independent). */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_params_size(void) { return (int)sizeof(orc_params); }

/* ------------------------------------------------------------------------ */
/* Kernel family (Sec. 2.3: cubic spline of Monaghan 1992; Wendland C2, C4, */
/* C6 of Dehnen & Aly 2012).  W(r, H) = sigma f(r/H) / H^3, support q < 1.  */
/* ------------------------------------------------------------------------ */

double orc_sigma(int kernel) {
    switch (kernel) {
    case 0: return 8.0 / ORC_PI;
    case 1: return 21.0 / (2.0 * ORC_PI);
    case 2: return 495.0 / (32.0 * ORC_PI);
    case 3: return 1365.0 / (64.0 * ORC_PI);
    }
    return NAN;
}

/* f(q) and g(q) = f'(q)/q (finite at q = 0) for the shape functions. */
static void shape(int kernel, double q, double *f, double *g) {
    if (q >= 1.0) { *f = 0.0; *g = 0.0; return; }
    double s = 1.0 - q;
    switch (kernel) {
    case 0:
        if (q < 0.5) {
            *f = 1.0 - 6.0 * q * q + 6.0 * q * q * q;
            *g = -12.0 + 18.0 * q;
        } else {
            *f = 2.0 * s * s * s;
            *g = -6.0 * s * s / q;
        }
        return;
    case 1: {
        double s3 = s * s * s;
        *f = s3 * s * (1.0 + 4.0 * q);
        *g = -20.0 * s3;
        return;
    }
    case 2: {
        double s5 = s * s * s * s * s;
        *f = s5 * s * (1.0 + 6.0 * q + (35.0 / 3.0) * q * q);
        *g = -(56.0 / 3.0) * s5 * (1.0 + 5.0 * q);
        return;
    }
    case 3: {
        double s7 = s * s * s * s * s * s * s;
        *f = s7 * s * (1.0 + 8.0 * q + 25.0 * q * q + 32.0 * q * q * q);
        *g = -22.0 * s7 * (1.0 + 7.0 * q + 16.0 * q * q);
        return;
    }
    }
    *f = NAN; *g = NAN;
}

/* Exported for the kernel pins: f(q) and f'(q) on an array of q. */
void orc_kernel_shape(int kernel, int64_t n, const double *q, double *f, double *fp) {
    for (int64_t k = 0; k < n; ++k) {
        double fv, gv;
        shape(kernel, q[k], &fv, &gv);
        f[k] = fv;
        fp[k] = gv * q[k];
    }
}

/* W(r,H), dW/dr and dW/dH exported for the derivative pins. */
void orc_kernel_w(int kernel, int64_t n, const double *r, const double *H,
                  double *w, double *dwdr, double *dwdh) {
    double sig = orc_sigma(kernel);
    for (int64_t k = 0; k < n; ++k) {
        double q = r[k] / H[k];
        double fv, gv;
        shape(kernel, q, &fv, &gv);
        double h3 = H[k] * H[k] * H[k];
        w[k] = sig * fv / h3;
        dwdr[k] = sig * gv * q / (h3 * H[k]);
        dwdh[k] = -sig * (3.0 * fv + q * q * gv) / (h3 * H[k]);
    }
}

/* ------------------------------------------------------------------------ */
/* Geometry: minimum image and the pair distance.                            */
/* ------------------------------------------------------------------------ */

static inline double min_image(double d, double L, double halfL) {
    if (d > halfL) return d - L;
    if (d < -halfL) return d + L;
    return d;
}

/* d = x_j - x_i per component (minimum image when periodic); returns r^2. */
static inline double pair_d(const orc_params *p, const double *L, const double *hL,
                            const double *x, const double *y, const double *z,
                            int64_t i, int64_t j, double *dx, double *dy, double *dz) {
    double ex = x[j] - x[i], ey = y[j] - y[i], ez = z[j] - z[i];
    if (p->periodic) {
        ex = min_image(ex, L[0], hL[0]);
        ey = min_image(ey, L[1], hL[1]);
        ez = min_image(ez, L[2], hL[2]);
    }
    *dx = ex; *dy = ey; *dz = ez;
    double r2 = ex * ex + ey * ey;
    r2 = r2 + ez * ez;
    return r2;
}

/* ------------------------------------------------------------------------ */
/* Uniform cell list: deliberately a different search structure from the    */
/* tree of the method, so that the two cannot share a mistake.              */
/* ------------------------------------------------------------------------ */

typedef struct {
    int nc[3];
    double lo[3], cs[3];
    int periodic;
    int64_t *start; /* ncell + 1 */
    int64_t *idx;   /* particles grouped by cell */
} grid;

static int64_t cell_coord(double v, double lo, double cs, int nc) {
    double t = floor((v - lo) / cs);
    if (t < 0) t = 0;
    if (t > nc - 1) t = nc - 1;
    return (int64_t)t;
}

static int grid_build(grid *g, const orc_params *p, int64_t n, const double *x,
                      const double *y, const double *z, double rmin) {
    double lo[3], hi[3];
    if (p->periodic) {
        for (int a = 0; a < 3; ++a) { lo[a] = p->lo[a]; hi[a] = p->hi[a]; }
    } else {
        const double *c[3] = {x, y, z};
        for (int a = 0; a < 3; ++a) {
            double mn = INFINITY, mx = -INFINITY;
            for (int64_t i = 0; i < n; ++i) {
                if (c[a][i] < mn) mn = c[a][i];
                if (c[a][i] > mx) mx = c[a][i];
            }
            if (n == 0) { mn = 0; mx = 1; }
            double pad = 1e-9 * (fabs(mn) + fabs(mx) + 1.0);
            lo[a] = mn - pad;
            hi[a] = mx + pad;
        }
    }
    if (!(rmin > 0)) rmin = 1e-30;
    int64_t cap = 4 * n + 64;
    for (;;) {
        int64_t tot = 1;
        for (int a = 0; a < 3; ++a) {
            double L = hi[a] - lo[a];
            double k = floor(L / rmin);
            if (k < 1) k = 1;
            if (k > 1 << 20) k = 1 << 20;
            g->nc[a] = (int)k;
            g->cs[a] = L / k;
            g->lo[a] = lo[a];
            tot *= (int64_t)k;
        }
        if (tot <= cap) break;
        rmin *= 1.5;
    }
    g->periodic = p->periodic;
    int64_t ncell = (int64_t)g->nc[0] * g->nc[1] * g->nc[2];
    g->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    g->idx = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *cell = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!g->start || !g->idx || !cell) { free(cell); return -1; }
    for (int64_t i = 0; i < n; ++i) {
        int64_t cx = cell_coord(x[i], g->lo[0], g->cs[0], g->nc[0]);
        int64_t cy = cell_coord(y[i], g->lo[1], g->cs[1], g->nc[1]);
        int64_t cz = cell_coord(z[i], g->lo[2], g->cs[2], g->nc[2]);
        cell[i] = (cz * g->nc[1] + cy) * g->nc[0] + cx;
        g->start[cell[i] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) g->start[c + 1] += g->start[c];
    int64_t *fill = (int64_t *)malloc((size_t)ncell * sizeof(int64_t) + 8);
    memcpy(fill, g->start, (size_t)ncell * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) g->idx[fill[cell[i]]++] = i;
    free(fill);
    free(cell);
    return 0;
}

static void grid_free(grid *g) { free(g->start); free(g->idx); }

/* Per-thread growable list of (j, r^2). */
typedef struct { int64_t *j; double *r2; int64_t n, cap; } plist;

static void plist_push(plist *l, int64_t j, double r2) {
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 1024;
        l->j = (int64_t *)realloc(l->j, (size_t)l->cap * sizeof(int64_t));
        l->r2 = (double *)realloc(l->r2, (size_t)l->cap * sizeof(double));
    }
    l->j[l->n] = j; l->r2[l->n] = r2; l->n++;
}

/* All j != i with r_ij^2 < R^2 (R^2 = R*R).  Each j is visited once. */
static void grid_query(const grid *g, const orc_params *p, const double *L, const double *hL,
                       const double *x, const double *y, const double *z,
                       int64_t i, double R, plist *out) {
    out->n = 0;
    double R2 = R * R;
    int64_t c0[3] = {cell_coord(x[i], g->lo[0], g->cs[0], g->nc[0]),
                     cell_coord(y[i], g->lo[1], g->cs[1], g->nc[1]),
                     cell_coord(z[i], g->lo[2], g->cs[2], g->nc[2])};
    int64_t kmin[3], kmax[3];
    int full[3];
    for (int a = 0; a < 3; ++a) {
        double kk = ceil(R / g->cs[a]);
        if (!(kk < 1e9)) kk = 1e9;
        int64_t k = (int64_t)kk;
        if (k < 1) k = 1;
        full[a] = (2 * k + 1 >= g->nc[a]);
        if (full[a]) { kmin[a] = 0; kmax[a] = g->nc[a] - 1; }
        else { kmin[a] = c0[a] - k; kmax[a] = c0[a] + k; }
        if (!g->periodic && !full[a]) {
            if (kmin[a] < 0) kmin[a] = 0;
            if (kmax[a] > g->nc[a] - 1) kmax[a] = g->nc[a] - 1;
        }
    }
    for (int64_t cz = kmin[2]; cz <= kmax[2]; ++cz) {
        int64_t wz = ((cz % g->nc[2]) + g->nc[2]) % g->nc[2];
        for (int64_t cy = kmin[1]; cy <= kmax[1]; ++cy) {
            int64_t wy = ((cy % g->nc[1]) + g->nc[1]) % g->nc[1];
            for (int64_t cx = kmin[0]; cx <= kmax[0]; ++cx) {
                int64_t wx = ((cx % g->nc[0]) + g->nc[0]) % g->nc[0];
                int64_t c = (wz * g->nc[1] + wy) * g->nc[0] + wx;
                for (int64_t t = g->start[c]; t < g->start[c + 1]; ++t) {
                    int64_t j = g->idx[t];
                    if (j == i) continue;
                    double dx, dy, dz;
                    double r2 = pair_d(p, L, hL, x, y, z, i, j, &dx, &dy, &dz);
                    if (r2 < R2) plist_push(out, j, r2);
                }
            }
        }
    }
}

static void box_lengths(const orc_params *p, double *L, double *hL) {
    for (int a = 0; a < 3; ++a) {
        L[a] = p->hi[a] - p->lo[a];
        hL[a] = 0.5 * L[a];
    }
}

static int cmp_i64(const void *a, const void *b) {
    int64_t u = *(const int64_t *)a, v = *(const int64_t *)b;
    return (u > v) - (u < v);
}

static double max_of(int64_t n, const double *v) {
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i) if (v[i] > m) m = v[i];
    return m;
}

/* ------------------------------------------------------------------------ */
/* Neighbour sets (Sec. 2.3.2): mode 0 gather G_i, mode 1 force set F_i.    */
/* Call with idx == NULL to get the row lengths in counts[]; then call      */
/* again with offsets (n+1, exclusive prefix of counts) and idx to fill      */
/* rows sorted ascending.                                                    */
/* ------------------------------------------------------------------------ */

int orc_neighbors(const orc_params *p, int64_t n, const double *x, const double *y,
                  const double *z, const double *H, int mode, int64_t *counts,
                  const int64_t *offsets, int64_t *idx) {
    double L[3], hL[3];
    box_lengths(p, L, hL);
    double Hmax = max_of(n, H);
    grid g;
    if (grid_build(&g, p, n, x, y, z, Hmax) != 0) return -1;
    #pragma omp parallel
    {
        plist l = {0};
        #pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            double R = (mode == 0) ? H[i] : Hmax;
            grid_query(&g, p, L, hL, x, y, z, i, R, &l);
            int64_t cnt = 0;
            int64_t base = idx ? offsets[i] : 0;
            for (int64_t t = 0; t < l.n; ++t) {
                int64_t j = l.j[t];
                double Hi2 = H[i] * H[i];
                double Hs = (mode == 0) ? H[i] : (H[i] > H[j] ? H[i] : H[j]);
                double Hs2 = (mode == 0) ? Hi2 : Hs * Hs;
                if (l.r2[t] < Hs2) {
                    if (idx) idx[base + cnt] = j;
                    cnt++;
                }
            }
            if (idx) qsort(idx + base, (size_t)cnt, sizeof(int64_t), cmp_i64);
            else counts[i] = cnt;
        }
        free(l.j); free(l.r2);
    }
    grid_free(&g);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Density at a given H (eq:Density_estimate) and the grad-h term Omega     */
/* (Sec. 2.3.3).  Self contribution included.                                */
/*   rho    = sum_{j in G_i + i} m_j W(r_ij, H_i)                            */
/*   drho   = d rho / dH_i = sum m_j dW/dH                                   */
/*   Omega  = 1 + (H_i / (3 rho)) drho  (h d/dh = H d/dH since h = H/2)      */
/* ------------------------------------------------------------------------ */

typedef struct { double rho, drho; int64_t count; } dens_val;

/* Sum over a list of (m_j, r_j) at support H; list holds every j with
 * r_j < some R >= H; membership is re-tested as r^2 < H^2.              */
static dens_val dens_sum(int kernel, double sig, double mi, double H,
                         int64_t nl, const double *mj, const double *r2j, const double *rj) {
    double H2 = H * H;
    double sf = mi;               /* self: f(0) = 1 */
    double sd = 3.0 * mi;         /* self: 3 f(0) + q^2 g = 3 */
    int64_t cnt = 0;
    for (int64_t t = 0; t < nl; ++t) {
        if (!(r2j[t] < H2)) continue;
        double q = rj[t] / H;
        double f, g;
        shape(kernel, q, &f, &g);
        sf += mj[t] * f;
        sd += mj[t] * (3.0 * f + q * q * g);
        cnt++;
    }
    dens_val v;
    double H3 = H * H * H;
    v.rho = sig * sf / H3;
    v.drho = -sig * sd / (H3 * H);
    v.count = cnt;
    return v;
}

/* Rows: which == NULL computes every particle (outputs indexed by particle);
 * otherwise only particles which[0..nw) (outputs indexed 0..nw). */
int orc_density(const orc_params *p, int64_t n, const double *x, const double *y,
                const double *z, const double *m, const double *H, const int64_t *which,
                int64_t nw, double *rho, double *drho, double *omega, int64_t *count) {
    double L[3], hL[3];
    box_lengths(p, L, hL);
    double sig = orc_sigma(p->kernel);
    grid g;
    if (grid_build(&g, p, n, x, y, z, max_of(n, H)) != 0) return -1;
    #pragma omp parallel
    {
        plist l = {0};
        double *mj = NULL, *rj = NULL;
        int64_t cap = 0;
        if (!which) nw = n;
        #pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < nw; ++k) {
            int64_t i = which ? which[k] : k;
            grid_query(&g, p, L, hL, x, y, z, i, H[i], &l);
            if (l.n > cap) {
                cap = l.n;
                mj = (double *)realloc(mj, (size_t)cap * sizeof(double));
                rj = (double *)realloc(rj, (size_t)cap * sizeof(double));
            }
            for (int64_t t = 0; t < l.n; ++t) { mj[t] = m[l.j[t]]; rj[t] = sqrt(l.r2[t]); }
            dens_val v = dens_sum(p->kernel, sig, m[i], H[i], l.n, mj, l.r2, rj);
            rho[k] = v.rho;
            drho[k] = v.drho;
            omega[k] = 1.0 + H[i] * v.drho / (3.0 * v.rho);
            count[k] = v.count;
        }
        free(l.j); free(l.r2); free(mj); free(rj);
    }
    grid_free(&g);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Interface correction (Sec. 2.3.4), at given H (h = H/2):                  */
/* kernel imbalance (eq:Kernel_imbalance)                                   */
/*   I_i = alpha |sum_j kappa_ij (x_j - x_i) m_j W_ij(h_i)|                 */
/*         / (h_i sum_j m_j W_ij(h_i)),                                     */
/* kappa_ij = +1 if i and j are of the same material, -1 otherwise (mat ==  */
/* NULL: one material); x_j - x_i is the minimum image; the sums run over   */
/* G_i and i itself (which adds only to the denominator).                   */
/* ------------------------------------------------------------------------ */
int orc_imbalance(const orc_params *p, int64_t n, const double *x, const double *y,
                  const double *z, const double *m, const double *H, const double *mat,
                  double alpha, const int64_t *which, int64_t nw, double *I) {
    double L[3], hL[3];
    box_lengths(p, L, hL);
    grid g;
    if (grid_build(&g, p, n, x, y, z, max_of(n, H)) != 0) return -1;
    #pragma omp parallel
    {
        plist l = {0};
        if (!which) nw = n;
        #pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < nw; ++k) {
            int64_t i = which ? which[k] : k;
            grid_query(&g, p, L, hL, x, y, z, i, H[i], &l);
            double f, gq;
            shape(p->kernel, 0.0, &f, &gq);
            double den = m[i] * f;   /* self term */
            double nx = 0.0, ny = 0.0, nz = 0.0;
            for (int64_t t = 0; t < l.n; ++t) {
                int64_t j = l.j[t];
                double dx, dy, dz;
                double r2 = pair_d(p, L, hL, x, y, z, i, j, &dx, &dy, &dz);   /* d = x_j - x_i */
                shape(p->kernel, sqrt(r2) / H[i], &f, &gq);
                double w = m[j] * f;   /* W up to the common factor sigma / H_i^3 */
                double kappa = (mat && mat[j] != mat[i]) ? -1.0 : 1.0;
                den += w;
                nx += kappa * w * dx;
                ny += kappa * w * dy;
                nz += kappa * w * dz;
            }
            I[k] = alpha * sqrt(nx * nx + ny * ny + nz * nz) / (0.5 * H[i] * den);
        }
        free(l.j); free(l.r2);
    }
    grid_free(&g);
    return 0;
}

/* Interface-correction averages (Sec. 2.3.4): with w_ij = exp(-I_j^2)      */
/* W_ij(h_i) over G_i and i itself,                                         */
/*   Tbar_i = sum_j w_ij T_j / sum_j w_ij,   Pbar_i likewise.               */
int orc_ic_average(const orc_params *p, int64_t n, const double *x, const double *y,
                   const double *z, const double *H, const double *I, const double *T,
                   const double *P, const int64_t *which, int64_t nw, double *Tbar,
                   double *Pbar) {
    double L[3], hL[3];
    box_lengths(p, L, hL);
    grid g;
    if (grid_build(&g, p, n, x, y, z, max_of(n, H)) != 0) return -1;
    #pragma omp parallel
    {
        plist l = {0};
        if (!which) nw = n;
        #pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < nw; ++k) {
            int64_t i = which ? which[k] : k;
            grid_query(&g, p, L, hL, x, y, z, i, H[i], &l);
            double f, gq;
            shape(p->kernel, 0.0, &f, &gq);
            double w = exp(-I[i] * I[i]) * f;   /* self term */
            double sw = w, st = w * T[i], sp = w * P[i];
            for (int64_t t = 0; t < l.n; ++t) {
                int64_t j = l.j[t];
                shape(p->kernel, sqrt(l.r2[t]) / H[i], &f, &gq);
                w = exp(-I[j] * I[j]) * f;
                sw += w;
                st += w * T[j];
                sp += w * P[j];
            }
            Tbar[k] = st / sw;
            Pbar[k] = sp / sw;
        }
        free(l.j); free(l.r2);
    }
    grid_free(&g);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Smoothing length (Sec. 2.3.3): the kernel keeps a constant effective     */
/* mass, (4 pi / 3) H^3 rho_i(H) = n_ngb m_i.  The left side is             */
/* (4 pi / 3) sigma sum_j m_j f(r_j / H): non-decreasing in H, so the root  */
/* is unique.  Found here by Newton's method (dF/dH = 4 pi H^2 rho Omega)   */
/* safeguarded by bisection on a bracket.  The iteration need not copy the  */
/* GPU's; only the root matters.  H is capped at h_max (and below half the  */
/* box when periodic); a capped particle is counted as not converged.       */
/* ------------------------------------------------------------------------ */

/* H holds the first guesses of every particle on entry; on return H[i] (or
 * H[k] for a row subset, see orc_density) holds the solution. */
int orc_solve_h(const orc_params *p, int64_t n, const double *x, const double *y,
                const double *z, const double *m, const double *H0, const int64_t *which,
                int64_t nw, double *H, double *rho, double *omega, int64_t *count,
                int32_t *iters, int64_t *n_noconv) {
    double L[3], hL[3];
    box_lengths(p, L, hL);
    double sig = orc_sigma(p->kernel);
    double cap = p->h_max;
    if (p->periodic) {
        double lmin = L[0] < L[1] ? L[0] : L[1];
        lmin = lmin < L[2] ? lmin : L[2];
        if (0.5 * lmin < cap) cap = 0.5 * lmin;
    }
    double tol = p->nr_tol > 0 ? p->nr_tol : 1e-14;
    int maxit = p->nr_maxit > 0 ? p->nr_maxit : 200;
    double c43 = 4.0 * ORC_PI / 3.0;
    grid g;
    double Hm = max_of(n, H0);
    if (Hm > cap) Hm = cap;
    if (grid_build(&g, p, n, x, y, z, Hm) != 0) return -1;
    int64_t bad = 0;
    #pragma omp parallel reduction(+ : bad)
    {
        plist l = {0};
        double *mj = NULL, *rj = NULL;
        int64_t lcap = 0;
        if (!which) nw = n;
        #pragma omp for schedule(dynamic, 16)
        for (int64_t k = 0; k < nw; ++k) {
            int64_t i = which ? which[k] : k;
            double target = p->n_ngb * m[i];
            double Hg = H0[i];
            if (!(Hg > 0)) Hg = cap * 0.01;
            if (Hg > cap) Hg = cap;
            /* Bracket: F(0+) < 0; grow hi until F(hi) >= 0 or the cap. */
            double hi = Hg;
            int capped = 0;
            dens_val v;
            for (;;) {
                grid_query(&g, p, L, hL, x, y, z, i, hi, &l);
                if (l.n > lcap) {
                    lcap = l.n;
                    mj = (double *)realloc(mj, (size_t)lcap * sizeof(double));
                    rj = (double *)realloc(rj, (size_t)lcap * sizeof(double));
                }
                for (int64_t t = 0; t < l.n; ++t) { mj[t] = m[l.j[t]]; rj[t] = sqrt(l.r2[t]); }
                v = dens_sum(p->kernel, sig, m[i], hi, l.n, mj, l.r2, rj);
                double F = c43 * hi * hi * hi * v.rho - target;
                if (F >= 0) break;
                if (hi >= cap) { capped = 1; break; }
                hi *= 1.25;
                if (hi > cap) hi = cap;
            }
            int it = 0;
            double Hc = hi;
            if (capped) {
                bad++;
            } else {
                double lo = 0.0;
                double h = Hg < hi ? Hg : hi;
                for (it = 1; it <= maxit; ++it) {
                    v = dens_sum(p->kernel, sig, m[i], h, l.n, mj, l.r2, rj);
                    double F = c43 * h * h * h * v.rho - target;
                    double om = 1.0 + h * v.drho / (3.0 * v.rho);
                    double dF = 4.0 * ORC_PI * h * h * v.rho * om;
                    if (F < 0) lo = h; else hi = h;
                    /* stop on the size of the Newton step itself: near the root it
                     * drops below the spacing of doubles, and h - step == h would
                     * otherwise look like a step leaving the bracket */
                    double step = (dF > 0) ? F / dF : NAN;
                    if (F == 0.0 || fabs(step) <= tol * h) { Hc = h; break; }
                    double hn = h - step;
                    if (!(hn > lo && hn < hi)) hn = 0.5 * (lo + hi);
                    h = hn;
                    Hc = h;
                }
                if (it > maxit) bad++;
            }
            v = dens_sum(p->kernel, sig, m[i], Hc, l.n, mj, l.r2, rj);
            H[k] = Hc;
            rho[k] = v.rho;
            omega[k] = 1.0 + Hc * v.drho / (3.0 * v.rho);
            count[k] = v.count;
            iters[k] = it;
        }
        free(l.j); free(l.r2); free(mj); free(rj);
    }
    grid_free(&g);
    *n_noconv = bad;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Equation of state (Sec. 2.3.1): built-in ideal gas P = (gamma-1) rho u,  */
/* c^2 = gamma (gamma-1) u; and the stiffened gas                           */
/* P = (gamma-1) rho u - gamma P0, c^2 = gamma (P + P0) / rho.  A negative   */
/* c^2 is clamped to zero; a negative P is kept.                             */
/* ------------------------------------------------------------------------ */

void orc_eos(const orc_params *p, int64_t n, const double *rho, const double *u,
             double *P, double *c) {
    double gm = p->gamma;
    for (int64_t i = 0; i < n; ++i) {
        double Pi, c2;
        if (p->eos == 0) {
            Pi = (gm - 1.0) * rho[i] * u[i];
            c2 = gm * (gm - 1.0) * u[i];
        } else {
            Pi = (gm - 1.0) * rho[i] * u[i] - gm * p->P0;
            c2 = gm * (Pi + p->P0) / rho[i];
        }
        P[i] = Pi;
        c[i] = c2 > 0.0 ? sqrt(c2) : 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Entropy-conserving update (Sec. 2.3.5): u_new = u(rho_new, s(rho_old,     */
/* u_old)), the internal energy that keeps the entropy of (rho_old, u_old)    */
/* at the new density.  Ideal gas (Springel & Hernquist 2002): P / rho^gamma  */
/* is the entropy function, so u scales as rho^(gamma-1).  Stiffened gas      */
/* P = (gamma-1) rho u - gamma P0: along an adiabat du = (P/rho^2) d rho,     */
/* whose solution keeps (P + P0) / rho^gamma fixed, i.e.                      */
/*   u - P0/rho  scales as rho^(gamma-1).                                     */
/* ------------------------------------------------------------------------ */
void orc_isentrope(const orc_params *p, int64_t n, const double *rho_old, const double *u_old,
                   const double *rho_new, double *u_new) {
    const double gm = p->gamma;
    for (int64_t i = 0; i < n; ++i) {
        const double ratio = pow(rho_new[i] / rho_old[i], gm - 1.0);
        if (p->eos == 0)
            u_new[i] = u_old[i] * ratio;
        else
            u_new[i] = (u_old[i] - p->P0 / rho_old[i]) * ratio + p->P0 / rho_new[i];
    }
}

/* ------------------------------------------------------------------------ */
/* Forces (Sec. 2.3.5).  For j in F_i, with x_ij = x_i - x_j, v_ij = v_i -  */
/* v_j, dW/dr(r, H_k) x_ij / r = G_k x_ij where G_k = sigma g(q_k) / H_k^5  */
/* (zero when r >= H_k), and A_k = P_k / (Omega_k rho_k^2):                 */
/*   a_i     = - sum m_j [A_i G_i + A_j G_j + Pi_ij (G_i + G_j)/2] x_ij      */
/*   du_i/dt =   A_i sum m_j G_i (v_ij . x_ij)                               */
/*             + 1/2 sum m_j Pi_ij (G_i + G_j)/2 (v_ij . x_ij)              */
/* Artificial viscosity (Monaghan 1992 form): hbar, cbar, rhobar arithmetic */
/* means, h = H/2;  mu = hbar (v_ij . x_ij) / (r^2 + eps hbar^2);           */
/* Pi = (-alpha cbar mu + beta mu^2) / rhobar if v_ij . x_ij < 0, else 0.   */
/* Time-step limits (Sec. 2.3.6): dt_a = eta_a sqrt(H_i / |a_i|);           */
/* dt_cfl = eta_c h_i / ((1 + 0.6 alpha) c_i + 0.6 beta max_j |min(0,mu)|); */
/* dt_i = min(dt_a, dt_cfl, dt_max).                                        */
/* ------------------------------------------------------------------------ */

/* With ORC_ENTROPY the PdV term is left out of du/dt: the entropy-conserving */
/* scheme (Sec. 2.3.5) changes u isentropically with the density instead      */
/* (orc_isentrope) and integrates only the viscous heating.  With ORC_EVOLVED */
/* the force pass also returns the continuity equation's rate of density     */
/* change (Sec. 2.3.3, evolved density), in the grad-h form                  */
/*   d rho_i/dt = (1/Omega_i) sum m_j (v_ij . x_ij) G_i.                     */
int orc_forces(const orc_params *p, int64_t n, const double *x, const double *y,
               const double *z, const double *vx, const double *vy, const double *vz,
               const double *m, const double *H, const double *rho, const double *omega,
               const double *P, const double *c, const int64_t *which, int64_t nw,
               double *ax, double *ay, double *az, double *dudt, double *dti, int64_t *count,
               double *drho) {
    double L[3], hL[3];
    box_lengths(p, L, hL);
    double sig = orc_sigma(p->kernel);
    double Hmax = max_of(n, H);
    double *A = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    for (int64_t i = 0; i < n; ++i) A[i] = P[i] / (omega[i] * rho[i] * rho[i]);
    grid g;
    if (grid_build(&g, p, n, x, y, z, Hmax) != 0) { free(A); return -1; }
    #pragma omp parallel
    {
        plist l = {0};
        if (!which) nw = n;
        #pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < nw; ++k) {
            int64_t i = which ? which[k] : k;
            grid_query(&g, p, L, hL, x, y, z, i, Hmax, &l);
            double Hi2 = H[i] * H[i];
            double hi_s = 0.5 * H[i];
            double sax = 0, say = 0, saz = 0, spdv = 0, sav = 0, mumax = 0;
            int64_t cnt = 0;
            for (int64_t t = 0; t < l.n; ++t) {
                int64_t j = l.j[t];
                double Hj2 = H[j] * H[j];
                double Hs2 = Hi2 > Hj2 ? Hi2 : Hj2;
                if (!(l.r2[t] < Hs2)) continue;
                cnt++;
                double dx, dy, dz;
                double r2 = pair_d(p, L, hL, x, y, z, i, j, &dx, &dy, &dz);
                /* x_ij = x_i - x_j = -d */
                double xx = -dx, xy = -dy, xz = -dz;
                double r = sqrt(r2);
                double Gi = 0.0, Gj = 0.0, f, gq;
                if (r2 < Hi2) {
                    shape(p->kernel, r / H[i], &f, &gq);
                    double h5 = Hi2 * Hi2 * H[i];
                    Gi = sig * gq / h5;
                }
                if (r2 < Hj2) {
                    shape(p->kernel, r / H[j], &f, &gq);
                    double h5 = Hj2 * Hj2 * H[j];
                    Gj = sig * gq / h5;
                }
                double wx = vx[i] - vx[j], wy = vy[i] - vy[j], wz = vz[i] - vz[j];
                double vdotx = wx * xx + wy * xy + wz * xz;
                double hbar = 0.5 * (hi_s + 0.5 * H[j]);
                double mu = hbar * vdotx / (r2 + p->eps_av * hbar * hbar);
                double Pi = 0.0;
                if (vdotx < 0.0) {
                    double cbar = 0.5 * (c[i] + c[j]);
                    double rbar = 0.5 * (rho[i] + rho[j]);
                    Pi = (-p->alpha * cbar * mu + p->beta * mu * mu) / rbar;
                }
                double Gbar = 0.5 * (Gi + Gj);
                double s = m[j] * (A[i] * Gi + A[j] * Gj + Pi * Gbar);
                sax -= s * xx;
                say -= s * xy;
                saz -= s * xz;
                spdv += m[j] * Gi * vdotx;
                sav += m[j] * Pi * Gbar * vdotx;
                if (-mu > mumax) mumax = -mu;
            }
            ax[k] = sax; ay[k] = say; az[k] = saz;
            const double heat = 0.5 * sav;   /* viscous heating, eq:AV_heating */
            dudt[k] = (p->flags & ORC_ENTROPY) ? heat : A[i] * spdv + heat;
            if (drho) drho[k] = spdv / omega[i];
            count[k] = cnt;
            double amag = sqrt(sax * sax + say * say + saz * saz);
            double dt = p->dt_max;
            if (amag > 0.0) {
                double ta = p->eta_a * sqrt(H[i] / amag);
                if (ta < dt) dt = ta;
            }
            double den = (1.0 + 0.6 * p->alpha) * c[i] + 0.6 * p->beta * mumax;
            if (den > 0.0) {
                double tc = p->eta_c * hi_s / den;
                if (tc < dt) dt = tc;
            }
            dti[k] = dt;
        }
        free(l.j); free(l.r2);
    }
    grid_free(&g);
    free(A);
    return 0;
}
