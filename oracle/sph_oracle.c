/*
 * sph_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow FP64 CPU evaluation of the SPH quantities defined in
 * P. Gonnet, "Efficient and Scalable Algorithms for Smoothed Particle
 * Hydrodynamics on Hybrid Shared/Distributed-Memory Architectures" (2014):
 *
 *   - the cubic-spline kernel W(r,h) of Sec. 2.1 (unnumbered equation),
 *   - the density sum, Eq. (2),
 *   - the weighted neighbour count and its h-derivative, Eq. (3), and the
 *     Newton iteration on h that keeps it at a target value,
 *   - the correction term Omega and pressure P of Sec. 2.1,
 *   - the accelerations and internal-energy rates, Eqs. (4)-(5),
 *   - the Monaghan-Balsara viscosity and Balsara switch of Sec. 4.1,
 *   - the per-particle time step of Eq. (6).
 *
 * Every sum is a one-sided gather over neighbours found by a plain periodic
 * cell list: no sorting, no symmetric updates, no blocking.  Only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark may load this
 * file; the GPU library shares no code with it.
 *
 * Neighbour search: particles are binned into uniform periodic grids at
 * several resolutions (edge L/2^k).  A query of radius R picks the finest
 * grid whose cell edge is >= R and visits the 3x3x3 block around the query
 * cell (all cells of a dimension with fewer than 3 cells).  Cells are found
 * by binary search in a key-sorted particle list.  Distances use the minimum
 * periodic image, so every query requires R < L/2 in each dimension.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_PI 3.14159265358979323846
#define ORA_MAXLEV 24

enum { ORA_OK = 0, ORA_E_ARG = 1, ORA_E_H_TOO_LARGE = 2, ORA_E_NOT_CONVERGED = 3, ORA_E_OOM = 4 };

/* ---------------------------------------------------------------------------
 * Kernel, Sec. 2.1: W(r,h) = 8/(pi h^3) w(r/h) with
 *   w(q) = 1 - 6 q^2 + 6 q^3    for 0 <= q <= 1/2,
 *          2 (1-q)^3            for 1/2 < q <= 1,
 *          0                    for q > 1.
 * ------------------------------------------------------------------------- */
double ora_w(double q)
{
    if (q < 0.0) q = -q;
    if (q <= 0.5) return 1.0 - 6.0 * q * q + 6.0 * q * q * q;
    if (q <= 1.0) { double t = 1.0 - q; return 2.0 * t * t * t; }
    return 0.0;
}

/* dw/dq */
double ora_dw(double q)
{
    if (q < 0.0) q = -q;
    if (q <= 0.5) return -12.0 * q + 18.0 * q * q;
    if (q <= 1.0) { double t = 1.0 - q; return -6.0 * t * t; }
    return 0.0;
}

/* d^2w/dq^2 */
double ora_d2w(double q)
{
    if (q < 0.0) q = -q;
    if (q <= 0.5) return -12.0 + 36.0 * q;
    if (q <= 1.0) return 12.0 * (1.0 - q);
    return 0.0;
}

double ora_W(double r, double h) { return 8.0 / (ORA_PI * h * h * h) * ora_w(r / h); }

/* dW/dr */
double ora_dWdr(double r, double h) { return 8.0 / (ORA_PI * h * h * h * h) * ora_dw(r / h); }

/* d(dW/dr)/d(ln h) at fixed r: dW/dr = 8/(pi h^4) w'(r/h) */
double ora_dWdr_dlnh(double r, double h)
{
    double q = r / h;
    return -8.0 / (ORA_PI * h * h * h * h) * (4.0 * ora_dw(q) + q * ora_d2w(q));
}

/* dW/dh at fixed r: W = 8/(pi h^3) w(r/h) */
double ora_dWdh(double r, double h)
{
    double q = r / h;
    return -8.0 / (ORA_PI * h * h * h * h) * (3.0 * ora_w(q) + q * ora_dw(q));
}

/* ---------------------------------------------------------------------------
 * Multi-resolution periodic cell list.
 * ------------------------------------------------------------------------- */
typedef struct {
    int nlev;
    int n[ORA_MAXLEV][3];
    double e[ORA_MAXLEV][3];
    uint64_t *key[ORA_MAXLEV]; /* sorted cell keys */
    int32_t *idx[ORA_MAXLEV];  /* particle index in the same order */
    double L[3];
    const double *x, *y, *z;
    int64_t np;
} ora_grid;

typedef struct { uint64_t k; int32_t i; } ora_kv;

static int kv_cmp(const void *a, const void *b)
{
    const ora_kv *p = (const ora_kv *)a, *q = (const ora_kv *)b;
    if (p->k < q->k) return -1;
    if (p->k > q->k) return 1;
    return (p->i < q->i) ? -1 : (p->i > q->i);
}

static double wrap(double v, double L)
{
    double w = fmod(v, L);
    if (w < 0.0) w += L;
    if (w >= L) w -= L;
    return w;
}

static int cell_coord(double v, double L, double e, int n)
{
    int c = (int)floor(wrap(v, L) / e);
    if (c < 0) c = 0;
    if (c >= n) c = n - 1;
    return c;
}

static void grid_free(ora_grid *g)
{
    for (int l = 0; l < g->nlev; l++) { free(g->key[l]); free(g->idx[l]); }
    g->nlev = 0;
}

/* Build levels from the coarsest (one cell per dimension... up to L/2^k) down to
 * the finest level whose edge is still >= rmin. */
static int grid_build(ora_grid *g, int64_t np, const double *x, const double *y, const double *z,
                      const double L[3], double rmin)
{
    memset(g, 0, sizeof(*g));
    g->np = np; g->x = x; g->y = y; g->z = z;
    for (int d = 0; d < 3; d++) g->L[d] = L[d];
    double Lmax = fmax(L[0], fmax(L[1], L[2]));
    if (!(rmin > 0.0)) rmin = Lmax;
    ora_kv *tmp = (ora_kv *)malloc(sizeof(ora_kv) * (size_t)(np > 0 ? np : 1));
    if (!tmp) return ORA_E_OOM;
    for (int l = 0; l < ORA_MAXLEV; l++) {
        double et = Lmax / (double)(1u << l);
        int ok = 1;
        for (int d = 0; d < 3; d++) {
            int n = (int)floor(L[d] / et);
            if (n < 1) n = 1;
            if (n > (1 << 20)) { ok = 0; break; }
            g->n[l][d] = n;
            g->e[l][d] = L[d] / n;
        }
        if (!ok) break;
        /* stop adding levels once the smallest edge drops below rmin, or once
         * the grid has many more cells than particles */
        double emin = fmin(g->e[l][0], fmin(g->e[l][1], g->e[l][2]));
        double ncell = (double)g->n[l][0] * (double)g->n[l][1] * (double)g->n[l][2];
        if (l > 0 && ncell > 8.0 * (double)np + 64.0) break;
        if (l > 0 && emin < rmin) break;
        g->key[l] = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(np > 0 ? np : 1));
        g->idx[l] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(np > 0 ? np : 1));
        if (!g->key[l] || !g->idx[l]) { g->nlev = l + 1; grid_free(g); free(tmp); return ORA_E_OOM; }
        g->nlev = l + 1;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < np; i++) {
            uint64_t cx = (uint64_t)cell_coord(x[i], L[0], g->e[l][0], g->n[l][0]);
            uint64_t cy = (uint64_t)cell_coord(y[i], L[1], g->e[l][1], g->n[l][1]);
            uint64_t cz = (uint64_t)cell_coord(z[i], L[2], g->e[l][2], g->n[l][2]);
            tmp[i].k = (cx * (uint64_t)g->n[l][1] + cy) * (uint64_t)g->n[l][2] + cz;
            tmp[i].i = (int32_t)i;
        }
        qsort(tmp, (size_t)np, sizeof(ora_kv), kv_cmp);
        for (int64_t i = 0; i < np; i++) { g->key[l][i] = tmp[i].k; g->idx[l][i] = tmp[i].i; }
        if (emin < rmin) break;
    }
    free(tmp);
    return ORA_OK;
}

static int64_t lower_bound_u64(const uint64_t *a, int64_t n, uint64_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) { int64_t mid = lo + (hi - lo) / 2; if (a[mid] < v) lo = mid + 1; else hi = mid; }
    return lo;
}

/* neighbour record: index and minimum-image separation x_i - x_j */
typedef struct { int32_t j; double dx, dy, dz, r2; } ora_nb;

typedef struct { ora_nb *v; int64_t n, cap; } ora_list;

static int list_push(ora_list *l, ora_nb nb)
{
    if (l->n == l->cap) {
        int64_t nc = l->cap ? 2 * l->cap : 256;
        ora_nb *p = (ora_nb *)realloc(l->v, sizeof(ora_nb) * (size_t)nc);
        if (!p) return ORA_E_OOM;
        l->v = p; l->cap = nc;
    }
    l->v[l->n++] = nb;
    return ORA_OK;
}

static double min_image(double d, double L) { return d - L * nearbyint(d / L); }

/* Every particle j (including i itself) with minimum-image distance r < R. */
static int grid_gather(const ora_grid *g, double xi, double yi, double zi, double R, ora_list *out)
{
    out->n = 0;
    for (int d = 0; d < 3; d++) if (!(R < 0.5 * g->L[d])) return ORA_E_H_TOO_LARGE;
    int l = 0;
    for (int k = g->nlev - 1; k >= 0; k--) {
        if (g->e[k][0] >= R && g->e[k][1] >= R && g->e[k][2] >= R) { l = k; break; }
    }
    int c[3], lo[3], cnt[3];
    double pos[3] = {xi, yi, zi};
    for (int d = 0; d < 3; d++) {
        c[d] = cell_coord(pos[d], g->L[d], g->e[l][d], g->n[l][d]);
        if (g->n[l][d] >= 3) { lo[d] = c[d] - 1; cnt[d] = 3; } else { lo[d] = 0; cnt[d] = g->n[l][d]; }
    }
    double R2 = R * R;
    for (int a = 0; a < cnt[0]; a++) {
        int cx = ((lo[0] + a) % g->n[l][0] + g->n[l][0]) % g->n[l][0];
        for (int b = 0; b < cnt[1]; b++) {
            int cy = ((lo[1] + b) % g->n[l][1] + g->n[l][1]) % g->n[l][1];
            for (int cc = 0; cc < cnt[2]; cc++) {
                int cz = ((lo[2] + cc) % g->n[l][2] + g->n[l][2]) % g->n[l][2];
                uint64_t key = ((uint64_t)cx * (uint64_t)g->n[l][1] + (uint64_t)cy) * (uint64_t)g->n[l][2] + (uint64_t)cz;
                int64_t s = lower_bound_u64(g->key[l], g->np, key);
                for (int64_t t = s; t < g->np && g->key[l][t] == key; t++) {
                    int32_t j = g->idx[l][t];
                    double dx = min_image(xi - g->x[j], g->L[0]);
                    double dy = min_image(yi - g->y[j], g->L[1]);
                    double dz = min_image(zi - g->z[j], g->L[2]);
                    double r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 < R2) {
                        ora_nb nb = {j, dx, dy, dz, r2};
                        if (list_push(out, nb)) return ORA_E_OOM;
                    }
                }
            }
        }
    }
    return ORA_OK;
}

/* selection helper: sel == NULL means all particles */
static inline int64_t sel_index(const int64_t *sel, int64_t k) { return sel ? sel[k] : k; }

/* relative width of the band around the support radius inside which a pair
 * may legitimately be classified either way (rounding of r and h). */
#define ORA_BAND 1e-6

/* ---------------------------------------------------------------------------
 * Weighted neighbour count of Eq. (3) and its h-derivative, for one particle,
 * from a cached neighbour list (which must hold every j with r < h).
 *   N(h)     = 4/3 pi h^3 sum_j W(r_ij, h) = 32/3 sum_j w(r_ij/h)
 *   dN/dh    = -(32/3) (1/h) sum_j q w'(q)
 * ------------------------------------------------------------------------- */
static void count_and_derivative(const ora_list *l, double h, double *N, double *dN)
{
    double s = 0.0, sd = 0.0;
    for (int64_t k = 0; k < l->n; k++) {
        double r = sqrt(l->v[k].r2);
        if (r < h) {
            double q = r / h;
            s += ora_w(q);
            sd += q * ora_dw(q);
        }
    }
    *N = 32.0 / 3.0 * s;
    *dN = -32.0 / 3.0 / h * sd;
}

/*
 * Solve N_i(h_i) = target for the selected particles (Sec. 2.1, Eq. (3):
 * Newton iteration using dN/dh).  N_i(h) is non-decreasing in h and equals
 * 32/3 (self term only) for small h, so the root is unique; the Newton step is
 * safeguarded by a bracket [lo, hi] with bisection (or doubling while no upper
 * bound is known) whenever the step leaves the bracket.
 *
 * h_inout: on entry the initial guesses of all particles, on exit the solved
 * values of the selected ones.  iters_out (optional): Newton evaluations used,
 * -1 if not converged within maxit.
 */
int ora_solve_h(int64_t np, const double *x, const double *y, const double *z,
                const double L[3], double target, double tol, int maxit,
                int64_t nsel, const int64_t *sel, double *h_inout, int32_t *iters_out)
{
    if (np <= 0 || !x || !y || !z || !h_inout || !(target > 32.0 / 3.0)) return ORA_E_ARG;
    double hmin = INFINITY;
    for (int64_t k = 0; k < nsel; k++) { double hh = h_inout[sel_index(sel, k)]; if (!(hh > 0.0)) return ORA_E_ARG; if (hh < hmin) hmin = hh; }
    ora_grid g;
    int st = grid_build(&g, np, x, y, z, L, hmin / 16.0);
    if (st) return st;
    double Lmin = fmin(L[0], fmin(L[1], L[2]));
    int status = ORA_OK;
#pragma omp parallel
    {
        ora_list l = {0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < nsel; k++) {
            int64_t i = sel_index(sel, k);
            double h = h_inout[i], lo = 0.0, hi = INFINITY, R = 0.0;
            int it, done = 0, err = 0;
            for (it = 1; it <= maxit; it++) {
                if (h >= R) {
                    R = fmin(1.5 * h, 0.4999 * Lmin);
                    if (!(h < R)) { err = ORA_E_H_TOO_LARGE; break; }
                    if (grid_gather(&g, x[i], y[i], z[i], R, &l)) { err = ORA_E_OOM; break; }
                }
                double N, dN;
                count_and_derivative(&l, h, &N, &dN);
                double f = N - target;
                if (fabs(f) <= tol) { done = 1; break; }
                if (f < 0.0) lo = h; else hi = h;
                double hn = h - f / dN;
                int ok = (dN > 0.0) && (hn > lo) && (hn < hi) && (hn >= 0.5 * h) && (hn <= 2.0 * h);
                if (!ok) hn = isinf(hi) ? 2.0 * h : 0.5 * (lo + hi);
                h = hn;
            }
            h_inout[i] = h;
            if (iters_out) iters_out[i] = done ? it : -1;
            if (err || !done) {
#pragma omp critical
                { if (status == ORA_OK) status = err ? err : ORA_E_NOT_CONVERGED; }
            }
        }
        free(l.v);
    }
    grid_free(&g);
    return status;
}

/*
 * Density-stage sums at given smoothing lengths, for the selected particles.
 * Range is one-sided, r_ij < h_i, and includes j = i (Eq. (2)).
 *   rho_i    = sum_j m_j W(r_ij, h_i)                                   Eq. (2)
 *   N_i      = 4/3 pi h_i^3 sum_j W(r_ij, h_i)                           Eq. (3)
 *   dN_i     = dN_i/dh_i
 *   drho_i   = sum_j m_j dW(r_ij,h_i)/dh_i   (so Omega_i = 1 + h_i/(3 rho_i) drho_i)
 *   div_i    = 1/rho_i sum_j m_j (v_j - v_i) . grad W(r_ij, h_i)        Sec. 4.1
 *   curl_i   = -1/rho_i sum_j m_j (v_j - v_i) x grad W(r_ij, h_i)       Sec. 4.1
 * grad W(r_ij,h) is the gradient with respect to r_ij = x_i - x_j:
 *   grad W = dW/dr * r_ij / r (zero at r = 0).
 * count_i: neighbours j != i with r < h_i; band_i: pairs with |r/h_i - 1| < 1e-6.
 */
int ora_density(int64_t np, const double *x, const double *y, const double *z,
                const double *vx, const double *vy, const double *vz, const double *m,
                const double *h, const double L[3], int64_t nsel, const int64_t *sel,
                double *rho, double *nngb, double *dndh, double *drhodh,
                double *div, double *curl /* 3 per particle */, int32_t *count, int32_t *band)
{
    if (np <= 0 || !x || !h || !m) return ORA_E_ARG;
    double hmin = INFINITY;
    for (int64_t k = 0; k < nsel; k++) { double hh = h[sel_index(sel, k)]; if (!(hh > 0.0)) return ORA_E_ARG; if (hh < hmin) hmin = hh; }
    ora_grid g;
    int st = grid_build(&g, np, x, y, z, L, hmin);
    if (st) return st;
    int status = ORA_OK;
#pragma omp parallel
    {
        ora_list l = {0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < nsel; k++) {
            int64_t i = sel_index(sel, k);
            double hi = h[i];
            int e = grid_gather(&g, x[i], y[i], z[i], hi * (1.0 + 2.0 * ORA_BAND), &l);
            if (e) {
#pragma omp critical
                { if (status == ORA_OK) status = e; }
                continue;
            }
            double srho = 0, sw = 0, sqdw = 0, sdrho = 0, sdiv = 0, scx = 0, scy = 0, scz = 0;
            int32_t c = 0, b = 0;
            for (int64_t t = 0; t < l.n; t++) {
                ora_nb nb = l.v[t];
                double r = sqrt(nb.r2);
                if (fabs(r / hi - 1.0) < ORA_BAND) b++;
                if (!(r < hi)) continue;
                int64_t j = nb.j;
                double q = r / hi;
                double w = ora_w(q), dw = ora_dw(q);
                srho += m[j] * ora_W(r, hi);
                sw += w;
                sqdw += q * dw;
                sdrho += m[j] * ora_dWdh(r, hi);
                if (j != i) {
                    c++;
                    if (r > 0.0 && vx) {
                        double g1 = ora_dWdr(r, hi) / r; /* grad W = g1 * r_ij */
                        double gx = g1 * nb.dx, gy = g1 * nb.dy, gz = g1 * nb.dz;
                        double dvx = vx[j] - vx[i], dvy = vy[j] - vy[i], dvz = vz[j] - vz[i];
                        sdiv += m[j] * (dvx * gx + dvy * gy + dvz * gz);
                        scx += m[j] * (dvy * gz - dvz * gy);
                        scy += m[j] * (dvz * gx - dvx * gz);
                        scz += m[j] * (dvx * gy - dvy * gx);
                    }
                }
            }
            if (rho) rho[i] = srho;
            if (nngb) nngb[i] = 32.0 / 3.0 * sw;
            if (dndh) dndh[i] = -32.0 / 3.0 / hi * sqdw;
            if (drhodh) drhodh[i] = sdrho;
            if (div) div[i] = sdiv / srho;
            if (curl) { curl[3 * i + 0] = -scx / srho; curl[3 * i + 1] = -scy / srho; curl[3 * i + 2] = -scz / srho; }
            if (count) count[i] = c;
            if (band) band[i] = b;
        }
        free(l.v);
    }
    grid_free(&g);
    return status;
}

/*
 * Per-particle quantities between the two stages (the "ghost" of Sec. 3.4):
 *   Omega_i = 1 + h_i/(3 rho_i) drho_i/dh_i                             Sec. 2.1
 *   P_i     = (gamma-1) rho_i u_i                                        Sec. 2.1
 *   c_i     = sqrt(gamma P_i / rho_i)            (speed of sound; the paper uses it
 *                                                 without defining it)
 *   A_i     = P_i / (Omega_i rho_i^2)            (the factor in Eqs. (4)-(5))
 *   f_i     = |curl v_i| / (|div v_i| + |curl v_i| + 1e-4 c_i/h_i)       Sec. 4.1
 * f_i = 0 where its denominator vanishes.
 */
void ora_ghost(int64_t n, const double *rho, const double *drhodh, const double *h, const double *u,
               const double *div, const double *curl, double gamma, int form,
               double *omega, double *P, double *c, double *A, double *f)
{
    for (int64_t i = 0; i < n; i++) {
        double om = 1.0 + h[i] / (3.0 * rho[i]) * drhodh[i];
        double p = (gamma - 1.0) * rho[i] * u[i];
        double cs = sqrt(gamma * p / rho[i]);
        double a = p / (om * rho[i] * rho[i]);
        double cm = sqrt(curl[3 * i] * curl[3 * i] + curl[3 * i + 1] * curl[3 * i + 1] + curl[3 * i + 2] * curl[3 * i + 2]);
        double den = fabs(div[i]) + cm + 1e-4 * cs / h[i];
        /* form 0: |curl| on top, as Sec. 4.1 prints it; form 1: |div| on top,
         * the switch of Balsara (1995) that Sec. 4.1 cites */
        double num = form == 1 ? fabs(div[i]) : cm;
        omega[i] = om; P[i] = p; c[i] = cs; A[i] = a;
        f[i] = den > 0.0 ? num / den : 0.0;
    }
}

/*
 * Signal speed of the time-step criterion, Eq. (6):
 *   vsig_i = max_j (c_i + c_j + max(0, -3 v_ij . r_ij / r_ij)),
 *   dt_i   = C_CFL 2 h_i / vsig_i,
 * j running over the particles that interact with i in the force stage
 * (r_ij < max(h_i, h_j)) and over i itself, whose term is 2 c_i (r_ii = 0, no
 * approach speed).  vsig_lo and vsig_hi take the same maximum over the pairs
 * with r_ij < (1 - band) max(h_i, h_j) and r_ij < (1 + band) max(h_i, h_j):
 * a pair at the edge of the support may fall on either side in a lower
 * precision.  dt_i is +inf where vsig_i = 0.
 */
int ora_signal(int64_t np, const double *x, const double *y, const double *z,
               const double *vx, const double *vy, const double *vz, const double *h,
               const double *c, const double L[3], double cfl, int64_t nsel, const int64_t *sel,
               double *vsig, double *vsig_lo, double *vsig_hi, double *dt)
{
    if (np <= 0 || !x || !h || !c) return ORA_E_ARG;
    double hmax = 0.0, hmin = INFINITY;
    for (int64_t i = 0; i < np; i++) { if (h[i] > hmax) hmax = h[i]; if (h[i] < hmin) hmin = h[i]; }
    ora_grid g;
    int st = grid_build(&g, np, x, y, z, L, hmin);
    if (st) return st;
    int status = ORA_OK;
#pragma omp parallel
    {
        ora_list l = {0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < nsel; k++) {
            int64_t i = sel_index(sel, k);
            double R = fmax(h[i], hmax) * (1.0 + 2.0 * ORA_BAND);
            int e = grid_gather(&g, x[i], y[i], z[i], R, &l);
            if (e) {
#pragma omp critical
                { if (status == ORA_OK) status = e; }
                continue;
            }
            double s = 2.0 * c[i], slo = s, shi = s;
            for (int64_t t = 0; t < l.n; t++) {
                ora_nb nb = l.v[t];
                int64_t j = nb.j;
                if (j == i) continue;
                double r = sqrt(nb.r2);
                double hij = fmax(h[i], h[j]);
                if (!(r < hij * (1.0 + ORA_BAND))) continue;
                double vdotr = (vx[i] - vx[j]) * nb.dx + (vy[i] - vy[j]) * nb.dy + (vz[i] - vz[j]) * nb.dz;
                double approach = (r > 0.0) ? fmax(0.0, -3.0 * vdotr / r) : 0.0;
                double v = c[i] + c[j] + approach;
                if (v > shi) shi = v;
                if (r < hij && v > s) s = v;
                if (r < hij * (1.0 - ORA_BAND) && v > slo) slo = v;
            }
            if (vsig) vsig[i] = s;
            if (vsig_lo) vsig_lo[i] = slo;
            if (vsig_hi) vsig_hi[i] = shi;
            if (dt) dt[i] = s > 0.0 ? cfl * 2.0 * h[i] / s : INFINITY;
        }
        free(l.v);
    }
    grid_free(&g);
    return status;
}

/*
 * Force-stage sums, Eqs. (4)-(5) plus the viscosity terms of Sec. 4.1, for the
 * selected particles; range r_ij < max(h_i, h_j), j != i:
 *   Pi_ij = -alpha (c_i + c_j - 3 w_ij) w_ij / (rho_i + rho_j),
 *   w_ij  = min(0, v_ij . r_ij / r_ij),  v_ij = v_i - v_j,  r_ij = x_i - x_j,
 *   a_i   = - sum_j m_j [A_i gW_i + A_j gW_j]
 *           - 1/4 sum_j m_j Pi_ij (gW_i + gW_j) (f_i + f_j),
 *   du_i  =   A_i sum_j m_j v_ij . gW_i
 *           + 1/8 sum_j m_j Pi_ij v_ij . (gW_i + gW_j) (f_i + f_j),
 * where gW_i = grad W(r_ij, h_i), gW_j = grad W(r_ij, h_j).  The pressure part
 * of du only has support r < h_i, which the kernel gradient enforces.
 * kappa_a / kappa_u: sum over j of the magnitudes of the individual pair
 * contributions (a scale for the cancellation in a_i and du_i).
 * sens_a / sens_u: sum over j of the magnitudes of the derivatives of each
 * pair contribution with respect to ln h_i and to ln h_j, rho, A, c and f
 * held fixed (how far a relative change of the smoothing lengths moves the
 * sums; near the edge of the support w' vanishes like (1-q)^2, so a term there
 * moves by up to 2q/(1-q) times that change).  Either may be NULL.
 */
int ora_force(int64_t np, const double *x, const double *y, const double *z,
              const double *vx, const double *vy, const double *vz, const double *m,
              const double *h, const double *rho, const double *A, const double *c,
              const double *f, const double L[3], double alpha, int64_t nsel, const int64_t *sel,
              double *ax, double *ay, double *az, double *dudt,
              double *kappa_a, double *kappa_u, int32_t *count, int32_t *band,
              double *sens_a, double *sens_u)
{
    if (np <= 0 || !x || !h || !m || !rho || !A || !c || !f) return ORA_E_ARG;
    double hmax = 0.0, hmin = INFINITY;
    for (int64_t i = 0; i < np; i++) { if (h[i] > hmax) hmax = h[i]; if (h[i] < hmin) hmin = h[i]; }
    ora_grid g;
    int st = grid_build(&g, np, x, y, z, L, hmin);
    if (st) return st;
    int status = ORA_OK;
#pragma omp parallel
    {
        ora_list l = {0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < nsel; k++) {
            int64_t i = sel_index(sel, k);
            double R = fmax(h[i], hmax) * (1.0 + 2.0 * ORA_BAND);
            int e = grid_gather(&g, x[i], y[i], z[i], R, &l);
            if (e) {
#pragma omp critical
                { if (status == ORA_OK) status = e; }
                continue;
            }
            double sax = 0, say = 0, saz = 0, sdu = 0, ka = 0, ku = 0, sa = 0, su = 0;
            int32_t cnt = 0, b = 0;
            for (int64_t t = 0; t < l.n; t++) {
                ora_nb nb = l.v[t];
                int64_t j = nb.j;
                if (j == i) continue;
                double r = sqrt(nb.r2);
                double hij = fmax(h[i], h[j]);
                if (fabs(r / hij - 1.0) < ORA_BAND) b++;
                if (!(r < hij)) continue;
                cnt++;
                /* grad W(r, h) = dW/dr * r_vec / r; zero for coincident particles */
                double gi = (r > 0.0) ? ora_dWdr(r, h[i]) / r : 0.0;
                double gj = (r > 0.0) ? ora_dWdr(r, h[j]) / r : 0.0;
                double vxij = vx[i] - vx[j], vyij = vy[i] - vy[j], vzij = vz[i] - vz[j];
                double vdotr = vxij * nb.dx + vyij * nb.dy + vzij * nb.dz;
                double wij = (r > 0.0) ? fmin(0.0, vdotr / r) : 0.0;
                double Pi = -alpha * (c[i] + c[j] - 3.0 * wij) * wij / (rho[i] + rho[j]);
                double fij = f[i] + f[j];
                /* acceleration: scalar multiple of r_vec */
                double s = -m[j] * (A[i] * gi + A[j] * gj) - 0.25 * m[j] * Pi * (gi + gj) * fij;
                double pax = s * nb.dx, pay = s * nb.dy, paz = s * nb.dz;
                double pdu = A[i] * m[j] * vdotr * gi + 0.125 * m[j] * Pi * vdotr * (gi + gj) * fij;
                sax += pax; say += pay; saz += paz; sdu += pdu;
                ka += sqrt(pax * pax + pay * pay + paz * paz);
                ku += fabs(pdu);
                /* derivatives of gi, gj with respect to ln h_i, ln h_j */
                double di = (r > 0.0) ? ora_dWdr_dlnh(r, h[i]) / r : 0.0;
                double dj = (r > 0.0) ? ora_dWdr_dlnh(r, h[j]) / r : 0.0;
                sa += (fabs(m[j] * di * (A[i] + 0.25 * Pi * fij)) + fabs(m[j] * dj * (A[j] + 0.25 * Pi * fij))) * r;
                su += fabs(m[j] * vdotr * di * (A[i] + 0.125 * Pi * fij)) + fabs(0.125 * m[j] * Pi * vdotr * dj * fij);
            }
            ax[i] = sax; ay[i] = say; az[i] = saz; dudt[i] = sdu;
            if (kappa_a) kappa_a[i] = ka;
            if (kappa_u) kappa_u[i] = ku;
            if (sens_a) sens_a[i] = sa;
            if (sens_u) sens_u[i] = su;
            if (count) count[i] = cnt;
            if (band) band[i] = b;
        }
        free(l.v);
    }
    grid_free(&g);
    return status;
}

/*
 * Pairs that a smoothing length known only to a relative precision b may
 * classify either way.  With b_i the relative precision of h_i:
 *   dband_i: pairs j != i with |r_ij / h_i - 1| < b_i           (density range)
 *   fband_i: pairs j != i with |r_ij / max(h_i, h_j) - 1| < b_ij, b_ij the b
 *            of whichever of i, j has the larger h                (force range)
 * Only counts; no SPH arithmetic.  Either output may be NULL.
 */
int ora_bands(int64_t np, const double *x, const double *y, const double *z, const double *h,
              const double *bw, const double L[3], int64_t nsel, const int64_t *sel,
              int32_t *dband, int32_t *fband)
{
    if (np <= 0 || !x || !h || !bw) return ORA_E_ARG;
    double hmax = 0.0, hmin = INFINITY, bmax = 0.0;
    for (int64_t i = 0; i < np; i++) {
        if (h[i] > hmax) hmax = h[i];
        if (h[i] < hmin) hmin = h[i];
        if (bw[i] > bmax) bmax = bw[i];
    }
    ora_grid g;
    int st = grid_build(&g, np, x, y, z, L, hmin);
    if (st) return st;
    int status = ORA_OK;
#pragma omp parallel
    {
        ora_list l = {0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < nsel; k++) {
            int64_t i = sel_index(sel, k);
            int e = grid_gather(&g, x[i], y[i], z[i], fmax(h[i], hmax) * (1.0 + 2.0 * bmax), &l);
            if (e) {
#pragma omp critical
                { if (status == ORA_OK) status = e; }
                continue;
            }
            int32_t db = 0, fb = 0;
            for (int64_t t = 0; t < l.n; t++) {
                int64_t j = l.v[t].j;
                if (j == i) continue;
                double r = sqrt(l.v[t].r2);
                if (fabs(r / h[i] - 1.0) < bw[i]) db++;
                double hij = fmax(h[i], h[j]);
                double bij = h[i] >= h[j] ? bw[i] : bw[j];
                if (fabs(r / hij - 1.0) < bij) fb++;
            }
            if (dband) dband[i] = db;
            if (fband) fband[i] = fb;
        }
        free(l.v);
    }
    grid_free(&g);
    return status;
}

int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loops that follow (n >= 1). */
void ora_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
