/*
 * spic_oracle.c -- plain FP64 CPU oracle for the implicit particle mover and
 * the particle-to-grid moment gathering of the implicit PIC method
 * (sputniPIC, arXiv 2008.04397, Sec. II).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file: only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code, header, table or helper with the GPU
 * library; the two only consume the same seeded inputs.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no FMA
 * contraction, so every operation rounds once, in the order written).
 *
 * What it computes (readings of the paper are listed with each function):
 *   - linear weight function W (Sec. II, Eq. 3) read as the tensor product
 *     of 1-D hat functions with one spacing per axis (trilinear weights);
 *   - field gather E_p = sum_g E_g W, B_p = sum_g B_g W (Sec. II, Eq. 4);
 *   - implicit predictor-corrector for the mean velocity (Sec. II, Eq. 1
 *     and Eq. 2) with a fixed number of iterations (three in the paper),
 *     the fields being re-gathered at the current half-step position
 *     estimate on every iteration;
 *   - the update v^{n+1} = 2 vbar - v^n, x^{n+1} = x^n + vbar dt
 *     (Sec. II, Eq. 5), with periodic wrap into [0, L);
 *   - the ten moments {rho, J, P} = sum_p q {1, v, v (x) v} W
 *     (Sec. II, moment equation) deposited with the new state, once every
 *     particle has moved (Sec. III-B: mover and gathering fused, new
 *     position used for the gathering).
 *
 * Grid convention: periodic box [0,Lx)x[0,Ly)x[0,Lz), n_d cells and n_d
 * distinct nodes per axis at i*L_d/n_d, node (i,j,k) at flat index
 * (i*ny + j)*nz + k.  Moments are stored [10][nodes] in the order
 * rho, Jx, Jy, Jz, Pxx, Pxy, Pxz, Pyy, Pyz, Pzz, with no volume factor.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t nx, ny, nz, pad;
    double Lx, Ly, Lz;
} og_grid;

/* ---- periodic wrap and 1-D location ---------------------------------- */

/* Wrap s into [0, L).  Rounding can make s - L*floor(s/L) equal L (or a
 * negative zero-ish value); both are mapped to 0, the same point of the
 * periodic box. */
static double og_wrap(double s, double L)
{
    double r = s - L * floor(s / L);
    if (r >= L) r = 0.0;
    if (r < 0.0) r = 0.0;
    return r;
}

/* Left node index and the fractional offset inside the cell along one
 * axis.  The hat function of Eq. 3 is non-zero on the two nodes that bound
 * the cell; their weights are (1 - xi) and xi. */
static void og_locate(double s, double L, int n, int *i0, int *i1, double *w0, double *w1)
{
    double d = L / (double)n;
    double t = og_wrap(s, L) / d;
    int i = (int)floor(t);
    if (i > n - 1) i = n - 1;
    if (i < 0) i = 0;
    double xi = t - (double)i;
    *i0 = i;
    *i1 = (i + 1) % n;
    *w0 = 1.0 - xi;
    *w1 = xi;
}

/* The 8 nodes and trilinear weights of a point (Eq. 3, tensor-product
 * reading).  Corner c = a + 2b + 4c' picks axis offsets (a, b, c'). */
static void og_weights8(const og_grid *g, double x, double y, double z,
                        int64_t node[8], double wgt[8])
{
    int ix[2], iy[2], iz[2];
    double wx[2], wy[2], wz[2];
    og_locate(x, g->Lx, g->nx, &ix[0], &ix[1], &wx[0], &wx[1]);
    og_locate(y, g->Ly, g->ny, &iy[0], &iy[1], &wy[0], &wy[1]);
    og_locate(z, g->Lz, g->nz, &iz[0], &iz[1], &wz[0], &wz[1]);
    for (int c = 0; c < 8; ++c) {
        int a = c & 1, b = (c >> 1) & 1, cc = (c >> 2) & 1;
        node[c] = ((int64_t)ix[a] * g->ny + iy[b]) * g->nz + iz[cc];
        wgt[c] = wx[a] * wy[b] * wz[cc];
    }
}

/* Eq. 4: F_p = sum over the 8 non-zero nodes of F_g W. */
static void og_gather6(const og_grid *g, const double *const f[6],
                       double x, double y, double z, double out[6])
{
    int64_t node[8];
    double wgt[8];
    og_weights8(g, x, y, z, node, wgt);
    for (int m = 0; m < 6; ++m) {
        double acc = 0.0;
        for (int c = 0; c < 8; ++c) acc += f[m][node[c]] * wgt[c];
        out[m] = acc;
    }
}

/* ---- exported helpers for pinning tests ------------------------------ */

int oracle_weights(const og_grid *g, double x, double y, double z, int64_t *node8, double *w8)
{
    og_weights8(g, x, y, z, node8, w8);
    return 0;
}

int oracle_gather(const og_grid *g, const double *ex, const double *ey, const double *ez,
                  const double *bx, const double *by, const double *bz,
                  const double *px, const double *py, const double *pz, int64_t n,
                  double *out /* [6][n] */)
{
    const double *f[6] = {ex, ey, ez, bx, by, bz};
    for (int64_t p = 0; p < n; ++p) {
        double o[6];
        og_gather6(g, f, px[p], py[p], pz[p], o);
        for (int m = 0; m < 6; ++m) out[(int64_t)m * n + p] = o[m];
    }
    return 0;
}

/* ---- the mover -------------------------------------------------------- */

/* One implicit step of one particle (Sec. II).
 *   beta = q dt / (2 m)                          (factor of Eq. 1)
 *   repeat niter times, starting from xbar = x^n:
 *     E, B   = gather at xbar                    (Eq. 4)
 *     vt     = v^n + beta E                      (Eq. 1)
 *     bv     = (beta / c) B                      (the q dt / (2 m c) B of Eq. 2)
 *     vbar   = (vt + vt x bv + (vt . bv) bv) / (1 + bv . bv)      (Eq. 2)
 *     xbar   = x^n + vbar dt / 2                 (half-step position estimate)
 *   v^{n+1} = 2 vbar - v^n, x^{n+1} = x^n + vbar dt, wrapped     (Eq. 5)
 *
 * Sec. II also allows the iteration count to be set by a prescribed error
 * tolerance instead of being fixed.  With tol > 0, niter is the cap and the
 * iteration stops after the k-th pass (k >= 2) once the change of the mean
 * velocity over that pass, max_d |vbar^k_d - vbar^(k-1)_d|, is below tol
 * (an absolute tolerance in velocity units; the paper gives no criterion,
 * this is the reading used by the library too).  tol = 0 never stops early:
 * the fixed count.  Returns the number of passes made.
 */
static int og_move1(const og_grid *g, const double *const f[6], double dt, double c,
                    int niter, double tol, double qom, double *px, double *py, double *pz,
                    double *pu, double *pv, double *pw)
{
    const double x0 = *px, y0 = *py, z0 = *pz;
    const double u0 = *pu, v0 = *pv, w0 = *pw;
    const double beta = qom * dt / 2.0;
    double xb = x0, yb = y0, zb = z0;
    double ub = u0, vb = v0, wb = w0;
    int it = 0;
    while (it < niter) {
        const double pu_ = ub, pv_ = vb, pw_ = wb;
        double F[6];
        og_gather6(g, f, xb, yb, zb, F);
        double ut = u0 + beta * F[0];
        double vt = v0 + beta * F[1];
        double wt = w0 + beta * F[2];
        double bxv = beta / c * F[3];
        double byv = beta / c * F[4];
        double bzv = beta / c * F[5];
        double bb = bxv * bxv + byv * byv + bzv * bzv;
        double vdotb = ut * bxv + vt * byv + wt * bzv;
        double cx = vt * bzv - wt * byv;   /* vt x bv */
        double cy = wt * bxv - ut * bzv;
        double cz = ut * byv - vt * bxv;
        double den = 1.0 + bb;
        ub = (ut + cx + vdotb * bxv) / den;
        vb = (vt + cy + vdotb * byv) / den;
        wb = (wt + cz + vdotb * bzv) / den;
        xb = x0 + ub * dt / 2.0;
        yb = y0 + vb * dt / 2.0;
        zb = z0 + wb * dt / 2.0;
        ++it;
        if (it >= 2 && tol > 0.0) {
            double d = fabs(ub - pu_);
            if (fabs(vb - pv_) > d) d = fabs(vb - pv_);
            if (fabs(wb - pw_) > d) d = fabs(wb - pw_);
            if (d < tol) break;
        }
    }
    *pu = 2.0 * ub - u0;
    *pv = 2.0 * vb - v0;
    *pw = 2.0 * wb - w0;
    *px = og_wrap(x0 + ub * dt, g->Lx);
    *py = og_wrap(y0 + vb * dt, g->Ly);
    *pz = og_wrap(z0 + wb * dt, g->Lz);
    return it;
}

int oracle_mover(const og_grid *g, double dt, double c, int niter, double qom,
                 const double *ex, const double *ey, const double *ez,
                 const double *bx, const double *by, const double *bz,
                 double *x, double *y, double *z, double *u, double *v, double *w,
                 int64_t n)
{
    if (!g || n < 0 || niter < 0 || g->nx < 1 || g->ny < 1 || g->nz < 1) return -1;
    const double *f[6] = {ex, ey, ez, bx, by, bz};
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p)
        (void)og_move1(g, f, dt, c, niter, 0.0, qom, &x[p], &y[p], &z[p], &u[p], &v[p], &w[p]);
    return 0;
}

/* The mover with the tolerance-terminated iteration (tol > 0: niter is the
 * cap); iters[p] (may be NULL) receives the passes particle p made. */
int oracle_mover_tol(const og_grid *g, double dt, double c, int niter, double tol, double qom,
                     const double *ex, const double *ey, const double *ez,
                     const double *bx, const double *by, const double *bz,
                     double *x, double *y, double *z, double *u, double *v, double *w,
                     int64_t n, int32_t *iters)
{
    if (!g || n < 0 || niter < 0 || !(tol >= 0.0) || g->nx < 1 || g->ny < 1 || g->nz < 1) return -1;
    const double *f[6] = {ex, ey, ez, bx, by, bz};
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        int k = og_move1(g, f, dt, c, niter, tol, qom, &x[p], &y[p], &z[p], &u[p], &v[p], &w[p]);
        if (iters) iters[p] = k;
    }
    return 0;
}

/* ---- the moment gathering -------------------------------------------- */

/* Deposit of one particle: for each of the 8 nodes g with weight W,
 * m[k][g] += q W {1, u, v, w, uu, uv, uw, vv, vw, ww}[k]. */
static void og_deposit1(const og_grid *g, int64_t nn, double *m, double x, double y, double z,
                        double u, double v, double w, double q)
{
    int64_t node[8];
    double wgt[8];
    og_weights8(g, x, y, z, node, wgt);
    const double val[10] = {1.0, u, v, w, u * u, u * v, u * w, v * v, v * w, w * w};
    for (int cn = 0; cn < 8; ++cn) {
        double qw = q * wgt[cn];
        for (int k = 0; k < 10; ++k) m[(int64_t)k * nn + node[cn]] += qw * val[k];
    }
}

/* Moments of n particles into mom[10][nodes]; overwrite unless accumulate.
 * Each thread sums its static block of particles, in particle order, into a
 * private grid; the private grids are then added in thread order, node by
 * node. */
int oracle_deposit(const og_grid *g, const double *x, const double *y, const double *z,
                   const double *u, const double *v, const double *w, const double *q,
                   int64_t n, double *mom, int accumulate)
{
    if (!g || n < 0 || !mom) return -1;
    const int64_t nn = (int64_t)g->nx * g->ny * g->nz;
    if (!accumulate) memset(mom, 0, sizeof(double) * 10 * (size_t)nn);
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    if ((int64_t)nt > n / 4096 + 1) nt = (int)(n / 4096 + 1);
    double *priv = (double *)calloc((size_t)nt * 10 * (size_t)nn, sizeof(double));
    if (!priv) return -2;
#pragma omp parallel num_threads(nt)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
        double *m = priv + (size_t)t * 10 * (size_t)nn;
        for (int64_t p = lo; p < hi; ++p)
            og_deposit1(g, nn, m, x[p], y[p], z[p], u[p], v[p], w[p], q[p]);
    }
    /* node by node, the threads' grids in thread order (the same additions,
     * in the same order, as adding whole grids one after the other) */
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int64_t i = 0; i < 10 * nn; ++i) {
        double acc = mom[i];
        for (int t = 0; t < nt; ++t) acc += priv[(size_t)t * 10 * (size_t)nn + (size_t)i];
        mom[i] = acc;
    }
    free(priv);
    return 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads the oracle's parallel loops use from now on (>= 1); returns the
 * count in effect.  Lets the CPU timing run on one core and on all. */
int oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
