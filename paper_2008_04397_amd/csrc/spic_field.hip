// spic_field.hip -- the implicit field solve that closes the cycle (Sec. II,
// step 3: a linear system from the implicit-in-time discretisation of
// Maxwell's equations solved with GMRes, and a Poisson equation solved with
// CG each cycle -- divergence cleaning -- so that the continuity equation
// holds; Sec. VI names the solver's residual as the next GPU port).
//
// Discretisation (the paper prints none; this is the reading documented in
// include/spic.h): the periodic node grid of the particle step, central
// differences D_d f = (f(+e_d) - f(-e_d)) / (2 dx_d), curl/div/grad built
// from them, and the Poisson operator div grad (a radius-2 stencil), so a
// gradient correction moves the discrete divergence by exactly the Poisson
// right-hand side.  Vectors are [3][nodes] FP64 arrays.
//
// Kernels: stencils (susceptibility and implicit current from the moments,
// the right-hand side, the field operator, the Poisson operator, gradient
// and update), and deterministic two-stage reductions for the dot products
// of classical Gram-Schmidt (applied twice) and CG.  The host drives GMRes
// and CG: one device-to-host copy of a few scalars per iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "spic_ctx.h"
#include "spic_impl.h"

namespace spic {
namespace field {

constexpr int kMaxSpecies = 16;
constexpr int kMaxRestart = 64;
constexpr int kBlock = 256;
constexpr int kRedBlocks = 1024;  // partial sums per reduction

struct Geo {
    int nx, ny, nz;
    double ih[3];  // 1 / (2 dx_d)
};

// moments and charge-to-mass ratios of the species (read only)
struct Species {
    const double *m[kMaxSpecies];
    double qom[kMaxSpecies];
    int n;
};

// a + d wrapped into [0, n) for |d| <= 2 <= n (the grid has at least two
// nodes per axis): one conditional add or subtract, no division
__device__ __forceinline__ int wrapi(int a, int n) {
    a += a < 0 ? n : 0;
    a -= a >= n ? n : 0;
    return a;
}

// flat index of node (i + di, j + dj, k + dk), periodic
__device__ __forceinline__ int64_t nb(const Geo &g, int i, int j, int k, int di, int dj, int dk) {
    return ((int64_t)wrapi(i + di, g.nx) * g.ny + wrapi(j + dj, g.ny)) * g.nz + wrapi(k + dk, g.nz);
}

// D_axis f at (i, j, k)
__device__ __forceinline__ double dif(const Geo &g, const double *f, int i, int j, int k, int axis) {
    const int di = axis == 0, dj = axis == 1, dk = axis == 2;
    return (f[nb(g, i, j, k, di, dj, dk)] - f[nb(g, i, j, k, -di, -dj, -dk)]) * g.ih[axis];
}

// D_a D_b f at (i, j, k) (a == b: the radius-2 second difference)
__device__ __forceinline__ double dif2(const Geo &g, const double *f, int i, int j, int k, int a, int b) {
    const int ai = a == 0, aj = a == 1, ak = a == 2;
    const int bi = b == 0, bj = b == 1, bk = b == 2;
    const double s = f[nb(g, i, j, k, ai + bi, aj + bj, ak + bk)] - f[nb(g, i, j, k, ai - bi, aj - bj, ak - bk)] -
                     f[nb(g, i, j, k, bi - ai, bj - aj, bk - ak)] + f[nb(g, i, j, k, -ai - bi, -aj - bj, -ak - bk)];
    return s * g.ih[a] * g.ih[b];
}

__device__ __forceinline__ void node_ijk(const Geo &g, int64_t p, int &i, int &j, int &k) {
    k = (int)(p % g.nz);
    const int64_t q = p / g.nz;
    j = (int)(q % g.ny);
    i = (int)(q / g.ny);
}

// A scalar that an earlier kernel of the stream wrote (a dot product, a CG
// coefficient), read with a device-scope load: a plain uniform load goes
// through the scalar cache, which can still hold the value an earlier
// kernel read at that address when no host synchronisation came between.
__device__ __forceinline__ double dev_scalar(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// R(b): the rotation of the mover's Eq. 2 (R v solves vhat = v + vhat x b)
__device__ __forceinline__ void rotation(double bx, double by, double bz, double R[9]) {
    const double d = 1.0 / (1.0 + bx * bx + by * by + bz * bz);
    R[0] = (1.0 + bx * bx) * d; R[1] = (bz + bx * by) * d;  R[2] = (-by + bx * bz) * d;
    R[3] = (-bz + by * bx) * d; R[4] = (1.0 + by * by) * d; R[5] = (bx + by * bz) * d;
    R[6] = (by + bz * bx) * d;  R[7] = (-bx + bz * by) * d; R[8] = (1.0 + bz * bz) * d;
}

// susceptibility mu (9 arrays, row major) and, with jh, the implicit current
// Jhat = sum_s R(b_s) (J_s - dt/2 div P_s) at every node
__global__ void k_mu_jhat(Geo g, int64_t N, const double *__restrict__ B, Species sp, double dt, double c,
                          double theta, double fourpi, double *__restrict__ mu, double *__restrict__ jh) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        node_ijk(g, p, i, j, k);
        const double Bx = B[p], By = B[N + p], Bz = B[2 * N + p];
        double M[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, J[3] = {0, 0, 0};
        for (int s = 0; s < sp.n; ++s) {
            const double q = sp.qom[s], *m = sp.m[s];
            const double h = q * dt / (2.0 * c);
            double R[9];
            rotation(h * Bx, h * By, h * Bz, R);
            const double coef = 0.5 * fourpi * theta * dt * dt * q * m[p];
#pragma unroll
            for (int e = 0; e < 9; ++e) M[e] += coef * R[e];
            if (jh) {
                // P components: xx xy xz yy yz zz at moments 4..9
                const double *P[6];
#pragma unroll
                for (int e = 0; e < 6; ++e) P[e] = m + (4 + e) * N;
                const int pi[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
                double src[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    double dv = 0.0;
#pragma unroll
                    for (int b = 0; b < 3; ++b) dv += dif(g, P[pi[a][b]], i, j, k, b);
                    src[a] = m[(1 + a) * N + p] - 0.5 * dt * dv;
                }
#pragma unroll
                for (int a = 0; a < 3; ++a) J[a] += R[3 * a] * src[0] + R[3 * a + 1] * src[1] + R[3 * a + 2] * src[2];
            }
        }
#pragma unroll
        for (int e = 0; e < 9; ++e) mu[e * N + p] = M[e];
        if (jh)
#pragma unroll
            for (int a = 0; a < 3; ++a) jh[a * N + p] = J[a];
    }
}

// rhs = E + theta dt (c curl B - fourpi Jhat)
__global__ void k_rhs(Geo g, int64_t N, const double *__restrict__ E, const double *__restrict__ B,
                      const double *__restrict__ jh, double theta, double dt, double c, double fourpi,
                      double *__restrict__ rhs) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        node_ijk(g, p, i, j, k);
        const double *Bx = B, *By = B + N, *Bz = B + 2 * N;
        const double cb[3] = {dif(g, Bz, i, j, k, 1) - dif(g, By, i, j, k, 2),
                              dif(g, Bx, i, j, k, 2) - dif(g, Bz, i, j, k, 0),
                              dif(g, By, i, j, k, 0) - dif(g, Bx, i, j, k, 1)};
#pragma unroll
        for (int a = 0; a < 3; ++a) rhs[a * N + p] = E[a * N + p] + theta * dt * (c * cb[a] - fourpi * jh[a * N + p]);
    }
}

// y = (I + mu) x + acc curl curl x, with curl curl x = grad div x - div grad x
// written out per component: (curl curl x)_a = sum_{b != a} (D_a D_b x_b - D_b D_b x_a)
__global__ void k_apply(Geo g, int64_t N, const double *__restrict__ mu, const double *__restrict__ x, double acc,
                        double *__restrict__ y) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        node_ijk(g, p, i, j, k);
        const double xv[3] = {x[p], x[N + p], x[2 * N + p]};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double cc = 0.0;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                if (b == a) continue;
                cc += dif2(g, x + b * N, i, j, k, a, b) - dif2(g, x + a * N, i, j, k, b, b);
            }
            const double m = mu[(3 * a) * N + p] * xv[0] + mu[(3 * a + 1) * N + p] * xv[1] +
                             mu[(3 * a + 2) * N + p] * xv[2];
            y[a * N + p] = xv[a] + m + acc * cc;
        }
    }
}

// b = fourpi rho - div E (the right-hand side of -div grad phi = -(div E - fourpi rho))
__global__ void k_poisson_rhs(Geo g, int64_t N, const double *__restrict__ E, const double *__restrict__ rho,
                              double fourpi, double *__restrict__ b) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        node_ijk(g, p, i, j, k);
        const double dv = dif(g, E, i, j, k, 0) + dif(g, E + N, i, j, k, 1) + dif(g, E + 2 * N, i, j, k, 2);
        b[p] = fourpi * rho[p] - dv;
    }
}

// E -= grad phi
__global__ void k_sub_grad(Geo g, int64_t N, const double *__restrict__ phi, double *__restrict__ E) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        node_ijk(g, p, i, j, k);
#pragma unroll
        for (int a = 0; a < 3; ++a) E[a * N + p] -= dif(g, phi, i, j, k, a);
    }
}

// E^{n+1} = (E^theta - (1 - theta) E^n) / theta, B^{n+1} = B^n - c dt curl E^theta,
// written to the caller's six arrays
__global__ void k_update(Geo g, int64_t N, const double *__restrict__ Eth, const double *__restrict__ En,
                         const double *__restrict__ B, double theta, double c, double dt, double *ex, double *ey,
                         double *ez, double *bx, double *by, double *bz) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        node_ijk(g, p, i, j, k);
        const double *X = Eth, *Y = Eth + N, *Z = Eth + 2 * N;
        const double ce[3] = {dif(g, Z, i, j, k, 1) - dif(g, Y, i, j, k, 2),
                              dif(g, X, i, j, k, 2) - dif(g, Z, i, j, k, 0),
                              dif(g, Y, i, j, k, 0) - dif(g, X, i, j, k, 1)};
        double *Eo[3] = {ex, ey, ez}, *Bo[3] = {bx, by, bz};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            Eo[a][p] = (Eth[a * N + p] - (1.0 - theta) * En[a * N + p]) / theta;
            Bo[a][p] = B[a * N + p] - c * dt * ce[a];
        }
    }
}

// three separate arrays -> one [3][N] array
__global__ void k_pack3(int64_t N, const double *a, const double *b, const double *c3, double *out) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
        out[p] = a[p];
        out[N + p] = b[p];
        out[2 * N + p] = c3[p];
    }
}

// rho = sum over species of the moment rho
__global__ void k_rho(int64_t N, Species sp, double *__restrict__ rho) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
        double r = 0.0;
        for (int s = 0; s < sp.n; ++s) r += sp.m[s][p];
        rho[p] = r;
    }
}

// sign of null mode `mode` at node (i, j, k): bit d of the mode alternates along axis d
__device__ __forceinline__ double mode_sign(int mode, int i, int j, int k) {
    const int par = ((mode & 1) ? i : 0) + ((mode & 2) ? j : 0) + ((mode & 4) ? k : 0);
    return (par & 1) ? -1.0 : 1.0;
}

// block sums of the null-mode projections sum_p sign_mode(p) r(p), modes 0..7
__global__ void k_mode_partials(Geo g, int64_t N, const double *__restrict__ r, double *__restrict__ part) {
    __shared__ double red[8][kBlock / 64];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        node_ijk(g, p, i, j, k);
#pragma unroll
        for (int m = 0; m < 8; ++m) acc[m] += mode_sign(m, i, j, k) * r[p];
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        double v = acc[m];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
        if (lane == 0) red[m][w] = v;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        double v = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) v += red[threadIdx.x][q];
        part[threadIdx.x * gridDim.x + blockIdx.x] = v;
    }
}

// r -= sum over the present modes of coef[mode] sign_mode
struct ModeCoef {
    double c[8];
};
__global__ void k_sub_modes(Geo g, int64_t N, ModeCoef mc, double *__restrict__ r) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        node_ijk(g, p, i, j, k);
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < 8; ++m) s += mc.c[m] * mode_sign(m, i, j, k);
        r[p] -= s;
    }
}

// block partial sums of the dot products of w with V_0 .. V_{nv-1} (vectors
// of length L, V_q at V + q L): part[q][block]; w's chunk of each block is
// read once per vector from L2, the sums reduced in a fixed order
__global__ void k_mdot(const double *__restrict__ V, int64_t L, int nv, const double *__restrict__ w,
                       double *__restrict__ part) {
    __shared__ double red[kBlock / 64];
    const int64_t chunk = (L + gridDim.x - 1) / gridDim.x;
    const int64_t lo = blockIdx.x * chunk, hi = std::min<int64_t>(L, lo + chunk);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int q = 0; q < nv; ++q) {
        const double *v = V + q * L;
        double acc = 0.0;
        for (int64_t t = lo + threadIdx.x; t < hi; t += blockDim.x) acc += v[t] * w[t];
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
        if (lane == 0) red[wv] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int r = 0; r < (int)(blockDim.x >> 6); ++r) s += red[r];
            part[q * gridDim.x + blockIdx.x] = s;
        }
        __syncthreads();
    }
}

// out[q] (+)= sum over blocks of part[q][*]; one block per q
__global__ void k_msum(const double *__restrict__ part, int nblk, double *__restrict__ out, int add) {
    __shared__ double red[kBlock / 64];
    const int q = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) acc += part[q * nblk + b];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int r = 0; r < (int)(blockDim.x >> 6); ++r) s += red[r];
        out[q] = add ? dev_scalar(out + q) + s : s;
    }
}

// w -= sum_q h[q] V_q  (h on the device, nv <= kMaxRestart + 1)
__global__ void k_maxpy(const double *__restrict__ V, int64_t L, int nv, const double *h, double *__restrict__ w) {
    __shared__ double hs[kMaxRestart + 1];
    for (int q = threadIdx.x; q < nv; q += blockDim.x) hs[q] = dev_scalar(h + q);
    __syncthreads();
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < L; t += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int q = 0; q < nv; ++q) s += hs[q] * V[q * L + t];
        w[t] -= s;
    }
}

// y = a x + b y (b == 0: y = a x, y not read -- it may hold anything)
__global__ void k_axpby(int64_t L, double a, const double *x, double b, double *y) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < L; t += (int64_t)gridDim.x * blockDim.x)
        y[t] = b == 0.0 ? a * x[t] : a * x[t] + b * y[t];
}

// z = x - y
__global__ void k_sub(int64_t L, const double *__restrict__ x, const double *__restrict__ y, double *__restrict__ z) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < L; t += (int64_t)gridDim.x * blockDim.x)
        z[t] = x[t] - y[t];
}

// block-wide sum of one value per thread into part[blockIdx.x]
__device__ __forceinline__ void block_partial(double acc, double *part) {
    __shared__ double red[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += red[q];
        part[blockIdx.x] = s;
    }
}

// The sum of part[0 .. n) in a fixed order, the same bits in every block: a
// kernel that needs a dot product reduces the previous kernel's block
// partials itself, in each of its blocks, instead of a one-block reduction
// launch between the two.
__device__ __forceinline__ double block_sum(const double *__restrict__ part, int n) {
    __shared__ double red[kBlock / 64];
    __shared__ double total;
    double acc = 0.0;
    for (int b = threadIdx.x; b < n; b += blockDim.x) acc += part[b];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += red[q];
        total = s;
    }
    __syncthreads();
    return total;
}

// CG with its scalars on the device (no host round trip per iteration) in
// three kernels per iteration, each dot product fused into the kernel that
// writes its vector and reduced by the kernel that uses it; r.r alternates
// between sc[ia] (current) and sc[ib] (new).
// Ap = -div grad p, and the block partials of p . Ap
__global__ void k_cg_ap(Geo g, int64_t N, const double *__restrict__ p, double *__restrict__ Ap,
                        double *__restrict__ part) {
    double acc = 0.0;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < N; t += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        node_ijk(g, t, i, j, k);
        const double v = -(dif2(g, p, i, j, k, 0, 0) + dif2(g, p, i, j, k, 1, 1) + dif2(g, p, i, j, k, 2, 2));
        Ap[t] = v;
        acc += p[t] * v;
    }
    block_partial(acc, part);
}

// phi += alpha p, r -= alpha Ap with alpha = r.r / p.Ap (p.Ap from the
// nap partials of k_cg_ap), and the block partials of the new r . r;
// alpha = 0 once r.r <= thr2, so the iterations a batch runs past
// convergence change nothing (CG continued past convergence lets the
// residual wander)
__global__ void k_cg_x(int64_t N, const double *sc, int ia, double thr2, const double *__restrict__ p,
                       const double *__restrict__ Ap, double *__restrict__ phi, double *__restrict__ r,
                       const double *__restrict__ part_ap, int nap, double *__restrict__ part) {
    const double rr = dev_scalar(sc + ia), pap = block_sum(part_ap, nap);
    const double alpha = (pap > 0.0 && rr > thr2) ? rr / pap : 0.0;
    double acc = 0.0;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < N; t += (int64_t)gridDim.x * blockDim.x) {
        phi[t] += alpha * p[t];
        const double rv = r[t] - alpha * Ap[t];
        r[t] = rv;
        acc += rv * rv;
    }
    block_partial(acc, part);
}

// p = r + beta p with beta = new r.r / r.r (new r.r from the nrr partials
// of k_cg_x; block 0 stores it in sc[ib] for the next iteration and the host)
__global__ void k_cg_p(int64_t N, double *sc, int ia, int ib, const double *__restrict__ r,
                       double *__restrict__ p, const double *__restrict__ part_rr, int nrr) {
    const double rr = dev_scalar(sc + ia), rr1 = block_sum(part_rr, nrr);
    if (blockIdx.x == 0 && threadIdx.x == 0) sc[ib] = rr1;
    const double beta = rr > 0.0 ? rr1 / rr : 0.0;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < N; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = r[t] + beta * p[t];
}

__global__ void k_fill0(int64_t L, double *__restrict__ x) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < L; t += (int64_t)gridDim.x * blockDim.x)
        x[t] = 0.0;
}

// ------------------------------------------------------------------ host

inline int grid_for(int64_t n) { return (int)std::min<int64_t>(65536, std::max<int64_t>(1, (n + kBlock - 1) / kBlock)); }

struct Work {
    hipStream_t s;
    int64_t N, L;  // nodes, 3 nodes
    Geo g;
    int nred;      // blocks of the reductions
    double *part;  // partial sums [kMaxRestart + 2][nred]
    double *dres;  // device results [2 kMaxRestart + 8]
    std::vector<double> hres;
    hipError_t err = hipSuccess;

    void check(hipError_t e) {
        if (err == hipSuccess && e != hipSuccess) err = e;
    }
    void launched() { check(hipGetLastError()); }
    // out[0..nv) = V_q . w on the device (add: accumulate)
    void mdot(const double *V, int nv, const double *w, double *out, int64_t len, bool add = false) {
        hipLaunchKernelGGL(k_mdot, dim3(nred), dim3(kBlock), 0, s, V, len, nv, w, part);
        hipLaunchKernelGGL(k_msum, dim3(nv), dim3(kBlock), 0, s, part, nred, out, add ? 1 : 0);
        launched();
    }
    // copy n device results to the host (synchronises the stream)
    const double *fetch(const double *src, int n) {
        hres.resize(n);
        check(hipMemcpyAsync(hres.data(), src, n * sizeof(double), hipMemcpyDeviceToHost, s));
        check(hipStreamSynchronize(s));
        return hres.data();
    }
};

}  // namespace field
}  // namespace spic

using namespace spic;
using namespace spic::field;

namespace {

Geo make_geo(const spic_grid &gr) {
    Geo g;
    g.nx = gr.nx; g.ny = gr.ny; g.nz = gr.nz;
    g.ih[0] = 0.5 * gr.nx / gr.Lx;
    g.ih[1] = 0.5 * gr.ny / gr.Ly;
    g.ih[2] = 0.5 * gr.nz / gr.Lz;
    return g;
}

Species make_species(const spic_moment_array *mom, const double *qom, int nsp) {
    Species sp{};
    sp.n = nsp;
    for (int s = 0; s < nsp; ++s) {
        sp.m[s] = (const double *)mom[s].m;
        sp.qom[s] = qom[s];
    }
    return sp;
}

}  // namespace

// Validated arguments (spic_runtime.hip); device current.
int spic_ctx_s::field_apply(const spic_grid &gr, const spic_field_params &fp, const spic_em_state &em,
                            const spic_moment_array *mom, const double *qom, int32_t nsp, const double *x, double *y,
                            hipStream_t s) {
    const int64_t N = (int64_t)gr.nx * gr.ny * gr.nz;
    void *buf = nullptr;
    int rc;
    if ((rc = reserve("field_apply", (size_t)12 * N * sizeof(double), &buf))) return rc;
    double *mu = (double *)buf, *B = mu + 9 * N;
    const Geo g = make_geo(gr);
    const Species sp = make_species(mom, qom, nsp);
    hipLaunchKernelGGL(k_pack3, dim3(grid_for(N)), dim3(kBlock), 0, s, N, (const double *)em.bx,
                       (const double *)em.by, (const double *)em.bz, B);
    hipLaunchKernelGGL(k_mu_jhat, dim3(grid_for(N)), dim3(kBlock), 0, s, g, N, (const double *)B, sp, fp.dt, fp.c,
                       fp.theta, fp.fourpi, mu, (double *)nullptr);
    const double acc = (fp.c * fp.theta * fp.dt) * (fp.c * fp.theta * fp.dt);
    hipLaunchKernelGGL(k_apply, dim3(grid_for(N)), dim3(kBlock), 0, s, g, N, (const double *)mu, x, acc, y);
    return hip(hipGetLastError(), "field apply");
}

int spic_ctx_s::field_cycle(const spic_grid &gr, const spic_field_params &fp, spic_em_state &em,
                            const spic_moment_array *mom, const double *qom, int32_t nsp, spic_field_stats *stats,
                            hipStream_t s) {
    const int64_t N = (int64_t)gr.nx * gr.ny * gr.nz, L = 3 * N;
    const int m = fp.restart;
    // scratch: mu 9N | B, En, rhs, X, W, jh: 6 x 3N | rho, phi, r, p, Ap: 5N |
    // V (m + 1) x 3N | partial sums | device results
    const int nred = (int)std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, (L + kBlock - 1) / kBlock));
    const size_t words = (size_t)9 * N + 6 * (size_t)L + 5 * (size_t)N + (size_t)(m + 1) * L +
                         (size_t)(kMaxRestart + 2) * nred + 2 * kMaxRestart + 8;
    void *buf = nullptr;
    int rc;
    if ((rc = reserve("field_cycle", words * sizeof(double), &buf))) return rc;
    double *mu = (double *)buf, *B = mu + 9 * N, *En = B + L, *rhs = En + L, *X = rhs + L, *W = X + L, *jh = W + L;
    double *rho = jh + L, *phi = rho + N, *r = phi + N, *pp = r + N, *Ap = pp + N, *V = Ap + N;
    Work wk;
    wk.s = s;
    wk.N = N;
    wk.L = L;
    wk.g = make_geo(gr);
    wk.nred = nred;
    wk.part = V + (size_t)(m + 1) * L;
    wk.dres = wk.part + (size_t)(kMaxRestart + 2) * nred;
    const Geo &g = wk.g;
    const Species sp = make_species(mom, qom, nsp);
    const dim3 gn(grid_for(N)), gl(grid_for(L)), bk(kBlock);
    const double tol = fp.tol;
    spic_field_stats st{};

    // inputs: E^n and B^n packed, rho, the null-space part of rho removed
    hipLaunchKernelGGL(k_pack3, gn, bk, 0, s, N, (const double *)em.ex, (const double *)em.ey,
                       (const double *)em.ez, En);
    hipLaunchKernelGGL(k_pack3, gn, bk, 0, s, N, (const double *)em.bx, (const double *)em.by,
                       (const double *)em.bz, B);
    hipLaunchKernelGGL(k_rho, gn, bk, 0, s, N, sp, rho);
    {
        const int mb = std::min(nred, grid_for(N));
        hipLaunchKernelGGL(k_mode_partials, dim3(mb), bk, 0, s, g, N, (const double *)rho, wk.part);
        hipLaunchKernelGGL(k_msum, dim3(8), bk, 0, s, (const double *)wk.part, mb, wk.dres, 0);
        wk.launched();
        const double *sums = wk.fetch(wk.dres, 8);
        ModeCoef mc{};
        const int n3[3] = {gr.nx, gr.ny, gr.nz};
        for (int md = 0; md < 8; ++md) {
            bool present = true;
            for (int d = 0; d < 3; ++d)
                if ((md >> d & 1) && n3[d] % 2) present = false;
            mc.c[md] = present ? sums[md] / (double)N : 0.0;
        }
        hipLaunchKernelGGL(k_sub_modes, gn, bk, 0, s, g, N, mc, rho);
    }

    // divergence cleaning: CG on -div grad phi = fourpi rho - div E^n
    hipLaunchKernelGGL(k_poisson_rhs, gn, bk, 0, s, g, N, (const double *)En, (const double *)rho, fp.fourpi, r);
    hipLaunchKernelGGL(k_fill0, gn, bk, 0, s, N, phi);
    hipLaunchKernelGGL(k_axpby, gn, bk, 0, s, N, 1.0, (const double *)r, 0.0, pp);
    wk.mdot(r, 1, r, wk.dres, N);
    double rr = wk.fetch(wk.dres, 1)[0];
    const double bnorm_c = std::sqrt(rr);
    // the scalars stay on the device; the host reads r.r every kCgCheck
    // iterations (past convergence the device stops moving phi and r)
    constexpr int kCgCheck = 8;
    int it = 0;
    double *sc = wk.dres;  // [0] / [2] r.r (alternating)
    double *part_ap = wk.part, *part_rr = wk.part + nred;
    const double thr2 = (tol * bnorm_c) * (tol * bnorm_c);
    const dim3 gred(nred);
    int ia = 0, ib = 2;
    while (wk.err == hipSuccess && bnorm_c > 0.0 && std::sqrt(rr) > tol * bnorm_c && it < fp.max_iter) {
        const int batch = std::min(kCgCheck, fp.max_iter - it);
        for (int q = 0; q < batch; ++q) {
            hipLaunchKernelGGL(k_cg_ap, gred, bk, 0, s, g, N, (const double *)pp, Ap, part_ap);
            hipLaunchKernelGGL(k_cg_x, gred, bk, 0, s, N, (const double *)sc, ia, thr2, (const double *)pp,
                               (const double *)Ap, phi, r, (const double *)part_ap, nred, part_rr);
            hipLaunchKernelGGL(k_cg_p, gn, bk, 0, s, N, sc, ia, ib, (const double *)r, pp, (const double *)part_rr,
                               nred);
            std::swap(ia, ib);
        }
        wk.launched();
        it += batch;
        rr = wk.fetch(sc + ia, 1)[0];
    }
    st.clean_iters = it;
    st.clean_resid = bnorm_c > 0.0 ? std::sqrt(rr) / bnorm_c : 0.0;
    hipLaunchKernelGGL(k_sub_grad, gn, bk, 0, s, g, N, (const double *)phi, En);

    // the field equation: GMRes(m) from x0 = the cleaned E^n
    hipLaunchKernelGGL(k_mu_jhat, gn, bk, 0, s, g, N, (const double *)B, sp, fp.dt, fp.c, fp.theta, fp.fourpi, mu,
                       jh);
    hipLaunchKernelGGL(k_rhs, gn, bk, 0, s, g, N, (const double *)En, (const double *)B, (const double *)jh,
                       fp.theta, fp.dt, fp.c, fp.fourpi, rhs);
    hipLaunchKernelGGL(k_axpby, gl, bk, 0, s, L, 1.0, (const double *)En, 0.0, X);
    const double acc = (fp.c * fp.theta * fp.dt) * (fp.c * fp.theta * fp.dt);
    wk.mdot(rhs, 1, rhs, wk.dres, L);
    const double bnorm = std::sqrt(wk.fetch(wk.dres, 1)[0]);
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), y(m);
    int total = 0;
    double resid = 0.0;
    bool done = bnorm == 0.0;
    while (!done && wk.err == hipSuccess) {
        // r0 = rhs - A x, V_0 = r0 / |r0|
        hipLaunchKernelGGL(k_apply, gn, bk, 0, s, g, N, (const double *)mu, (const double *)X, acc, W);
        hipLaunchKernelGGL(k_sub, gl, bk, 0, s, L, (const double *)rhs, (const double *)W, V);
        wk.mdot(V, 1, V, wk.dres, L);
        const double beta = std::sqrt(wk.fetch(wk.dres, 1)[0]);
        resid = beta / bnorm;
        if (resid <= tol || total >= fp.max_iter) break;
        hipLaunchKernelGGL(k_axpby, gl, bk, 0, s, L, 1.0 / beta, (const double *)V, 0.0, V);
        std::fill(gv.begin(), gv.end(), 0.0);
        gv[0] = beta;
        int jend = 0;
        for (int j = 0; j < m && total < fp.max_iter; ++j) {
            double *Vj = V + (size_t)j * L, *Vn = V + (size_t)(j + 1) * L;
            hipLaunchKernelGGL(k_apply, gn, bk, 0, s, g, N, (const double *)mu, (const double *)Vj, acc, W);
            // classical Gram-Schmidt, twice; h on the device, summed into dres[0..j]
            double *h1 = wk.dres, *h2 = wk.dres + kMaxRestart + 1;
            wk.mdot(V, j + 1, W, h1, L);
            hipLaunchKernelGGL(k_maxpy, gl, bk, 0, s, (const double *)V, L, j + 1, (const double *)h1, W);
            wk.mdot(V, j + 1, W, h2, L);
            hipLaunchKernelGGL(k_maxpy, gl, bk, 0, s, (const double *)V, L, j + 1, (const double *)h2, W);
            wk.mdot(W, 1, W, h2 + j + 1, L);
            const double *hr = wk.fetch(wk.dres, 2 * kMaxRestart + 3);
            for (int q = 0; q <= j; ++q) H[(size_t)q * m + j] = hr[q] + hr[kMaxRestart + 1 + q];
            const double hn = std::sqrt(hr[kMaxRestart + 1 + j + 1]);
            H[(size_t)(j + 1) * m + j] = hn;
            // previous rotations, then the one that zeroes H[j+1][j]
            for (int q = 0; q < j; ++q) {
                const double a = H[(size_t)q * m + j], b = H[(size_t)(q + 1) * m + j];
                H[(size_t)q * m + j] = cs[q] * a + sn[q] * b;
                H[(size_t)(q + 1) * m + j] = -sn[q] * a + cs[q] * b;
            }
            const double a = H[(size_t)j * m + j], b = H[(size_t)(j + 1) * m + j];
            const double den = std::hypot(a, b);
            cs[j] = den > 0.0 ? a / den : 1.0;
            sn[j] = den > 0.0 ? b / den : 0.0;
            H[(size_t)j * m + j] = den;
            H[(size_t)(j + 1) * m + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            ++total;
            jend = j + 1;
            resid = std::fabs(gv[j + 1]) / bnorm;
            if (resid <= tol || !(hn > 0.0)) break;
            if (j + 1 < m) hipLaunchKernelGGL(k_axpby, gl, bk, 0, s, L, 1.0 / hn, (const double *)W, 0.0, Vn);
        }
        // x += V y, H y = g (upper triangular)
        for (int q = jend - 1; q >= 0; --q) {
            double t = gv[q];
            for (int u = q + 1; u < jend; ++u) t -= H[(size_t)q * m + u] * y[u];
            y[q] = H[(size_t)q * m + q] != 0.0 ? t / H[(size_t)q * m + q] : 0.0;
        }
        for (int q = 0; q < jend; ++q) y[q] = -y[q];  // k_maxpy subtracts
        wk.check(hipMemcpyAsync(wk.dres, y.data(), jend * sizeof(double), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_maxpy, gl, bk, 0, s, (const double *)V, L, jend, (const double *)wk.dres, X);
        wk.launched();
        (void)wk.fetch(wk.dres, 1);  // the host vector y is reused: wait for the copy
        if (total >= fp.max_iter) done = true;
    }
    // true residual of the final iterate
    if (wk.err == hipSuccess && bnorm > 0.0) {
        hipLaunchKernelGGL(k_apply, gn, bk, 0, s, g, N, (const double *)mu, (const double *)X, acc, W);
        hipLaunchKernelGGL(k_sub, gl, bk, 0, s, L, (const double *)rhs, (const double *)W, W);
        wk.mdot(W, 1, W, wk.dres, L);
        resid = std::sqrt(wk.fetch(wk.dres, 1)[0]) / bnorm;
    }
    st.solve_iters = total;
    st.solve_resid = resid;
    hipLaunchKernelGGL(k_update, gn, bk, 0, s, g, N, (const double *)X, (const double *)En, (const double *)B,
                       fp.theta, fp.c, fp.dt, em.ex, em.ey, em.ez, em.bx, em.by, em.bz);
    wk.launched();
    if (wk.err == hipSuccess) wk.check(hipStreamSynchronize(s));
    if (stats) *stats = st;
    return hip(wk.err, "field cycle");
}
