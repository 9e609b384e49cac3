// spic_kernels.hip -- HIP kernels for gfx950: implicit mover (Sec. II,
// Eq. 1-5) fused with the ten-moment gathering (Sec. II, moment equation;
// Sec. III-B, fusion of mover and gathering).
//
// Arithmetic types:
//   TP  particle state and mover arithmetic (float or double)
//   TF  node field storage (float or double), converted to TP on load
//   TA  moment accumulation (double, or float for precision studies); the
//       deposit weights and products are computed in TA from the stored
//       (rounded) particle state.
#include <hip/hip_runtime.h>

#include "spic_impl.h"

namespace spic {

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ float dfloor(float x) { return __builtin_floorf(x); }
__device__ __forceinline__ double dfloor(double x) { return __builtin_floor(x); }

// Periodic wrap into [0, L): r = s - L floor(s/L); a rounding that lands on
// L (or below 0) is the same point of the box as 0.
template <typename T>
__device__ __forceinline__ T pwrap(T s, T L, T invL) {
    T r = s - L * dfloor(s * invL);
    r = (r >= L) ? T(0) : r;
    return (r < T(0)) ? T(0) : r;
}

// Left node index along one axis and the offset xi in [0,1] inside the cell;
// the two non-zero linear weights (Eq. 3) are 1 - xi and xi.
template <typename T>
__device__ __forceinline__ int plocate(T s, T L, T invL, T invd, int n, T &xi) {
    T t = pwrap(s, L, invL) * invd;
    int i = (int)t;                 // t >= 0
    i = (i > n - 1) ? n - 1 : i;
    xi = t - (T)i;
    return i;
}

// Cell of a point: flat index of the lower corner node, the flat offsets to
// the +1 neighbours along x, y, z (negative where the box wraps) and the
// in-cell offsets.
template <typename T>
struct Cell {
    int base, ox, oy, oz;
    T fx, fy, fz;
};

template <typename T>
__device__ __forceinline__ Cell<T> pcell(const GridT<T> &g, T x, T y, T z) {
    Cell<T> c;
    int i = plocate(x, g.L[0], g.invL[0], g.invd[0], g.nx, c.fx);
    int j = plocate(y, g.L[1], g.invL[1], g.invd[1], g.ny, c.fy);
    int k = plocate(z, g.L[2], g.invL[2], g.invd[2], g.nz, c.fz);
    const int nyz = g.ny * g.nz;
    c.base = i * nyz + j * g.nz + k;
    c.ox = (i == g.nx - 1) ? -(g.nx - 1) * nyz : nyz;
    c.oy = (j == g.ny - 1) ? -(g.ny - 1) * g.nz : g.nz;
    c.oz = (k == g.nz - 1) ? -(g.nz - 1) : 1;
    return c;
}

// Trilinear weights of the 8 corners, corner index a + 2b + 4c for axis
// offsets (a, b, c) -- Eq. 3 as a product of 1-D hats.
template <typename T>
__device__ __forceinline__ void pweights(T fx, T fy, T fz, T w[8]) {
    const T gx = T(1) - fx, gy = T(1) - fy, gz = T(1) - fz;
    const T a00 = gx * gy, a10 = fx * gy, a01 = gx * fy, a11 = fx * fy;
    w[0] = a00 * gz; w[1] = a10 * gz; w[2] = a01 * gz; w[3] = a11 * gz;
    w[4] = a00 * fz; w[5] = a10 * fz; w[6] = a01 * fz; w[7] = a11 * fz;
}

template <typename T>
__device__ __forceinline__ void pnodes(const Cell<T> &c, int n[8]) {
    n[0] = c.base;
    n[1] = c.base + c.ox;
    n[2] = c.base + c.oy;
    n[3] = c.base + c.ox + c.oy;
    n[4] = c.base + c.oz;
    n[5] = n[1] + c.oz;
    n[6] = n[2] + c.oz;
    n[7] = n[3] + c.oz;
}

// Eq. 4 from global memory.
template <typename T, typename TF>
__device__ __forceinline__ void gather_global(const GridT<T> &g, const FieldPtrs<TF> &f,
                                              T x, T y, T z, T out[6]) {
    Cell<T> c = pcell(g, x, y, z);
    T w[8];
    int nd[8];
    pweights(c.fx, c.fy, c.fz, w);
    pnodes(c, nd);
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < 8; ++k) acc += w[k] * (T)__ldg(f.f[m] + nd[k]);
        out[m] = acc;
    }
}

// One implicit step of one particle (Sec. II).  The mean velocity is
// iterated niter times; iteration k gathers E, B at the current estimate of
// the half-step position (x^n for the first), then
//   vt   = v^n + beta E                                   (Eq. 1)
//   b    = (beta/c) B
//   vbar = (vt + vt x b + (vt . b) b) / (1 + b . b)       (Eq. 2)
//   xbar = x^n + vbar dt/2
// and finally v^{n+1} = 2 vbar - v^n, x^{n+1} = x^n + vbar dt (Eq. 5),
// wrapped into the periodic box.
template <typename T, typename TF>
__device__ __forceinline__ void move_global(const GridT<T> &g, const FieldPtrs<TF> &f,
                                            const MoveT<T> &mv, T &x, T &y, T &z, T &u, T &v, T &w) {
    const T x0 = x, y0 = y, z0 = z, u0 = u, v0 = v, w0 = w;
    T xb = x0, yb = y0, zb = z0;
    T ub = u0, vb = v0, wb = w0;
    for (int it = 0; it < mv.niter; ++it) {
        T F[6];
        gather_global(g, f, xb, yb, zb, F);
        const T ut = u0 + mv.beta * F[0];
        const T vt = v0 + mv.beta * F[1];
        const T wt = w0 + mv.beta * F[2];
        const T bx = mv.bc * F[3], by = mv.bc * F[4], bz = mv.bc * F[5];
        const T vdb = ut * bx + vt * by + wt * bz;
        const T inv = T(1) / (T(1) + (bx * bx + by * by + bz * bz));
        ub = (ut + (vt * bz - wt * by) + vdb * bx) * inv;
        vb = (vt + (wt * bx - ut * bz) + vdb * by) * inv;
        wb = (wt + (ut * by - vt * bx) + vdb * bz) * inv;
        xb = x0 + ub * mv.hdt;
        yb = y0 + vb * mv.hdt;
        zb = z0 + wb * mv.hdt;
    }
    u = T(2) * ub - u0;
    v = T(2) * vb - v0;
    w = T(2) * wb - w0;
    x = pwrap(x0 + ub * mv.dt, g.L[0], g.invL[0]);
    y = pwrap(y0 + vb * mv.dt, g.L[1], g.invL[1]);
    z = pwrap(z0 + wb * mv.dt, g.L[2], g.invL[2]);
}

// Ten-moment deposit of one particle by global atomics (moment equation of
// Sec. II): node g of corner k receives q W_k {1, u, v, w, uu, uv, uw, vv,
// vw, ww}.
template <typename TA>
__device__ __forceinline__ void deposit_global(const GridT<TA> &g, TA *__restrict__ mom, int nn,
                                               TA x, TA y, TA z, TA u, TA v, TA w, TA q) {
    Cell<TA> c = pcell(g, x, y, z);
    TA wt[8];
    int nd[8];
    pweights(c.fx, c.fy, c.fz, wt);
    pnodes(c, nd);
    const TA val[10] = {TA(1), u, v, w, u * u, u * v, u * w, v * v, v * w, w * w};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const TA qw = q * wt[k];
#pragma unroll
        for (int m = 0; m < 10; ++m) atomicAdd(mom + (size_t)m * nn + nd[k], qw * val[m]);
    }
}

// ---------------------------------------------------------------- kernels

template <typename T>
__global__ void k_fill(T *__restrict__ p, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = T(0);
}

template <typename TP, typename TF, typename TA>
__global__ void __launch_bounds__(1024)
k_fused_generic(GridT<TP> g, GridT<TA> ga, FieldPtrs<TF> f, MoveT<TP> mv, PartPtrs<TP> p,
                TA *__restrict__ mom, int nn, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        TP x = p.x[i], y = p.y[i], z = p.z[i], u = p.u[i], v = p.v[i], w = p.w[i];
        move_global(g, f, mv, x, y, z, u, v, w);
        p.x[i] = x; p.y[i] = y; p.z[i] = z;
        p.u[i] = u; p.v[i] = v; p.w[i] = w;
        if (mom) deposit_global<TA>(ga, mom, nn, (TA)x, (TA)y, (TA)z, (TA)u, (TA)v, (TA)w, (TA)p.q[i]);
    }
}

template <typename TP, typename TA>
__global__ void __launch_bounds__(1024)
k_deposit_generic(GridT<TA> ga, PartPtrs<TP> p, TA *__restrict__ mom, int nn, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        deposit_global<TA>(ga, mom, nn, (TA)p.x[i], (TA)p.y[i], (TA)p.z[i], (TA)p.u[i], (TA)p.v[i],
                           (TA)p.w[i], (TA)p.q[i]);
}

// ---------------------------------------------------------------- host side

template <typename T>
static GridT<T> make_grid(const spic_grid &g) {
    GridT<T> r;
    r.nx = g.nx; r.ny = g.ny; r.nz = g.nz; r.pad = 0;
    const double L[3] = {g.Lx, g.Ly, g.Lz};
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int d = 0; d < 3; ++d) {
        r.L[d] = (T)L[d];
        r.invL[d] = (T)(1.0 / L[d]);
        r.invd[d] = (T)((double)n[d] / L[d]);
    }
    return r;
}

GridT<double> make_grid_d(const spic_grid &g) { return make_grid<double>(g); }
GridT<float> make_grid_f(const spic_grid &g) { return make_grid<float>(g); }

template <typename T>
static MoveT<T> make_move(const spic_params &p, double qom) {
    MoveT<T> m;
    const double beta = qom * p.dt / 2.0;
    m.beta = (T)beta;
    m.bc = (T)(beta / p.c);
    m.dt = (T)p.dt;
    m.hdt = (T)(p.dt / 2.0);
    m.niter = p.niter_mover;
    m.pad = 0;
    return m;
}

template <typename T>
static PartPtrs<T> parts(const SpeciesWork &w) {
    PartPtrs<T> p;
    p.x = (T *)w.a[0]; p.y = (T *)w.a[1]; p.z = (T *)w.a[2];
    p.u = (T *)w.a[3]; p.v = (T *)w.a[4]; p.w = (T *)w.a[5]; p.q = (T *)w.a[6];
    p.id = w.id;
    return p;
}

template <typename T>
static FieldPtrs<T> fields(const spic_fields &f) {
    FieldPtrs<T> r;
    r.f[0] = (const T *)f.ex; r.f[1] = (const T *)f.ey; r.f[2] = (const T *)f.ez;
    r.f[3] = (const T *)f.bx; r.f[4] = (const T *)f.by; r.f[5] = (const T *)f.bz;
    return r;
}

static dim3 grid_for(int64_t n, const LaunchCfg &cfg) {
    int64_t b = (n + cfg.block - 1) / cfg.block;
    if (b > cfg.grid_cap) b = cfg.grid_cap;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

hipError_t launch_fill(void *p, int dtype, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    LaunchCfg cfg;
    if (dtype == SPIC_F64)
        hipLaunchKernelGGL(k_fill<double>, grid_for(count, cfg), dim3(cfg.block), 0, s, (double *)p, count);
    else
        hipLaunchKernelGGL(k_fill<float>, grid_for(count, cfg), dim3(cfg.block), 0, s, (float *)p, count);
    return hipGetLastError();
}

template <typename TP, typename TF, typename TA>
static void fused_generic_t(const spic_grid &g, const spic_params &prm, const spic_fields &f,
                            const SpeciesWork &w, const LaunchCfg &cfg, hipStream_t s) {
    const int nn = g.nx * g.ny * g.nz;
    hipLaunchKernelGGL((k_fused_generic<TP, TF, TA>), grid_for(w.n, cfg), dim3(cfg.block), 0, s,
                       make_grid<TP>(g), make_grid<TA>(g), fields<TF>(f), make_move<TP>(prm, w.qom),
                       parts<TP>(w), (TA *)w.mom, nn, w.n);
}

hipError_t launch_fused_generic(const spic_grid &g, const spic_params &prm, const spic_fields &f,
                                const SpeciesWork &w, const LaunchCfg &cfg, hipStream_t s) {
    if (w.n <= 0) return hipSuccess;
    const bool f64acc = (w.mom == nullptr) || w.acc_dtype == SPIC_F64;
    if (w.dtype == SPIC_F64) {
        if (f.dtype != SPIC_F64 || !f64acc) return hipErrorInvalidValue;
        fused_generic_t<double, double, double>(g, prm, f, w, cfg, s);
    } else if (f.dtype == SPIC_F32) {
        if (f64acc) fused_generic_t<float, float, double>(g, prm, f, w, cfg, s);
        else fused_generic_t<float, float, float>(g, prm, f, w, cfg, s);
    } else {
        if (f64acc) fused_generic_t<float, double, double>(g, prm, f, w, cfg, s);
        else fused_generic_t<float, double, float>(g, prm, f, w, cfg, s);
    }
    return hipGetLastError();
}

hipError_t launch_deposit_generic(const spic_grid &g, const SpeciesWork &w, const LaunchCfg &cfg,
                                  hipStream_t s) {
    if (w.n <= 0) return hipSuccess;
    const int nn = g.nx * g.ny * g.nz;
    if (w.dtype == SPIC_F64) {
        if (w.acc_dtype != SPIC_F64) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_deposit_generic<double, double>), grid_for(w.n, cfg), dim3(cfg.block), 0, s,
                           make_grid<double>(g), parts<double>(w), (double *)w.mom, nn, w.n);
    } else if (w.acc_dtype == SPIC_F64) {
        hipLaunchKernelGGL((k_deposit_generic<float, double>), grid_for(w.n, cfg), dim3(cfg.block), 0, s,
                           make_grid<double>(g), parts<float>(w), (double *)w.mom, nn, w.n);
    } else {
        hipLaunchKernelGGL((k_deposit_generic<float, float>), grid_for(w.n, cfg), dim3(cfg.block), 0, s,
                           make_grid<float>(g), parts<float>(w), (float *)w.mom, nn, w.n);
    }
    return hipGetLastError();
}

}  // namespace spic
