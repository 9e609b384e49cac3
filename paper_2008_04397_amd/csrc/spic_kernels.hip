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

#include "spic_device.h"
#include "spic_impl.h"

namespace spic {

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

// --------------------------------------------- compensated FP32 moments
//
// SPIC_F32C: all arithmetic in FP32.  The cell offset of a position uses a
// two-float 1/dx (hi + lo) and recovers the rounding error of x * hi with
// an FMA, so f = x/dx - i keeps its precision although x/dx is up to n;
// each term is added to the high plane by an atomic that returns the old
// value, and the exact rounding error of that addition (two-sum) goes to
// the low plane.  The moment is high + low.
struct GridC {
    GridT<float> g;
    float il[3];  // 1/dx - (float)(1/dx), per axis
};

__device__ __forceinline__ int locate_c(float s, float L, float invL, float ih, float il, int n, float &f) {
#pragma clang fp contract(off)
    const float w = pwrap(s, L, invL);
    const float t = w * ih;
    int i = (int)t;
    i = i > n - 1 ? n - 1 : i;
    f = __builtin_fmaf(w, ih, -(float)i) + w * il;
    return i;
}

// hi += t by an atomic; lo += the exact rounding error of that addition
__device__ __forceinline__ void add_comp(float *hi, float *lo, float t) {
#pragma clang fp contract(off)
    const float old = atomicAdd(hi, t);
    const float sum = old + t;
    const float bp = sum - old;
    const float ap = sum - bp;
    const float e = (old - ap) + (t - bp);
    if (e != 0.0f) atomicAdd(lo, e);
}

__device__ __forceinline__ void deposit_global_comp(const GridC &gc, float *__restrict__ hi, float *__restrict__ lo,
                                                    int nn, float x, float y, float z, float u, float v, float w,
                                                    float q) {
    const GridT<float> &g = gc.g;
    Cell<float> c;
    const int i = locate_c(x, g.L[0], g.invL[0], g.invd[0], gc.il[0], g.nx, c.fx);
    const int j = locate_c(y, g.L[1], g.invL[1], g.invd[1], gc.il[1], g.ny, c.fy);
    const int k = locate_c(z, g.L[2], g.invL[2], g.invd[2], gc.il[2], g.nz, c.fz);
    const int nyz = g.ny * g.nz;
    c.base = i * nyz + j * g.nz + k;
    c.ox = (i == g.nx - 1) ? -(g.nx - 1) * nyz : nyz;
    c.oy = (j == g.ny - 1) ? -(g.ny - 1) * g.nz : g.nz;
    c.oz = (k == g.nz - 1) ? -(g.nz - 1) : 1;
    float wt[8];
    int nd[8];
    pweights(c.fx, c.fy, c.fz, wt);
    pnodes(c, nd);
    const float val[10] = {1.0f, u, v, w, u * u, u * v, u * w, v * v, v * w, w * w};
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
        const float qw = q * wt[kk];
#pragma unroll
        for (int m = 0; m < 10; ++m) add_comp(hi + (size_t)m * nn + nd[kk], lo + (size_t)m * nn + nd[kk], qw * val[m]);
    }
}

template <typename TF>
__global__ void __launch_bounds__(1024)
k_fused_generic_c(GridT<float> g, GridC gc, FieldPtrs<TF> f, MoveT<float> mv, PartPtrs<float> p,
                  float *__restrict__ mom, int nn, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        float x = p.x[i], y = p.y[i], z = p.z[i], u = p.u[i], v = p.v[i], w = p.w[i];
        move_global(g, f, mv, x, y, z, u, v, w);
        p.x[i] = x; p.y[i] = y; p.z[i] = z;
        p.u[i] = u; p.v[i] = v; p.w[i] = w;
        if (mom) deposit_global_comp(gc, mom, mom + (size_t)10 * nn, nn, x, y, z, u, v, w, p.q[i]);
    }
}

__global__ void __launch_bounds__(1024)
k_deposit_generic_c(GridC gc, PartPtrs<float> p, float *__restrict__ mom, int nn, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        deposit_global_comp(gc, mom, mom + (size_t)10 * nn, nn, p.x[i], p.y[i], p.z[i], p.u[i], p.v[i], p.w[i],
                            p.q[i]);
}

static GridC make_grid_c(const spic_grid &g) {
    GridC c;
    c.g = make_grid_t<float>(g);
    const double L[3] = {g.Lx, g.Ly, g.Lz};
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int d = 0; d < 3; ++d) c.il[d] = (float)((double)n[d] / L[d] - (double)c.g.invd[d]);
    return c;
}

// ---------------------------------------------------------------- host side


static dim3 grid_for(int64_t n, const LaunchCfg &cfg) {
    int64_t b = (n + cfg.block - 1) / cfg.block;
    if (b > cfg.grid_cap) b = cfg.grid_cap;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

hipError_t launch_zero32(void *p, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    LaunchCfg cfg;
    hipLaunchKernelGGL(k_fill<uint32_t>, grid_for(count, cfg), dim3(cfg.block), 0, s, (uint32_t *)p, count);
    return hipGetLastError();
}

hipError_t launch_fill(void *p, int dtype, int64_t count, hipStream_t s) {
    if (dtype == SPIC_F32C) {  // the high and the low plane
        dtype = SPIC_F32;
        count *= 2;
    }
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
                       make_grid_t<TP>(g), make_grid_t<TA>(g), field_ptrs<TF>(f), make_move<TP>(prm, w.qom),
                       part_ptrs<TP>(w), (TA *)w.mom, nn, w.n);
}

hipError_t launch_fused_generic(const spic_grid &g, const spic_params &prm, const spic_fields &f,
                                const SpeciesWork &w, const LaunchCfg &cfg, hipStream_t s) {
    if (w.n <= 0) return hipSuccess;
    const bool f64acc = (w.mom == nullptr) || w.acc_dtype == SPIC_F64;
    if (w.mom && w.acc_dtype == SPIC_F32C) {
        if (w.dtype != SPIC_F32) return hipErrorInvalidValue;
        const int nn = g.nx * g.ny * g.nz;
        if (f.dtype == SPIC_F32)
            hipLaunchKernelGGL(k_fused_generic_c<float>, grid_for(w.n, cfg), dim3(cfg.block), 0, s,
                               make_grid_t<float>(g), make_grid_c(g), field_ptrs<float>(f),
                               make_move<float>(prm, w.qom), part_ptrs<float>(w), (float *)w.mom, nn, w.n);
        else
            hipLaunchKernelGGL(k_fused_generic_c<double>, grid_for(w.n, cfg), dim3(cfg.block), 0, s,
                               make_grid_t<float>(g), make_grid_c(g), field_ptrs<double>(f),
                               make_move<float>(prm, w.qom), part_ptrs<float>(w), (float *)w.mom, nn, w.n);
        return hipGetLastError();
    }
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
    if (w.acc_dtype == SPIC_F32C) {
        if (w.dtype != SPIC_F32) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_deposit_generic_c, grid_for(w.n, cfg), dim3(cfg.block), 0, s, make_grid_c(g),
                           part_ptrs<float>(w), (float *)w.mom, nn, w.n);
        return hipGetLastError();
    }
    if (w.dtype == SPIC_F64) {
        if (w.acc_dtype != SPIC_F64) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_deposit_generic<double, double>), grid_for(w.n, cfg), dim3(cfg.block), 0, s,
                           make_grid_t<double>(g), part_ptrs<double>(w), (double *)w.mom, nn, w.n);
    } else if (w.acc_dtype == SPIC_F64) {
        hipLaunchKernelGGL((k_deposit_generic<float, double>), grid_for(w.n, cfg), dim3(cfg.block), 0, s,
                           make_grid_t<double>(g), part_ptrs<float>(w), (double *)w.mom, nn, w.n);
    } else {
        hipLaunchKernelGGL((k_deposit_generic<float, float>), grid_for(w.n, cfg), dim3(cfg.block), 0, s,
                           make_grid_t<float>(g), part_ptrs<float>(w), (float *)w.mom, nn, w.n);
    }
    return hipGetLastError();
}

}  // namespace spic
