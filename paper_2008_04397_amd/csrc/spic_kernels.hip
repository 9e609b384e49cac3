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
