// spic_impl.h -- internal declarations shared by the HIP kernels and the
// host runtime of libspic.so.  Not part of the public ABI (include/spic.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spic.h"

namespace spic {

// Grid constants in the arithmetic type T of a kernel: box lengths, their
// inverses, and inverse cell sizes (cells per unit length) per axis.
template <typename T>
struct GridT {
    int nx, ny, nz, pad;
    T L[3];
    T invL[3];
    T invd[3];
};

// Mover constants in T: beta = qom*dt/2 (Eq. 1), bc = beta/c (Eq. 2),
// dt and dt/2 (Eq. 5 and the half-step position).
template <typename T>
struct MoveT {
    T beta, bc, dt, hdt;
    int niter, pad;
};

template <typename T>
struct FieldPtrs {
    const T *f[6];  // ex, ey, ez, bx, by, bz
};

template <typename T>
struct PartPtrs {
    T *x, *y, *z, *u, *v, *w, *q;
    int64_t *id;
};

// Host-side description of one species' work, already validated.
struct SpeciesWork {
    int dtype;          // particle dtype
    int64_t n;
    double qom;
    void *a[7];         // x y z u v w q
    int64_t *id;
    void *mom;          // NULL or [10][nodes]
    int acc_dtype;
};

struct LaunchCfg {
    int block = 256;
    int grid_cap = 1 << 20;
};

GridT<double> make_grid_d(const spic_grid &g);
GridT<float> make_grid_f(const spic_grid &g);

hipError_t launch_fill(void *p, int dtype, int64_t count, hipStream_t s);

// Generic fused path: one lane per particle, gather from global memory,
// moments by global atomics.  Correct for any particle order.
hipError_t launch_fused_generic(const spic_grid &g, const spic_params &prm, const spic_fields &f,
                                const SpeciesWork &w, const LaunchCfg &cfg, hipStream_t s);

// Deposit only (no move), generic path.
hipError_t launch_deposit_generic(const spic_grid &g, const SpeciesWork &w, const LaunchCfg &cfg,
                                  hipStream_t s);

}  // namespace spic
