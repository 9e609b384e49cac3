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
    int block = 256;        // generic kernels
    int grid_cap = 1 << 20;
    int tile_block = 256;   // tiled fused kernel
    int variant = 0;        // tiled kernel variant (see spic_tiled.hip)
};

// Tiles of tx x ty x tz cells (at most 64 cells) cover the grid; ntx.. are
// tile counts per axis (edge tiles may be partial).  The tiled kernel stages
// a region of rx x ry x rz nodes per tile: the tile's cells plus `halo`
// cells on every side, plus the +1 corner nodes.
struct TileGeom {
    int tx, ty, tz, cells;
    int ntx, nty, ntz, ntiles;
    int halo, rx, ry, rz;
    int ryp, rzp, rnp, pad;  // padded LDS extents (bank spread) and slots rx*ryp*rzp
};

template <typename T>
inline GridT<T> make_grid_t(const spic_grid &g) {
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

template <typename T>
inline MoveT<T> make_move(const spic_params &p, double qom) {
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
inline PartPtrs<T> part_ptrs(const SpeciesWork &w) {
    PartPtrs<T> p;
    p.x = (T *)w.a[0]; p.y = (T *)w.a[1]; p.z = (T *)w.a[2];
    p.u = (T *)w.a[3]; p.v = (T *)w.a[4]; p.w = (T *)w.a[5]; p.q = (T *)w.a[6];
    p.id = w.id;
    return p;
}

template <typename T>
inline FieldPtrs<T> field_ptrs(const spic_fields &f) {
    FieldPtrs<T> r;
    r.f[0] = (const T *)f.ex; r.f[1] = (const T *)f.ey; r.f[2] = (const T *)f.ez;
    r.f[3] = (const T *)f.bx; r.f[4] = (const T *)f.by; r.f[5] = (const T *)f.bz;
    return r;
}

// Everything the tiled fused code needs for one species: grid constants in
// the mover and accumulation precisions, fields, mover constants, particle
// arrays, moment output, per-tile particle ranges and tile geometry.
template <typename TP, typename TF, typename TA>
struct TileJob {
    GridT<TP> g;
    GridT<TA> ga;
    FieldPtrs<TF> f;
    MoveT<TP> mv;
    PartPtrs<TP> p;
    TA *mom;
    const uint32_t *tile_off;
    TileGeom tg;
    int nn, pad;
};

template <typename TP, typename TF, typename TA>
inline TileJob<TP, TF, TA> make_tile_job(const spic_grid &g, const spic_params &prm, const spic_fields &f,
                                         const SpeciesWork &w, const TileGeom &tg, const uint32_t *tile_off) {
    TileJob<TP, TF, TA> J;
    J.g = make_grid_t<TP>(g);
    J.ga = make_grid_t<TA>(g);
    J.f = field_ptrs<TF>(f);
    J.mv = make_move<TP>(prm, w.qom);
    J.p = part_ptrs<TP>(w);
    J.mom = (TA *)w.mom;
    J.tile_off = tile_off;
    J.tg = tg;
    J.nn = g.nx * g.ny * g.nz;
    J.pad = 0;
    return J;
}

// Zero `count` elements of a float (SPIC_F32), double (SPIC_F64) array.
hipError_t launch_fill(void *p, int dtype, int64_t count, hipStream_t s);
// Zero `count` 32-bit words.
hipError_t launch_zero32(void *p, int64_t count, hipStream_t s);

// Generic fused path: one lane per particle, gather from global memory,
// moments by global atomics.  Correct for any particle order.
hipError_t launch_fused_generic(const spic_grid &g, const spic_params &prm, const spic_fields &f,
                                const SpeciesWork &w, const LaunchCfg &cfg, hipStream_t s);

// Deposit only (no move), generic path.
hipError_t launch_deposit_generic(const spic_grid &g, const SpeciesWork &w, const LaunchCfg &cfg,
                                  hipStream_t s);

// Sort (spic_sort.hip).
TileGeom make_tile_geom(const spic_grid &g, int tx, int ty, int tz, int halo);
size_t sort_scratch_bytes(int64_t n, int dtype, bool with_id, const TileGeom &tg);
hipError_t launch_sort(const spic_grid &g, const SpeciesWork &w, const TileGeom &tg, void *scratch,
                       uint32_t *tile_off, hipStream_t s);

// Tiled fused path (spic_tiled.hip): one workgroup per tile of a sorted
// species, fields and moments of the tile region staged in LDS.
size_t tiled_lds_bytes(const TileGeom &tg, int dtype, int acc_dtype);
hipError_t launch_fused_tiled(const spic_grid &g, const spic_params &prm, const spic_fields &f,
                              const SpeciesWork &w, const TileGeom &tg, const uint32_t *tile_off,
                              const LaunchCfg &cfg, hipStream_t s);

// Work lists (spic_tiled.hip).  combo: 0 f64/f64/f64, 1 f32/f32/f64,
// 2 f32/f32/f32, 3 f32/f64/f64, 4 f32/f64/f32 (particles/fields/moments);
// -1 for an unsupported combination.
int job_combo(int dtype, int fdtype, int acc_dtype);
size_t tile_job_bytes(int combo);
void write_tile_job(int combo, void *dst, const spic_grid &g, const spic_params &prm, const spic_fields &f,
                    const SpeciesWork &w, const TileGeom &tg, const uint32_t *tile_off);
int worklist_groups(int combo, int variant, size_t lds, int block, int nitems, int max_groups);
hipError_t launch_worklist(int combo, int variant, const void *jobs, const uint2 *items, int nitems,
                           unsigned *counter, size_t lds, int block, int groups, hipStream_t s);
hipError_t launch_fill_many(void *const *ptrs, const int64_t *counts, int narr, int elem_bytes, hipStream_t s);

}  // namespace spic
