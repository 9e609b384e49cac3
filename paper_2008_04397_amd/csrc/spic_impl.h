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
    int fixed_geo = 1;      // compile-time region geometry for the default tiling
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

// Padded LDS extents RYP >= ry, RZP >= rz of a region: the lower corners of
// a full tile's cells (one cell per lane) should hit the 16 pairs of 4-byte
// banks as evenly as possible, for every corner offset; among the most even
// paddings the one with the fewest slots wins.  constexpr so that kernels
// specialised for one tiling use the same layout as the host.
struct RegionPadding {
    int ryp, rzp;
};

constexpr RegionPadding region_padding(int tx, int ty, int tz, int halo) {
    const int rx = tx + 2 * halo + 1, ry = ty + 2 * halo + 1, rz = tz + 2 * halo + 1;
    int best_w = 1 << 30, best_n = 1 << 30, bry = ry, brz = rz;
    for (int ryp = ry; ryp < ry + 9; ++ryp)
        for (int rzp = rz; rzp < rz + 9; ++rzp) {
            const int sx = ryp * rzp, sy = rzp;
            int worst = 0;
            for (int c = 0; c < 8; ++c) {
                int cnt[16] = {};
                for (int li = 0; li < tx; ++li)
                    for (int lj = 0; lj < ty; ++lj)
                        for (int lk = 0; lk < tz; ++lk) {
                            const int slot = (li + halo + (c & 1)) * sx + (lj + halo + ((c >> 1) & 1)) * sy +
                                             (lk + halo + (c >> 2));
                            const int v = ++cnt[slot & 15];
                            worst = v > worst ? v : worst;
                        }
            }
            const int slots = rx * sx;
            if (worst < best_w || (worst == best_w && slots < best_n)) {
                best_w = worst;
                best_n = slots;
                bry = ryp;
                brz = rzp;
            }
        }
    return RegionPadding{bry, brz};
}

// Region geometry known at compile time (the default tiling): LDS offsets of
// corners and moment components fold into instruction immediates.
struct GeoRuntime {
    static constexpr bool fixed = false;
    static constexpr int tx = 0, ty = 0, tz = 0, halo = 0, rx = 0, ry = 0, rz = 0, ryp = 0, rzp = 0, rnp = 0;
};

template <int TX, int TY, int TZ, int HALO>
struct GeoFixed {
    static constexpr bool fixed = true;
    static constexpr int tx = TX, ty = TY, tz = TZ, halo = HALO;
    static constexpr int rx = TX + 2 * HALO + 1, ry = TY + 2 * HALO + 1, rz = TZ + 2 * HALO + 1;
    static constexpr int ryp = region_padding(TX, TY, TZ, HALO).ryp;
    static constexpr int rzp = region_padding(TX, TY, TZ, HALO).rzp;
    static constexpr int rnp = rx * ryp * rzp;
};

using GeoDefault = GeoFixed<4, 4, 4, 1>;

// The tiled kernels address particle arrays with 32-bit byte offsets.
inline bool tiled_fits(int64_t n, int dtype) {
    return n >= 0 && (uint64_t)n * (dtype == SPIC_F64 ? 8u : 4u) < ((uint64_t)1 << 32);
}

inline bool geo_is_default(const TileGeom &t) {
    return t.tx == GeoDefault::tx && t.ty == GeoDefault::ty && t.tz == GeoDefault::tz &&
           t.halo == GeoDefault::halo && t.ryp == GeoDefault::ryp && t.rzp == GeoDefault::rzp &&
           t.rnp == GeoDefault::rnp;
}

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
// prev: tile_off already holds the per-tile ranges of the particles'
// current order (an earlier sort with the same tiles and n); the key pass
// then walks tiles in that order, which keeps the scatter's writes local.
hipError_t launch_sort(const spic_grid &g, const SpeciesWork &w, const TileGeom &tg, void *scratch,
                       uint32_t *tile_off, bool prev, hipStream_t s);
inline bool same_tiling(const TileGeom &a, const TileGeom &b) {
    return a.tx == b.tx && a.ty == b.ty && a.tz == b.tz && a.halo == b.halo && a.ntiles == b.ntiles &&
           a.ntx == b.ntx && a.nty == b.nty && a.ntz == b.ntz;
}

// Tiled fused path (spic_tiled.hip): one workgroup per tile of a sorted
// species, fields and moments of the tile region staged in LDS.
// LDS bytes of one workgroup of the tiled kernel (variant and block size
// matter: variant 2 adds per-wave queues).
size_t tiled_lds_bytes(const TileGeom &tg, int dtype, int acc_dtype, int variant, int block);
hipError_t launch_fused_tiled(const spic_grid &g, const spic_params &prm, const spic_fields &f,
                              const SpeciesWork &w, const TileGeom &tg, const uint32_t *tile_off,
                              const LaunchCfg &cfg, hipStream_t s);

// Work lists (spic_tiled.hip).  combo: 0 f64/f64/f64, 1 f32/f32/f64,
// 2 f32/f32/f32, 3 f32/f64/f64, 4 f32/f64/f32 (particles/fields/moments);
// -1 for an unsupported combination.  fixed: every job of the launch uses
// the default tiling (GeoDefault) and the kernel compiled for it.
int job_combo(int dtype, int fdtype, int acc_dtype);
size_t tile_job_bytes(int combo);
void write_tile_job(int combo, void *dst, const spic_grid &g, const spic_params &prm, const spic_fields &f,
                    const SpeciesWork &w, const TileGeom &tg, const uint32_t *tile_off);
int worklist_groups(int combo, bool fixed, int variant, size_t lds, int block, int nitems, int max_groups);
hipError_t launch_worklist(int combo, bool fixed, int variant, const void *jobs, const uint2 *items, int nitems,
                           unsigned *counter, size_t lds, int block, int groups, hipStream_t s);
hipError_t launch_fill_many(void *const *ptrs, const int64_t *counts, int narr, int elem_bytes, hipStream_t s);

}  // namespace spic
