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
// dt and dt/2 (Eq. 5 and the half-step position); niter iterations, or at
// most niter with a tolerance tol > 0 on the change of the mean velocity.
template <typename T>
struct MoveT {
    T beta, bc, dt, hdt, tol;
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
    // when set, the tiled kernel reads the particles from src (the sort's
    // reordered copy) and writes all of them, q and id included, to a / id
    bool from_src = false;
    void *src[7] = {};
    int64_t *src_id = nullptr;
};

struct LaunchCfg {
    int block = 256;        // generic kernels
    int grid_cap = 1 << 20;
    int tile_block = -1;    // tiled fused kernel (-1: by variant)
    int variant = -1;       // tiled kernel variant (0..3; see spic_tiled.hip; -1: by precision)
    int fixed_geo = 1;      // compile-time region geometry for the default tiling
    int mover_halo = -1;    // variant 2: halo of the mover's field region (-1: tile halo + 1)
    int mover_cache = 1;    // variant 2: the mover keeps the last cell's field corners in registers
    int mover_block = 512;  // variant 2: threads per workgroup of the mover launch
    int tile_group = 4;     // tiles to workgroups: g >= 0 groups of 2^g tiles dealt to the XCDs, -1 XCD slabs
    size_t lds_max = 65536; // LDS bytes a workgroup may use on the device
};

// Default mapping of tiles to workgroups: groups of 16 consecutive tiles
// dealt to the XCDs in turn.  Measured as fast as XCD slabs on resident
// boxes, and it keeps a streamed batch (a contiguous eighth of the tiles)
// on all 8 XCDs where slabs would give it to one.
constexpr int kTileGroup = 4;

// Workgroups per XCD of a tiled launch over `ntiles` tiles (the grid is 8
// times this): ceil(ntiles / 8) for the XCD-slab mapping (glog < 0); whole
// groups of 2^glog tiles per XCD for the group mapping.
inline int tile_chunk(int ntiles, int glog) {
    if (glog < 0) return (ntiles + 7) / 8;
    const int g = 1 << glog;
    return ((ntiles + g - 1) / g + 7) / 8 * g;
}

// Tile of workgroup b (workgroup b runs on XCD b % 8).  Slab mapping (glog
// < 0): XCD x takes the contiguous tiles [x * chunk, (x + 1) * chunk), so
// a slab's fields and moments stay in that XCD's L2.  Group mapping (glog
// >= 0): groups of 2^glog consecutive tiles are dealt to the XCDs in turn,
// for launches whose particles occupy a contiguous fraction of the tiles
// (a streamed batch), which slabs would give to one XCD.  `chunk` is the
// number of workgroups per XCD (tile_chunk).
__host__ __device__ __forceinline__ int tile_of_block(int b, int chunk, int glog) {
    if (glog < 0) return (b & 7) * chunk + (b >> 3);
    const int r = b >> 3;
    return ((((r >> glog) << 3) + (b & 7)) << glog) | (r & ((1 << glog) - 1));
}

// Tiled-kernel variants (spic_tiled.hip): 0 one kernel with LDS-atomic
// deposits, 1 the same with the field corners of a thread's last cell in
// registers, 2 two launches -- the mover, then the sorted deposit into
// per-lane register sums, 3 both in one launch (FP32 particles; measured
// as fast as 2, not faster).  Defaults, measured fastest on the Harris boxes:
// 2 for FP32 particles, 1 for FP64 (the sorted deposit's 80 register sums
// take 160 VGPRs in FP64, which leaves it two waves per SIMD and spills).
// Workgroup size when the options leave it to the library: 512 for
// variant 0, 256 otherwise (variant 1's FP64 corner cache allows two
// waves per SIMD: two workgroups of 256 per CU).
constexpr int kVariantSplit = 2;
constexpr int kVariantLaneCell = 3;
// the variants whose deposit wants full rows (lane c on cell c)
inline bool variant_rows(int v) { return v == kVariantSplit || v == kVariantLaneCell; }
inline int auto_variant(int dtype, int) { return dtype == SPIC_F32 ? kVariantSplit : 1; }
inline int auto_tile_block(int variant) { return variant == 0 ? 512 : 256; }
inline LaunchCfg resolve_cfg(LaunchCfg c, int dtype, int acc_dtype) {
    if (c.variant < 0) c.variant = auto_variant(dtype, acc_dtype);
    if (c.tile_block < 0) c.tile_block = auto_tile_block(c.variant);
    return c;
}

// Tiles of tx x ty x tz cells (at most 64 cells) cover the grid; ntx.. are
// tile counts per axis (edge tiles may be partial).  The tiled kernel stages
// a region of rx x ry x rz nodes per tile: the tile's cells plus `halo`
// cells on every side, plus the +1 corner nodes.
struct TileGeom {
    int tx, ty, tz, cells;
    int ntx, nty, ntz, ntiles;
    int halo, rx, ry, rz;
    // Axis roles (0 x, 1 y, 2 z): a tile's cells are numbered with `slow`
    // slowest and `fast` fastest, and the region's LDS slot of a node with
    // region coordinates (a, b, c) is a*sx + b*sy + c*sz.
    int slow, mid, fast;
    int sx, sy, sz, rnp;  // slot strides and slots (padded for bank spread)
    // Order of a tile's particles after a sort (rank-major): rows = 1, full
    // rows -- a tile of n particles and C cells has R = n / C rows in which
    // slot (r, c) holds rank r of cell c whenever cell c has more than r
    // particles; the particles of ranks >= R fill the remaining slots of
    // those rows, then a last partial row -- so lane c of a row holds cell c
    // for all but a few particles even when the cell counts differ; rows =
    // 0, plain rank blocks (a rank's block holds only the cells that have
    // that rank, so a row never holds one cell twice).
    int rows;
};

// LDS bank spread of a region layout.  A wave deposits with one lane per
// cell of a tile (rank-major order), and an FP64 LDS access by 16
// consecutive lanes is conflict free when their slots are distinct modulo
// 16 (16 pairs of 4-byte banks).  The fast and middle extents are padded to
// P_fast >= r_fast, P_mid >= r_mid so that (1) every group of 16 consecutive
// cells hits the 16 pairs as evenly as possible, for every corner, (2)
// preferably the slow stride P_mid * P_fast is a multiple of 16, so that a
// particle that drifted one cell along the slow axis keeps its bank pair,
// and (3) the region has the fewest slots (without (2) for layout 0: the
// compact layout keeps two FP64 workgroups per CU).  Layout 2 is dense (no
// padding, bank spread ignored): for the kernels that deposit most of their
// moments from registers and want the smallest LDS footprint.  constexpr so
// that kernels specialised for one tiling use the same layout as the host.
struct RegionLayout {
    int sx, sy, sz, rnp;
};

constexpr RegionLayout region_layout(int tx, int ty, int tz, int halo, int slow, int mid, int fast,
                                     int layout = 1) {
    const int t[3] = {tx, ty, tz};
    const int r[3] = {tx + 2 * halo + 1, ty + 2 * halo + 1, tz + 2 * halo + 1};
    if (layout == 2) {
        int st[3] = {0, 0, 0};
        st[fast] = 1;
        st[mid] = r[fast];
        st[slow] = r[mid] * r[fast];
        return RegionLayout{st[0], st[1], st[2], r[0] * r[1] * r[2]};
    }
    const bool prefer_align = layout == 1;
    const int cells = tx * ty * tz;
    int best_w = 1 << 30, best_a = 2, best_n = 1 << 30, bpm = r[mid], bpf = r[fast];
    for (int pm = r[mid]; pm < r[mid] + 9; ++pm)
        for (int pf = r[fast]; pf < r[fast] + 9; ++pf) {
            int st[3] = {0, 0, 0};
            st[fast] = 1;
            st[mid] = pf;
            st[slow] = pm * pf;
            int worst = 0;
            for (int g0 = 0; g0 < cells; g0 += 16)
                for (int k = 0; k < 8; ++k) {
                    int cnt[16] = {};
                    for (int l = g0; l < g0 + 16 && l < cells; ++l) {
                        // local cell l -> (slow, mid, fast) coordinates
                        const int cf = l % t[fast], cm = (l / t[fast]) % t[mid], cs = l / (t[fast] * t[mid]);
                        int c3[3] = {0, 0, 0};
                        c3[slow] = cs;
                        c3[mid] = cm;
                        c3[fast] = cf;
                        int slot = 0;
                        for (int d = 0; d < 3; ++d) slot += (c3[d] + halo + ((k >> d) & 1)) * st[d];
                        const int v = ++cnt[slot & 15];
                        worst = v > worst ? v : worst;
                    }
                }
            const int align = (!prefer_align || (pm * pf) % 16 == 0) ? 0 : 1;
            const int slots = r[slow] * pm * pf;
            if (worst < best_w || (worst == best_w && (align < best_a || (align == best_a && slots < best_n)))) {
                best_w = worst;
                best_a = align;
                best_n = slots;
                bpm = pm;
                bpf = pf;
            }
        }
    int st[3] = {0, 0, 0};
    st[fast] = 1;
    st[mid] = bpf;
    st[slow] = bpm * bpf;
    return RegionLayout{st[0], st[1], st[2], r[slow] * bpm * bpf};
}

// Region geometry known at compile time (the default tiling): LDS offsets of
// corners and moment components fold into instruction immediates.
struct GeoRuntime {
    static constexpr bool fixed = false;
    static constexpr int tx = 0, ty = 0, tz = 0, halo = 0, rx = 0, ry = 0, rz = 0, slow = 0, mid = 0, fast = 0,
                         sx = 0, sy = 0, sz = 0, rnp = 0;
};

template <int TX, int TY, int TZ, int HALO, int SLOW, int MID, int FAST, int LAYOUT = 1>
struct GeoFixed {
    static constexpr bool fixed = true;
    static constexpr int tx = TX, ty = TY, tz = TZ, halo = HALO, slow = SLOW, mid = MID, fast = FAST;
    static constexpr int rx = TX + 2 * HALO + 1, ry = TY + 2 * HALO + 1, rz = TZ + 2 * HALO + 1;
    static constexpr RegionLayout lay = region_layout(TX, TY, TZ, HALO, SLOW, MID, FAST, LAYOUT);
    static constexpr int sx = lay.sx, sy = lay.sy, sz = lay.sz, rnp = lay.rnp;
};

// 4x4x4 tiles, halo 1, z slowest (the Harris boxes have their finest cells
// along z, which particles cross most often)
using GeoDefault = GeoFixed<4, 4, 4, 1, 2, 0, 1>;
// the same tiling with the dense layout
using GeoDense = GeoFixed<4, 4, 4, 1, 2, 0, 1, 2>;
// the mover launch of the split variant: two cells of halo (particles that
// drifted since the last sort still gather from LDS)
using GeoMover2 = GeoFixed<4, 4, 4, 2, 2, 0, 1>;
// the compact conflict-free layout (the FP64 default of the one-kernel
// variants)
using GeoCompact = GeoFixed<4, 4, 4, 1, 2, 0, 1, 0>;

// The tiled kernels address particle arrays with 32-bit byte offsets.
inline bool tiled_fits(int64_t n, int dtype) {
    return n >= 0 && (uint64_t)n * (dtype == SPIC_F64 ? 8u : 4u) < ((uint64_t)1 << 32);
}

template <class GEO>
inline bool geo_is(const TileGeom &t) {
    return t.tx == GEO::tx && t.ty == GEO::ty && t.tz == GEO::tz && t.halo == GEO::halo && t.slow == GEO::slow &&
           t.mid == GEO::mid && t.fast == GEO::fast && t.sx == GEO::sx && t.sy == GEO::sy && t.sz == GEO::sz &&
           t.rnp == GEO::rnp;
}

inline bool geo_is_default(const TileGeom &t) { return geo_is<GeoDefault>(t); }

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
    m.tol = (T)p.mover_tol;
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
    PartPtrs<TP> p;   // particles written
    PartPtrs<TP> in;  // particles read (p, or the sort's reordered copy)
    TA *mom;
    const uint32_t *tile_off;
    TileGeom tg;
    int nn;
    int copy_rest;    // in != p: also write q (and id) to p
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
    J.in = J.p;
    J.copy_rest = 0;
    if (w.from_src) {
        J.in.x = (TP *)w.src[0]; J.in.y = (TP *)w.src[1]; J.in.z = (TP *)w.src[2];
        J.in.u = (TP *)w.src[3]; J.in.v = (TP *)w.src[4]; J.in.w = (TP *)w.src[5]; J.in.q = (TP *)w.src[6];
        J.in.id = w.src_id;
        J.copy_rest = 1;
    }
    J.mom = (TA *)w.mom;
    J.tile_off = tile_off;
    J.tg = tg;
    J.nn = g.nx * g.ny * g.nz;
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
TileGeom make_tile_geom(const spic_grid &g, int tx, int ty, int tz, int halo, int layout = 1, bool rows = true);
size_t sort_scratch_bytes(int64_t n, int dtype, bool with_id, const TileGeom &tg);
// prev: tile_off already holds the per-tile ranges of the particles'
// current order (an earlier sort with the same tiles and n); the key pass
// then walks each tile in that order, which keeps the gather's reads local.
// sorted_out: when not NULL the reordered particles stay in the scratch and
// are not copied back; *sorted_out receives w with from_src/src set, for a
// tiled launch that reads them (and writes every array of w) right after.
hipError_t launch_sort(const spic_grid &g, const SpeciesWork &w, const TileGeom &tg, void *scratch,
                       uint32_t *tile_off, bool prev, hipStream_t s, SpeciesWork *sorted_out = nullptr);
inline bool same_tiling(const TileGeom &a, const TileGeom &b) {
    return a.tx == b.tx && a.ty == b.ty && a.tz == b.tz && a.ntx == b.ntx && a.nty == b.nty && a.ntz == b.ntz &&
           a.slow == b.slow && a.mid == b.mid && a.fast == b.fast && a.rows == b.rows;
}

// Tiled path (spic_tiled.hip): one workgroup per tile of a sorted species,
// fields and moments of the tile region staged in LDS.  LDS bytes of one
// workgroup (for variant 2 the larger of its two launches at the tile's
// halo).
size_t tiled_lds_bytes(const TileGeom &tg, int dtype, int acc_dtype, int variant, int block);
hipError_t launch_fused_tiled(const spic_grid &g, const spic_params &prm, const spic_fields &f,
                              const SpeciesWork &w, const TileGeom &tg, const uint32_t *tile_off,
                              const LaunchCfg &cfg, hipStream_t s);

// Work lists (spic_tiled.hip).  combo: 0 f64/f64/f64, 1 f32/f32/f64,
// 2 f32/f32/f32, 3 f32/f64/f64, 4 f32/f64/f32 (particles/fields/moments);
// -1 for an unsupported combination.  fixed: every job of the launch uses
// the default tiling (GeoDefault) and the kernels compiled for it.
int job_combo(int dtype, int fdtype, int acc_dtype);
size_t tile_job_bytes(int combo);
void write_tile_job(int combo, void *dst, const spic_grid &g, const spic_params &prm, const spic_fields &f,
                    const SpeciesWork &w, const TileGeom &tg, const uint32_t *tile_off);
// Launch sizes of one combination's work-list launches: variant 2 runs a
// persistent mover list (512 threads, fields) and then a deposit list of
// one `block`-thread workgroup per item; variants 0 and 1 one persistent
// list (`block` threads, `mover` fields).
struct WorklistGroups {
    int mover, deposit;
    size_t lds_mover, lds_deposit;
};
// tg: the largest region of the launch's jobs.  Also allows the LDS sizes;
// call before any stream capture.
WorklistGroups worklist_groups(int combo, bool fixed, int variant, const TileGeom &tg, int block, int nitems,
                               int max_groups);
// counters: two zeroed counters (variant 2 uses both).
hipError_t launch_worklist(int combo, bool fixed, int variant, const void *jobs, const uint2 *items, int nitems,
                           unsigned *counters, const WorklistGroups &gr, int block, hipStream_t s);
hipError_t launch_fill_many(void *const *ptrs, const int64_t *counts, int narr, int elem_bytes, hipStream_t s);

}  // namespace spic
