// spic_tiled.hip -- tiled fused mover + moment gathering for a species
// that has been sorted by cell (spic_sort.hip).
//
// One workgroup per tile of cells.  The workgroup stages the node fields of
// its region (the tile's cells, `halo` cells around them and the +1 corner
// nodes) in LDS, moves every particle of the tile's range (Eq. 1, Eq. 2,
// Eq. 5) gathering E and B from LDS (Eq. 3, Eq. 4), and deposits the ten
// moments of the moved particle (Sec. II moment equation; Sec. III-B:
// fused, from the new position).  The region's moments are then added to
// the global moments with coalesced global atomics (neighbouring tiles'
// regions overlap).
//
// Deposit.  Rank-major order inside a tile (spic_sort.hip) gives every lane
// of a wave a different cell (and every thread a run of particles from one
// cell), so the 80 FP64 LDS atomics per particle (8 corners x 10 moments)
// of one wave instruction hit distinct words.  The variants (below) differ
// in how they treat particles that have drifted out of their sort cell: in
// LDS, register accumulation of the home cell with a queue of drifted
// particles, or one lane per cell per atomic pass.
//
// LDS layout.  The region slot of a node is di*sx + dj*sy + dk*sz, with the
// strides of a padded layout whose slow axis is the one particles cross most
// often (region_layout): the nodes of a wave's 64 cells fall on distinct
// bank pairs per 16 lanes, and a particle that drifted along the slow axis
// keeps its bank pair.  Fields are node-major (6 values per slot), moments
// component-major ([10][slots]).
//
// Particles whose cell lies outside the region (they drifted farther than
// the halo since the last sort) take the global path for that gather or
// deposit, so the result does not depend on the particle order; the order
// only decides how much work stays in LDS and registers.
//
// Tiles are mapped to workgroups so that the 8 XCDs each take a contiguous
// slab of tiles: workgroup b runs on XCD b % 8, and gets tile
// (b % 8) * chunk + b / 8, keeping a slab's fields and moments in that XCD's
// L2.
#include <hip/hip_runtime.h>

#include "spic_device.h"
#include "spic_impl.h"

namespace spic {

template <typename TP>
struct LdsFieldNode {
    TP v[6];
};

// Location of a point relative to the region.  Returns true when the
// point's cell (with its +1 corners) lies inside the region; `slot` is the
// LDS slot of the cell's lower corner.  When it returns false the global
// cell is in c (base and wrap offsets), otherwise only c.f* are set.
template <typename T>
__device__ __forceinline__ bool region_locate(const GridT<T> &g, const TileGeom &tg, int ox, int oy, int oz, T x,
                                              T y, T z, int &slot, Cell<T> &c, int *ijk = nullptr) {
    const int i = plocate(x, g.L[0], g.invL[0], g.invd[0], g.nx, c.fx);
    const int j = plocate(y, g.L[1], g.invL[1], g.invd[1], g.ny, c.fy);
    const int k = plocate(z, g.L[2], g.invL[2], g.invd[2], g.nz, c.fz);
    if (ijk) {
        ijk[0] = i;
        ijk[1] = j;
        ijk[2] = k;
    }
    int di = i - ox, dj = j - oy, dk = k - oz;
    di += (di < 0) ? g.nx : 0;
    dj += (dj < 0) ? g.ny : 0;
    dk += (dk < 0) ? g.nz : 0;
    slot = di * tg.sx + dj * tg.sy + dk * tg.sz;
    const bool in = di < tg.rx - 1 && dj < tg.ry - 1 && dk < tg.rz - 1;
    if (!in) {
        const int nyz = g.ny * g.nz;
        c.base = i * nyz + j * g.nz + k;
        c.ox = (i == g.nx - 1) ? -(g.nx - 1) * nyz : nyz;
        c.oy = (j == g.ny - 1) ? -(g.ny - 1) * g.nz : g.nz;
        c.oz = (k == g.nz - 1) ? -(g.nz - 1) : 1;
    }
    return in;
}

template <typename TP>
__device__ __forceinline__ void gather_lds(const LdsFieldNode<TP> *__restrict__ fl, const TileGeom &tg, int rb,
                                           const Cell<TP> &c, TP out[6]) {
    TP w[8];
    pweights(c.fx, c.fy, c.fz, w);
    const int sx = tg.sx, sy = tg.sy, sz = tg.sz;
    const int nd[8] = {rb, rb + sx, rb + sy, rb + sx + sy, rb + sz, rb + sx + sz, rb + sy + sz, rb + sx + sy + sz};
#pragma unroll
    for (int m = 0; m < 6; ++m) out[m] = TP(0);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const LdsFieldNode<TP> fn = fl[nd[k]];
#pragma unroll
        for (int m = 0; m < 6; ++m) out[m] += w[k] * fn.v[m];
    }
}

// Ends the data flow of values loaded on a rare path inside that path.
// Without it the compiler may sink the path's last multiply-adds into the
// code both paths share, and the shared code then waits for every
// outstanding global load -- including the next particle's prefetch.
template <typename T, int N>
__device__ __forceinline__ void settle(T (&v)[N]) {
#pragma unroll
    for (int m = 0; m < N; ++m) asm volatile("" : "+v"(v[m]));
}

// Element i of a particle array through a 32-bit byte offset from the
// array base (the host sends only species with n * sizeof(T) < 2^32 here):
// a uniform 64-bit base plus one 32-bit offset per lane, shared by all
// seven arrays.
template <typename T>
__device__ __forceinline__ T ld32(const T *base, uint32_t byte_off) {
    return *(const T *)((const char *)base + byte_off);
}

template <typename T>
__device__ __forceinline__ void st32(T *base, uint32_t byte_off, T v) {
    *(T *)((char *)base + byte_off) = v;
}

// Periodic index o + r with 0 <= o < n, r >= 0: subtract n while needed
// (once, unless the region is wider than the grid).
__device__ __forceinline__ int pwrap_index(int v, int n) {
    while (v >= n) v -= n;
    return v;
}

// Logical region node r -> (ri, rj, rk), its padded LDS slot and its global
// node.
struct RegionNode {
    int slot, gnode;
};

__device__ __forceinline__ RegionNode region_node(const TileGeom &tg, int nx, int ny, int nz, int ox, int oy, int oz,
                                                  int r) {
    const int rzy = tg.ry * tg.rz;
    const int ri = r / rzy;
    const int rem = r - ri * rzy;
    const int rj = rem / tg.rz;
    const int rk = rem - rj * tg.rz;
    RegionNode n;
    n.slot = ri * tg.sx + rj * tg.sy + rk * tg.sz;
    n.gnode = (pwrap_index(ox + ri, nx) * ny + pwrap_index(oy + rj, ny)) * nz + pwrap_index(oz + rk, nz);
    return n;
}

// Ten moments of a particle whose cell left the region: global atomics
// (terms formed in T, added in the accumulation type TA).
template <typename T, typename TA>
__device__ __forceinline__ void deposit_global_cell(const Cell<T> &c, TA *__restrict__ mom, int nn, T qa,
                                                    const T val[10]) {
    T wt8[8];
    pweights(c.fx, c.fy, c.fz, wt8);
    int nd[8];
    pnodes(c, nd);
#pragma unroll 1
    for (int k = 0; k < 8; ++k) {
        const T qw = qa * wt8[k];
        TA *dst = mom + nd[k];
#pragma unroll 1
        for (int m = 0; m < 10; ++m) atomicAdd(dst + (size_t)m * nn, (TA)(qw * val[m]));
    }
}

// Ten moments of one moved particle into the region accumulator with LDS
// atomics, or into the global moments when its cell left the region.
template <typename TA, class GEO>
__device__ __forceinline__ void deposit_one(const GridT<TA> &ga, const TileGeom &tg, int ox, int oy, int oz,
                                            TA *__restrict__ ml, TA *__restrict__ mom, int nn, TA x, TA y, TA z,
                                            TA qa, TA ua, TA va, TA wa) {
    const int RNP = tg.rnp, sx = tg.sx, sy = tg.sy, sz = tg.sz;
    int rb;
    Cell<TA> c;
    const bool in = region_locate(ga, tg, ox, oy, oz, x, y, z, rb, c);
    const TA val[10] = {TA(1), ua, va, wa, ua * ua, ua * va, ua * wa, va * va, va * wa, wa * wa};
    if (in) {
        TA wt8[8];
        pweights(c.fx, c.fy, c.fz, wt8);
        const int coff[8] = {0, sx, sy, sx + sy, sz, sx + sz, sy + sz, sx + sy + sz};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const TA qw = qa * wt8[k];
            TA *dst = ml + rb + coff[k];
#pragma unroll
            for (int m = 0; m < 10; ++m) atomicAdd(dst + m * RNP, qw * val[m]);
        }
    } else {  // rare: the particle left the region
        deposit_global_cell(c, mom, nn, qa, val);
    }
}

// deposit_one with the corner loop rolled and the velocity products formed
// per corner instead of held for all ten moments: few live registers (the
// second pass of the two-phase variants keeps 80 sums live across it).
template <typename TA, class GEO>
__device__ __forceinline__ void deposit_tight(const GridT<TA> &ga, const TileGeom &tg, int ox, int oy, int oz,
                                              TA *__restrict__ ml, TA *__restrict__ mom, int nn, TA x, TA y, TA z,
                                              TA qa, TA ua, TA va, TA wa) {
    const int RNP = tg.rnp, sx = tg.sx, sy = tg.sy, sz = tg.sz;
    int rb;
    Cell<TA> c;
    const bool in = region_locate(ga, tg, ox, oy, oz, x, y, z, rb, c);
    if (in) {
#pragma unroll 1
        for (int k = 0; k < 8; ++k) {
            const TA wx = (k & 1) ? c.fx : TA(1) - c.fx;
            const TA wy = (k & 2) ? c.fy : TA(1) - c.fy;
            const TA wz = (k & 4) ? c.fz : TA(1) - c.fz;
            const TA qw = qa * ((wx * wy) * wz);
            TA *dst = ml + rb + (k & 1) * sx + ((k >> 1) & 1) * sy + (k >> 2) * sz;
            atomicAdd(dst, qw * TA(1));
            atomicAdd(dst + RNP, qw * ua);
            atomicAdd(dst + 2 * RNP, qw * va);
            atomicAdd(dst + 3 * RNP, qw * wa);
            atomicAdd(dst + 4 * RNP, qw * (ua * ua));
            atomicAdd(dst + 5 * RNP, qw * (ua * va));
            atomicAdd(dst + 6 * RNP, qw * (ua * wa));
            atomicAdd(dst + 7 * RNP, qw * (va * va));
            atomicAdd(dst + 8 * RNP, qw * (va * wa));
            atomicAdd(dst + 9 * RNP, qw * (wa * wa));
        }
    } else {
        const TA val[10] = {TA(1), ua, va, wa, ua * ua, ua * va, ua * wa, va * va, va * wa, wa * wa};
        deposit_global_cell(c, mom, nn, qa, val);
    }
}

// deposit_tight with the terms formed in the particle precision T (FP32
// particles: FP32 weights and products, as the register sums of the lane
// cells) and added to the accumulation type TA.
template <typename T, typename TA, class GEO>
__device__ __forceinline__ void deposit_mixed(const GridT<T> &g, const TileGeom &tg, int ox, int oy, int oz,
                                              TA *__restrict__ ml, TA *__restrict__ mom, int nn, T x, T y, T z,
                                              T qa, T ua, T va, T wa) {
    const int RNP = tg.rnp, sx = tg.sx, sy = tg.sy, sz = tg.sz;
    int rb;
    Cell<T> c;
    const bool in = region_locate(g, tg, ox, oy, oz, x, y, z, rb, c);
    const T val[10] = {T(1), ua, va, wa, ua * ua, ua * va, ua * wa, va * va, va * wa, wa * wa};
    if (in) {
#pragma unroll 1
        for (int k = 0; k < 8; ++k) {
            const T wx = (k & 1) ? c.fx : T(1) - c.fx;
            const T wy = (k & 2) ? c.fy : T(1) - c.fy;
            const T wz = (k & 4) ? c.fz : T(1) - c.fz;
            const T qw = qa * ((wx * wy) * wz);
            TA *dst = ml + rb + (k & 1) * sx + ((k >> 1) & 1) * sy + (k >> 2) * sz;
#pragma unroll
            for (int m = 0; m < 10; ++m) atomicAdd(dst + m * RNP, (TA)(qw * val[m]));
        }
    } else {
        deposit_global_cell(c, mom, nn, qa, val);
    }
}

// LDS slot of local cell `lane` of a full tile of 64 cells (the cell a
// rank-major sort puts at that lane of every full rank block), or -1 when
// the tile is ragged or does not hold 64 cells.
__device__ __forceinline__ int lane_cell(const TileGeom &tg, int nx, int ny, int nz, int txi, int tyi, int tzi,
                                         int lane) {
    const int t3[3] = {tg.tx, tg.ty, tg.tz};
    const int ext[3] = {min(tg.tx, nx - txi * tg.tx), min(tg.ty, ny - tyi * tg.ty), min(tg.tz, nz - tzi * tg.tz)};
    if (tg.cells != 64 || ext[0] != t3[0] || ext[1] != t3[1] || ext[2] != t3[2]) return -1;
    int loc[3];
    loc[tg.fast] = lane % t3[tg.fast];
    loc[tg.mid] = (lane / t3[tg.fast]) % t3[tg.mid];
    loc[tg.slow] = lane / (t3[tg.fast] * t3[tg.mid]);
    return (tg.halo + loc[0]) * tg.sx + (tg.halo + loc[1]) * tg.sy + (tg.halo + loc[2]) * tg.sz;
}

// Orders one wave's LDS accesses across lanes (a wave's LDS operations are
// processed in issue order; this keeps the compiler from reordering them).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A moved particle staged in LDS (variants 2 and 3).
template <typename TP>
struct StagedParticle {
    TP x, y, z, u, v, w, q, pad;
};

// Variant 3: bank-balanced deposit.  An FP64 LDS access by 16 consecutive
// lanes is conflict free when their slots differ modulo 16; the rank-major
// order gives that for particles still in their sort cells, but drifted
// particles land on the bank pairs of their neighbours (measured: 8 clk per
// atomic instruction without drift, 22-28 clk with a quarter to half of the
// lanes drifted).  Before its 80 atomics a wave therefore re-places its
// moved particles: the r-th particle (r < 4) whose slot is b modulo 16 goes
// to lane 16 r + b, so each group of 16 lanes holds distinct bank pairs;
// the rest fill the lanes left empty.  All 64 lanes must be active.
struct BalanceLds {
    int count[16];  // particles per bank pair
    int hole[64];   // lanes left empty, in lane order
};

// TIGHT picks deposit_tight (corner loop rolled, few live registers) for the
// deposit of the re-placed particles.
template <typename TP, typename TA, class GEO, bool TIGHT = false>
__device__ __forceinline__ void deposit_balanced(const GridT<TA> &ga, const TileGeom &tg, int ox, int oy, int oz,
                                                 TA *__restrict__ ml, TA *__restrict__ mom, int nn,
                                                 StagedParticle<TP> *__restrict__ stage, BalanceLds *__restrict__ bl,
                                                 int lane, bool valid, TP x, TP y, TP z, TP u, TP v, TP w, TP q) {
    int rb = 0;
    bool rec = false;
    if (valid) {
        Cell<TA> c;
        rec = region_locate(ga, tg, ox, oy, oz, (TA)x, (TA)y, (TA)z, rb, c);
        if (!rec)  // rare: outside the region, straight to the global moments
            deposit_one<TA, GEO>(ga, tg, ox, oy, oz, ml, mom, nn, (TA)x, (TA)y, (TA)z, (TA)q, (TA)u, (TA)v, (TA)w);
    }
    if (lane < 16) bl->count[lane] = 0;
    wave_sync();
    const int b = rb & 15;
    int r = 0;
    if (rec) r = (int)atomicAdd(&bl->count[b], 1);
    wave_sync();
    StagedParticle<TP> me;
    me.x = x; me.y = y; me.z = z; me.u = u; me.v = v; me.w = w; me.q = q; me.pad = TP(0);
    const bool primary = rec && r < 4;
    const bool over = rec && r >= 4;
    if (primary) stage[16 * r + b] = me;
    // lane l is filled by a primary particle iff bank pair l % 16 has more than l / 16 of them
    const bool hole = bl->count[lane & 15] <= (lane >> 4);
    const unsigned long long hmask = __ballot(hole), omask = __ballot(over);
    const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int h = __popcll(hmask & below), k = __popcll(omask & below);
    if (hole) bl->hole[h] = lane;
    wave_sync();
    if (over) stage[bl->hole[k]] = me;
    wave_sync();
    if (!hole || h < __popcll(omask)) {
        const StagedParticle<TP> s = stage[lane];
        if constexpr (TIGHT)
            deposit_tight<TA, GEO>(ga, tg, ox, oy, oz, ml, mom, nn, (TA)s.x, (TA)s.y, (TA)s.z, (TA)s.q, (TA)s.u,
                                   (TA)s.v, (TA)s.w);
        else
            deposit_one<TA, GEO>(ga, tg, ox, oy, oz, ml, mom, nn, (TA)s.x, (TA)s.y, (TA)s.z, (TA)s.q, (TA)s.u,
                                 (TA)s.v, (TA)s.w);
    }
    wave_sync();  // the stage is rewritten by the next call
}

// Variant 4: segmented wave pre-reduction of the deposit.  In cell-major
// order a wave's lanes mostly hold particles of one cell; lanes whose moved
// particles sit in the same region cell, in consecutive lanes, form a
// segment, and the 80 contributions (8 corners x 10 moments) are summed
// over each segment by an inclusive segmented scan across the wave (DPP row
// shifts and row broadcasts, FP64), after which only each segment's last
// lane issues the LDS atomics: 80 atomic instructions per wave, each with a
// handful of active lanes on distinct words, instead of 80 per particle
// lane with bank conflicts.  All 64 lanes must be active.
namespace seg {
// DPP controls (GFX9 encoding): row shift right by 1/2/4/8 lanes, and the
// broadcasts of lane 15 of each row to the next row / of lane 31 to rows 2-3
constexpr int kShr1 = 0x111, kShr2 = 0x112, kShr4 = 0x114, kShr8 = 0x118, kBcast15 = 0x142, kBcast31 = 0x143;
constexpr int kWaveShr1 = 0x138;  // whole-wave shift right by one lane

template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Which of the six scan steps may add the source lane's partial sum: the
// source lane lies in this lane's segment.
struct Steps {
    bool s1, s2, s4, s8, b15, b31;
};

__device__ __forceinline__ Steps steps_for(int lane, int start) {
    Steps t;
    const int r = lane & 15, row = lane >> 4;
    t.s1 = r >= 1 && lane - 1 >= start;
    t.s2 = r >= 2 && lane - 2 >= start;
    t.s4 = r >= 4 && lane - 4 >= start;
    t.s8 = r >= 8 && lane - 8 >= start;
    t.b15 = (row == 1 || row == 3) && 16 * row - 1 >= start;
    t.b31 = row >= 2 && 31 >= start;
    return t;
}

// Inclusive segmented scan of N values at once (N independent chains keep
// the VALU busy between the dependent DPP steps).
template <int N>
__device__ __forceinline__ void scan(double (&v)[N], const Steps &t) {
    double x[N];
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = dpp<kShr1, 0xF>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += t.s1 ? x[i] : 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = dpp<kShr2, 0xF>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += t.s2 ? x[i] : 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = dpp<kShr4, 0xF>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += t.s4 ? x[i] : 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = dpp<kShr8, 0xF>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += t.s8 ? x[i] : 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = dpp<kBcast15, 0xA>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += t.b15 ? x[i] : 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = dpp<kBcast31, 0xC>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += t.b31 ? x[i] : 0.0;
}
}  // namespace seg

template <typename TA, class GEO>
__device__ __forceinline__ void deposit_segmented(const GridT<TA> &ga, const TileGeom &tg, int ox, int oy, int oz,
                                                  TA *__restrict__ ml, TA *__restrict__ mom, int nn, int lane,
                                                  bool valid, TA x, TA y, TA z, TA qa, TA ua, TA va, TA wa) {
    const int RNP = tg.rnp, sx = tg.sx, sy = tg.sy, sz = tg.sz;
    int rb = 0;
    Cell<TA> c;
    c.fx = c.fy = c.fz = TA(0);
    bool in = false;
    if (valid) {
        in = region_locate(ga, tg, ox, oy, oz, x, y, z, rb, c);
        if (!in)  // rare: outside the region, straight to the global moments
            deposit_one<TA, GEO>(ga, tg, ox, oy, oz, ml, mom, nn, x, y, z, qa, ua, va, wa);
    }
    // segments: runs of consecutive lanes in the same region cell; lanes
    // without an LDS deposit get a key of their own
    const int key = in ? rb : -1 - lane;
    const int left = __builtin_amdgcn_update_dpp(-1 - 64, key, seg::kWaveShr1, 0xF, 0xF, false);
    const unsigned long long heads = __ballot(lane == 0 || left != key);
    const unsigned long long upto = heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1));
    const int start = 63 - __clzll(upto);
    const bool tail = lane == 63 || ((heads >> (lane + 1)) & 1ull);
    const seg::Steps st = seg::steps_for(lane, start);
    TA wt8[8];
    pweights(c.fx, c.fy, c.fz, wt8);
    const TA q0 = in ? qa : TA(0);
    const TA val[10] = {TA(1), ua, va, wa, ua * ua, ua * va, ua * wa, va * va, va * wa, wa * wa};
    const int coff[8] = {0, sx, sy, sx + sy, sz, sx + sz, sy + sz, sx + sy + sz};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const TA qw = q0 * wt8[k];
        double sum[10];
#pragma unroll
        for (int m = 0; m < 10; ++m) sum[m] = (double)(qw * val[m]);
        seg::scan(sum, st);
        if (in && tail) {
#pragma unroll
            for (int m = 0; m < 10; ++m) atomicAdd(ml + rb + coff[k] + m * RNP, (TA)sum[m]);
        }
    }
}

// LDS bytes of the per-wave staging of variants 2 (queue) and 3 (balance).
constexpr int kQueueCap = 128;  // variant 2: at most 63 wait between drains, one iteration adds <= 64
inline size_t stage_lds_bytes(int variant, int block, int dtype) {
    const size_t rec = 8 * (dtype == SPIC_F64 ? 8 : 4);
    if (variant == 2) return (size_t)(block / 64) * kQueueCap * rec;
    if (variant == 3) return (size_t)(block / 64) * (64 * rec + sizeof(BalanceLds));
    if (variant == 5 || variant == 7 || variant == 9)  // queue, reused as the balancing stage when flushed
        return (size_t)(block / 64) * (64 * rec + sizeof(BalanceLds));
    if (variant == 8)  // the deposit kernel: queue and balancing stage side by side
        return (size_t)(block / 64) * (64 * 7 * (rec / 8) + 64 * rec + sizeof(BalanceLds));
    if (variant == 6) return (size_t)(block / 64) * 64 * 7 * (dtype == SPIC_F64 ? 8 : 4);
    return 0;
}

// One tile of one species: stage the region, move and deposit the tile's
// particles, flush the region's moments.  Called by the per-species tiled
// kernel and by the work-list kernel of the batch engine; `t` is uniform
// across the workgroup.  The particle loop is uniform per wave (lanes past
// the end of the range idle), so wave-wide votes are safe inside it.
template <typename TP, typename TF, typename TA, int VAR, class GEO>
__device__ __forceinline__ void tile_body(const TileJob<TP, TF, TA> &J, int t, unsigned char *smem) {
    constexpr bool HOME = VAR == 2;   // home-cell registers + queue of drifted particles
    constexpr bool CACHE = VAR == 1;  // field corners of the last cell in registers
    constexpr bool BAL = VAR == 3;    // bank-balanced deposit
    constexpr bool SEG = VAR == 4;    // segmented wave pre-reduction of the deposit
    constexpr bool LANE = VAR == 5 || VAR == 7;  // lane-cell registers in particle precision + compact queue
    constexpr bool AUX = VAR == 7;    // + a second register set for the first cell a lane's particles drift to
    constexpr bool SPLIT = VAR == 6;  // as 5, with the deposit in a second pass over the moved particles
    const GridT<TP> &g = J.g;
    TileGeom tg = J.tg;
    if constexpr (GEO::fixed) {  // the host launches this only for a matching tiling
        tg.tx = GEO::tx; tg.ty = GEO::ty; tg.tz = GEO::tz; tg.halo = GEO::halo;
        tg.rx = GEO::rx; tg.ry = GEO::ry; tg.rz = GEO::rz;
        tg.slow = GEO::slow; tg.mid = GEO::mid; tg.fast = GEO::fast;
        tg.sx = GEO::sx; tg.sy = GEO::sy; tg.sz = GEO::sz; tg.rnp = GEO::rnp;
    }
    const FieldPtrs<TF> &f = J.f;
    const PartPtrs<TP> &p = J.p;
    TA *__restrict__ mom = J.mom;
    const int nn = J.nn;
    const uint32_t beg = J.tile_off[t], end = J.tile_off[t + 1];
    if (beg == end) return;  // uniform: no particle in this tile

    const int RNP = tg.rnp;
    const size_t fbytes = (RNP * sizeof(LdsFieldNode<TP>) + 15) & ~(size_t)15;
    LdsFieldNode<TP> *fl = (LdsFieldNode<TP> *)smem;
    TA *ml = (TA *)(smem + fbytes);
    const int tzi = t % tg.ntz, tyi = (t / tg.ntz) % tg.nty, txi = t / (tg.ntz * tg.nty);
    int ox = (txi * tg.tx - tg.halo) % g.nx; ox += ox < 0 ? g.nx : 0;
    int oy = (tyi * tg.ty - tg.halo) % g.ny; oy += oy < 0 ? g.ny : 0;
    int oz = (tzi * tg.tz - tg.halo) % g.nz; oz += oz < 0 ? g.nz : 0;
    const int RL = tg.rx * tg.ry * tg.rz;  // logical region nodes
    const int sx = tg.sx, sy = tg.sy, sz = tg.sz;

    // stage the region's node fields, zero the region's moments
    for (int r = threadIdx.x; r < RL; r += blockDim.x) {
        const RegionNode rn = region_node(tg, g.nx, g.ny, g.nz, ox, oy, oz, r);
        LdsFieldNode<TP> fn;
#pragma unroll
        for (int m = 0; m < 6; ++m) fn.v[m] = (TP)f.f[m][rn.gnode];
        fl[rn.slot] = fn;
    }
    if (mom)
        for (int q = threadIdx.x; q < 10 * RNP; q += blockDim.x) ml[q] = TA(0);
    __syncthreads();

    const int coff[8] = {0, sx, sy, sx + sy, sz, sx + sz, sy + sz, sx + sy + sz};
    TA acc[HOME ? 80 : 1];
#pragma unroll
    for (int q = 0; q < (HOME ? 80 : 1); ++q) acc[q] = TA(0);
    int home = -1;
    LdsFieldNode<TP> corner[CACHE ? 8 : 1];  // field corners of the cell `cached`
    int cached = -1;
    // per-wave staging after the moments: variant 2's queue of drifted
    // particles (a stack of qn records), variant 3's balance buffers
    unsigned char *wstage = smem + fbytes + (((size_t)10 * RNP * sizeof(TA) + 15) & ~(size_t)15);
    StagedParticle<TP> *queue = nullptr;
    int qn = 0;  // uniform across the wave
    if constexpr (HOME) queue = (StagedParticle<TP> *)wstage + (threadIdx.x >> 6) * kQueueCap;
    StagedParticle<TP> *stage = nullptr;
    BalanceLds *bal = nullptr;
    if constexpr (BAL) {
        unsigned char *mine = wstage + (threadIdx.x >> 6) * (64 * sizeof(StagedParticle<TP>) + sizeof(BalanceLds));
        stage = (StagedParticle<TP> *)mine;
        bal = (BalanceLds *)(mine + 64 * sizeof(StagedParticle<TP>));
    }
    const int lane = threadIdx.x & 63;
    // variant 5: lane l of every full rank block holds a particle sorted
    // into local cell l, so lane l keeps the moments of that cell's 8 nodes
    // in registers (particle precision) and queues the particles that left
    // it; lcell = -1 where the tile is ragged or not 64 cells
    TP lacc[LANE ? 80 : 1];
#pragma unroll
    for (int q = 0; q < (LANE ? 80 : 1); ++q) lacc[q] = TP(0);
    int lcell = -1;
    // variant 7: the sheet species drift coherently across one face of
    // their cells, so a lane's drifted particles mostly share one cell: the
    // first one names it (acell) and those that follow it accumulate in a
    // second register set
    TP xacc[AUX ? 80 : 1];
#pragma unroll
    for (int q = 0; q < (AUX ? 80 : 1); ++q) xacc[q] = TP(0);
    int acell = -1;
    TP *lq = nullptr;  // per-wave queue, 7 arrays of 64 (x y z u v w q)
    StagedParticle<TP> *lstage = nullptr;  // the same bytes while the queue is deposited
    BalanceLds *lbal = nullptr;
    if constexpr (LANE) {
        unsigned char *mine = wstage + (threadIdx.x >> 6) * (64 * sizeof(StagedParticle<TP>) + sizeof(BalanceLds));
        lq = (TP *)mine;
        lstage = (StagedParticle<TP> *)mine;
        lbal = (BalanceLds *)(mine + 64 * sizeof(StagedParticle<TP>));
        lcell = lane_cell(tg, g.nx, g.ny, g.nz, txi, tyi, tzi, lane);
    }

    const uint32_t stride = blockDim.x;
    constexpr uint32_t ES = sizeof(TP);
    uint32_t i = beg + threadIdx.x;
    TP nx_ = 0, ny_ = 0, nz_ = 0, nu_ = 0, nv_ = 0, nw_ = 0, nq_ = 0;
    int64_t nid_ = 0;
    const PartPtrs<TP> &pin = J.in;
    const bool copy_id = J.copy_rest && pin.id;  // ids move with the sort's copy
    if (i < end) {
        const uint32_t o = i * ES;
        nx_ = ld32(pin.x, o); ny_ = ld32(pin.y, o); nz_ = ld32(pin.z, o);
        nu_ = ld32(pin.u, o); nv_ = ld32(pin.v, o); nw_ = ld32(pin.w, o); nq_ = ld32(pin.q, o);
        if (copy_id) nid_ = pin.id[i];
    }
    // uniform per wave: the first index of this wave's lane 0
    for (uint32_t i0 = beg + (threadIdx.x & ~63u); i0 < end; i0 += stride, i += stride) {
        const bool valid = i < end;
        TP xn = nx_, yn = ny_, zn = nz_, un = nu_, vn = nv_, wn = nw_;
        const TP qp = nq_;
        const int64_t idp = nid_;
        const uint32_t inext = i + stride;
        if (inext < end) {  // prefetch the next particle while this one is moved
            const uint32_t o = inext * ES;
            nx_ = ld32(pin.x, o); ny_ = ld32(pin.y, o); nz_ = ld32(pin.z, o);
            nu_ = ld32(pin.u, o); nv_ = ld32(pin.v, o); nw_ = ld32(pin.w, o); nq_ = ld32(pin.q, o);
            if (copy_id) nid_ = pin.id[inext];
        }
        bool enq = false;
        if (valid) {
            // the cell located by the first gather of this particle; later
            // gathers inside it reuse it (same result as locating again)
            int c_ijk[3] = {-1, 0, 0}, c_rb = 0;
            bool c_in = false;
            Cell<TP> c_cell;
            implicit_move(
                g, J.mv,
                [&](TP px, TP py, TP pz, TP F[6]) {
                    int rb;
                    Cell<TP> c;
                    bool in;
                    const TP tx = cell_coord(px, g.invd[0]) - (TP)c_ijk[0];
                    const TP ty = cell_coord(py, g.invd[1]) - (TP)c_ijk[1];
                    const TP tz = cell_coord(pz, g.invd[2]) - (TP)c_ijk[2];
                    if (c_ijk[0] >= 0 && px >= TP(0) && px < g.L[0] && py >= TP(0) && py < g.L[1] &&
                        pz >= TP(0) && pz < g.L[2] && tx >= TP(0) && tx < TP(1) && ty >= TP(0) && ty < TP(1) &&
                        tz >= TP(0) && tz < TP(1)) {
                        c = c_cell;
                        c.fx = tx;
                        c.fy = ty;
                        c.fz = tz;
                        rb = c_rb;
                        in = c_in;
                    } else {
                        in = region_locate(g, tg, ox, oy, oz, px, py, pz, rb, c, c_ijk);
                        if (in) {  // the global cell is needed only outside the region
                            c.base = 0; c.ox = 0; c.oy = 0; c.oz = 0;
                        }
                        c_cell = c;
                        c_rb = rb;
                        c_in = in;
                    }
                    if (in) {
                        if (!CACHE) {
                            gather_lds(fl, tg, rb, c, F);
                        } else {
                            // the corners of the last LDS cell stay in
                            // registers: a thread's particles share their sort cell
                            if (rb != cached) {
#pragma unroll
                                for (int k = 0; k < 8; ++k) corner[k] = fl[rb + coff[k]];
                                cached = rb;
                            }
                            TP w[8];
                            pweights(c.fx, c.fy, c.fz, w);
#pragma unroll
                            for (int m = 0; m < 6; ++m) F[m] = TP(0);
#pragma unroll
                            for (int k = 0; k < 8; ++k)
#pragma unroll
                                for (int m = 0; m < 6; ++m) F[m] += w[k] * corner[k].v[m];
                        }
                    } else {
                        gather_cell_global(f, c, F);
                        settle(*(TP(*)[6])F);
                    }
                },
                xn, yn, zn, un, vn, wn);
            const uint32_t o = i * ES;
            st32(p.x, o, xn); st32(p.y, o, yn); st32(p.z, o, zn);
            st32(p.u, o, un); st32(p.v, o, vn); st32(p.w, o, wn);
            if (J.copy_rest) {  // reading the sort's copy: q and id move too
                st32(p.q, o, qp);
                if (copy_id) p.id[i] = idp;
            }

            if (!SPLIT && mom) {
                // deposit of the new state in the accumulation precision
                const TA qa = (TA)qp;
                const TA ua = (TA)un, va = (TA)vn, wa = (TA)wn;
                if constexpr (HOME) {
                    int rb;
                    Cell<TA> c;
                    const bool in = region_locate(J.ga, tg, ox, oy, oz, (TA)xn, (TA)yn, (TA)zn, rb, c);
                    if (in && home < 0) home = rb;
                    if (in && rb == home) {
                        TA wt8[8];
                        pweights(c.fx, c.fy, c.fz, wt8);
                        const TA val[10] = {TA(1), ua, va, wa, ua * ua, ua * va, ua * wa, va * va, va * wa, wa * wa};
#pragma unroll
                        for (int k = 0; k < 8; ++k) {
                            const TA qw = qa * wt8[k];
#pragma unroll
                            for (int m = 0; m < 10; ++m) acc[(k * 10 + m) % (HOME ? 80 : 1)] += qw * val[m];
                        }
                    } else {
                        enq = true;  // another cell, or outside the region
                    }
                } else if constexpr (LANE) {
                    // cell and weights from the position in the accumulation
                    // precision (the cell-relative coordinate of an FP32
                    // position loses ~ulp(x)/dx in FP32), the weighted charge
                    // then rounded once to the particle precision
                    int rb;
                    Cell<TA> c;
                    const bool in = region_locate(J.ga, tg, ox, oy, oz, (TA)xn, (TA)yn, (TA)zn, rb, c);
                    if (AUX && in && lcell >= 0 && rb != lcell && acell < 0) acell = rb;
                    if (in && rb == lcell) {
                        TA wt8[8];
                        pweights(c.fx, c.fy, c.fz, wt8);
                        const TP val[10] = {TP(1), un, vn, wn, un * un, un * vn, un * wn, vn * vn, vn * wn, wn * wn};
#pragma unroll
                        for (int k = 0; k < 8; ++k) {
                            const TP qw = (TP)(qa * wt8[k]);
#pragma unroll
                            for (int m = 0; m < 10; ++m) lacc[(k * 10 + m) % (LANE ? 80 : 1)] += qw * val[m];
                        }
                    } else if (AUX && in && rb == acell) {
                        TA wt8[8];
                        pweights(c.fx, c.fy, c.fz, wt8);
                        const TP val[10] = {TP(1), un, vn, wn, un * un, un * vn, un * wn, vn * vn, vn * wn, wn * wn};
#pragma unroll
                        for (int k = 0; k < 8; ++k) {
                            const TP qw = (TP)(qa * wt8[k]);
#pragma unroll
                            for (int m = 0; m < 10; ++m) xacc[(k * 10 + m) % (AUX ? 80 : 1)] += qw * val[m];
                        }
                    } else {
                        enq = true;
                    }
                } else if constexpr (!BAL && !SEG) {
                    deposit_one<TA, GEO>(J.ga, tg, ox, oy, oz, ml, mom, nn, (TA)xn, (TA)yn, (TA)zn, qa, ua, va, wa);
                }
            }
        }
        if constexpr (BAL) {
            if (mom)
                deposit_balanced<TP, TA, GEO>(J.ga, tg, ox, oy, oz, ml, mom, nn, stage, bal, lane, valid, xn, yn, zn,
                                              un, vn, wn, qp);
        }
        if constexpr (SEG) {
            if (mom)
                deposit_segmented<TA, GEO>(J.ga, tg, ox, oy, oz, ml, mom, nn, lane, valid, (TA)xn, (TA)yn, (TA)zn,
                                           (TA)qp, (TA)un, (TA)vn, (TA)wn);
        }
        if constexpr (LANE) {
            // queue the particles that left their lane's cell; whenever 64
            // wait, deposit them with every lane active.  The queue holds
            // 64: lanes past it wait until the full queue has been read.
            const unsigned long long vote = __ballot(enq);
            if (vote) {
                const int cnt = __popcll(vote);
                const int pos = qn + __popcll(vote & ((1ull << lane) - 1ull));
                const TP rec[7] = {xn, yn, zn, un, vn, wn, qp};
                if (enq && pos < 64)
#pragma unroll
                    for (int a = 0; a < 7; ++a) lq[a * 64 + pos] = rec[a];
                if (qn + cnt >= 64) {
                    // deposit the 64 queued particles re-placed across the
                    // lanes so that each 16-lane group hits distinct bank
                    // pairs (they sit in arbitrary cells), then queue the
                    // lanes that did not fit
                    wave_sync();
                    TP r[7];
#pragma unroll
                    for (int a = 0; a < 7; ++a) r[a] = lq[a * 64 + lane];
                    wave_sync();
                    deposit_balanced<TP, TA, GEO>(J.ga, tg, ox, oy, oz, ml, mom, nn, lstage, lbal, lane, true,
                                                        r[0], r[1], r[2], r[3], r[4], r[5], r[6]);
                    if (enq && pos >= 64)
#pragma unroll
                        for (int a = 0; a < 7; ++a) lq[a * 64 + pos - 64] = rec[a];
                    qn += cnt - 64;
                } else {
                    qn += cnt;
                }
            }
        }
        if constexpr (HOME) {
            // queue the drifted particles of this iteration; once 64 wait,
            // deposit them with every lane active
            const unsigned long long vote = __ballot(enq);
            if (vote) {
                const unsigned long long below = lane ? (vote & (~0ull >> (64 - lane))) : 0ull;
                if (enq) {
                    StagedParticle<TP> r;
                    r.x = xn; r.y = yn; r.z = zn; r.u = un; r.v = vn; r.w = wn; r.q = qp; r.pad = TP(0);
                    queue[qn + __popcll(below)] = r;
                }
                qn += __popcll(vote);
                if (qn >= 64) {
                    // the records written above by other lanes of this wave
                    // are visible after a wave-scope fence
                    wave_sync();
                    qn -= 64;
                    const StagedParticle<TP> r = queue[qn + lane];
                    wave_sync();
                    deposit_one<TA, GEO>(J.ga, tg, ox, oy, oz, ml, mom, nn, (TA)r.x, (TA)r.y, (TA)r.z, (TA)r.q,
                                         (TA)r.u, (TA)r.v, (TA)r.w);
                }
            }
        }
    }
    if (!mom) return;
    if constexpr (SPLIT) {
        // second pass: each thread re-reads the particles it moved (its own
        // stores, same indices), so no barrier is needed; the mover's
        // registers are dead here, leaving room for the 80 lane-cell sums
        const int lc = lane_cell(tg, g.nx, g.ny, g.nz, txi, tyi, tzi, lane);
        TP sacc[SPLIT ? 80 : 1];
#pragma unroll
        for (int q = 0; q < (SPLIT ? 80 : 1); ++q) sacc[q] = TP(0);
        TP *sq = (TP *)wstage + (threadIdx.x >> 6) * (7 * 64);
        int sqn = 0;
        uint32_t ii = beg + threadIdx.x;
        for (uint32_t i0 = beg + (threadIdx.x & ~63u); i0 < end; i0 += stride, ii += stride) {
            const bool valid = ii < end;
            bool enq = false;
            TP rec[7] = {TP(0), TP(0), TP(0), TP(0), TP(0), TP(0), TP(0)};  // x y z u v w q
            if (valid) {
                const uint32_t o = ii * ES;
                rec[0] = ld32(p.x, o); rec[1] = ld32(p.y, o); rec[2] = ld32(p.z, o);
                rec[3] = ld32(p.u, o); rec[4] = ld32(p.v, o); rec[5] = ld32(p.w, o); rec[6] = ld32(p.q, o);
                // cell and weights in the accumulation precision, as in
                // variant 5
                int rb;
                Cell<TA> c;
                const bool in = region_locate(J.ga, tg, ox, oy, oz, (TA)rec[0], (TA)rec[1], (TA)rec[2], rb, c);
                if (in && rb == lc) {
                    TA wt8[8];
                    pweights(c.fx, c.fy, c.fz, wt8);
                    const TP u = rec[3], v = rec[4], w = rec[5];
                    const TP val[10] = {TP(1), u, v, w, u * u, u * v, u * w, v * v, v * w, w * w};
                    const TA qa6 = (TA)rec[6];
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const TP qw = (TP)(qa6 * wt8[k]);
#pragma unroll
                        for (int m = 0; m < 10; ++m) sacc[(k * 10 + m) % (SPLIT ? 80 : 1)] += qw * val[m];
                    }
                } else {
                    enq = true;
                }
            }
            const unsigned long long vote = __ballot(enq);
            if (vote) {
                const int cnt = __popcll(vote);
                const int pos = sqn + __popcll(vote & ((1ull << lane) - 1ull));
                if (enq && pos < 64)
#pragma unroll
                    for (int a = 0; a < 7; ++a) sq[a * 64 + pos] = rec[a];
                if (sqn + cnt >= 64) {
                    wave_sync();
                    TP r[7];
#pragma unroll
                    for (int a = 0; a < 7; ++a) r[a] = sq[a * 64 + lane];
                    wave_sync();
                    if (enq && pos >= 64)
#pragma unroll
                        for (int a = 0; a < 7; ++a) sq[a * 64 + pos - 64] = rec[a];
                    deposit_tight<TA, GEO>(J.ga, tg, ox, oy, oz, ml, mom, nn, (TA)r[0], (TA)r[1], (TA)r[2],
                                          (TA)r[6], (TA)r[3], (TA)r[4], (TA)r[5]);
                    sqn += cnt - 64;
                } else {
                    sqn += cnt;
                }
            }
        }
        wave_sync();
        if (lane < sqn) {
            TP r[7];
#pragma unroll
            for (int a = 0; a < 7; ++a) r[a] = sq[a * 64 + lane];
            deposit_tight<TA, GEO>(J.ga, tg, ox, oy, oz, ml, mom, nn, (TA)r[0], (TA)r[1], (TA)r[2], (TA)r[6],
                                  (TA)r[3], (TA)r[4], (TA)r[5]);
        }
        // the sums stay in the particle precision until here (without the
        // barrier the compiler widens them early on the zero-trip path)
        settle(sacc);
        if (lc >= 0) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                TA *dst = ml + lc + coff[k];
#pragma unroll
                for (int m = 0; m < 10; ++m) atomicAdd(dst + m * RNP, (TA)sacc[(k * 10 + m) % (SPLIT ? 80 : 1)]);
            }
        }
    }
    if constexpr (LANE) {
        wave_sync();
        TP r[7] = {TP(0), TP(0), TP(0), TP(0), TP(0), TP(0), TP(0)};
        if (lane < qn)
#pragma unroll
            for (int a = 0; a < 7; ++a) r[a] = lq[a * 64 + lane];
        wave_sync();
        if (qn > 0)  // uniform
            deposit_balanced<TP, TA, GEO>(J.ga, tg, ox, oy, oz, ml, mom, nn, lstage, lbal, lane, lane < qn, r[0],
                                                r[1], r[2], r[3], r[4], r[5], r[6]);
        settle(lacc);
        if (lcell >= 0) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                TA *dst = ml + lcell + coff[k];
#pragma unroll
                for (int m = 0; m < 10; ++m) atomicAdd(dst + m * RNP, (TA)lacc[(k * 10 + m) % (LANE ? 80 : 1)]);
            }
        }
        if constexpr (AUX) {
            settle(xacc);
            if (acell >= 0) {
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    TA *dst = ml + acell + coff[k];
#pragma unroll
                    for (int m = 0; m < 10; ++m) atomicAdd(dst + m * RNP, (TA)xacc[(k * 10 + m) % (AUX ? 80 : 1)]);
                }
            }
        }
    }
    if constexpr (HOME) {
        wave_sync();
        if (lane < qn) {
            const StagedParticle<TP> r = queue[lane];
            deposit_one<TA, GEO>(J.ga, tg, ox, oy, oz, ml, mom, nn, (TA)r.x, (TA)r.y, (TA)r.z, (TA)r.q, (TA)r.u,
                                 (TA)r.v, (TA)r.w);
        }
        if (home >= 0) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                TA *dst = ml + home + coff[k];
#pragma unroll
                for (int m = 0; m < 10; ++m) atomicAdd(dst + m * RNP, acc[(k * 10 + m) % (HOME ? 80 : 1)]);
            }
        }
    }
    __syncthreads();
    // flush: region accumulator -> global moments (skip exact zeros: halo
    // nodes no particle reached); consecutive threads take consecutive region
    // nodes, so each moment's atomics are coalesced along z
    for (int r = threadIdx.x; r < RL; r += blockDim.x) {
        const RegionNode rn = region_node(tg, g.nx, g.ny, g.nz, ox, oy, oz, r);
#pragma unroll
        for (int m = 0; m < 10; ++m) {
            const TA val = ml[m * RNP + rn.slot];
            if (val != TA(0)) atomicAdd(mom + (size_t)m * nn + rn.gnode, val);
        }
    }
}

// Variant 9: variant 5 with two particles per thread in flight.  At the two
// waves per SIMD that variant 5's LDS allows, a lone particle's chain of
// three dependent LDS gathers leaves the SIMD idle; here each thread moves
// the particles i and i + B (B threads, the same lane of the next rank
// block: the same sort cell) together, so the gathers and rotations of the
// two are interleaved.  Deposit as variant 5 (lane-cell registers, queue
// deposited bank-balanced).
template <typename TP>
struct CellCache {
    int ijk[3];
    int rb;
    bool in;
    Cell<TP> c;
};

// Cell of a point for an LDS gather: the cached cell when the point is still
// inside it (exactly the offsets a fresh locate gives), else a new locate.
template <typename TP>
__device__ __forceinline__ bool pair_locate(const GridT<TP> &g, const TileGeom &tg, int ox, int oy, int oz, TP px,
                                            TP py, TP pz, CellCache<TP> &cc, int &rb, Cell<TP> &c) {
    const TP tx = cell_coord(px, g.invd[0]) - (TP)cc.ijk[0];
    const TP ty = cell_coord(py, g.invd[1]) - (TP)cc.ijk[1];
    const TP tz = cell_coord(pz, g.invd[2]) - (TP)cc.ijk[2];
    if (cc.ijk[0] >= 0 && px >= TP(0) && px < g.L[0] && py >= TP(0) && py < g.L[1] && pz >= TP(0) &&
        pz < g.L[2] && tx >= TP(0) && tx < TP(1) && ty >= TP(0) && ty < TP(1) && tz >= TP(0) && tz < TP(1)) {
        c = cc.c;
        c.fx = tx;
        c.fy = ty;
        c.fz = tz;
        rb = cc.rb;
        return cc.in;
    }
    const bool in = region_locate(g, tg, ox, oy, oz, px, py, pz, rb, c, cc.ijk);
    if (in) {
        c.base = 0; c.ox = 0; c.oy = 0; c.oz = 0;
    }
    cc.c = c;
    cc.rb = rb;
    cc.in = in;
    return in;
}

template <typename TP>
__device__ __forceinline__ void pair_rotate(const MoveT<TP> &mv, const TP F[6], TP x0, TP y0, TP z0, TP u0, TP v0,
                                            TP w0, TP &ub, TP &vb, TP &wb, TP &xb, TP &yb, TP &zb) {
    const TP ut = u0 + mv.beta * F[0];
    const TP vt = v0 + mv.beta * F[1];
    const TP wt = w0 + mv.beta * F[2];
    const TP bx = mv.bc * F[3], by = mv.bc * F[4], bz = mv.bc * F[5];
    const TP vdb = ut * bx + vt * by + wt * bz;
    const TP inv = recip_ge1(TP(1) + (bx * bx + by * by + bz * bz));
    ub = (ut + (vt * bz - wt * by) + vdb * bx) * inv;
    vb = (vt + (wt * bx - ut * bz) + vdb * by) * inv;
    wb = (wt + (ut * by - vt * bx) + vdb * bz) * inv;
    xb = x0 + ub * mv.hdt;
    yb = y0 + vb * mv.hdt;
    zb = z0 + wb * mv.hdt;
}

// The implicit step (same arithmetic as implicit_move) of two particles in
// lock-step; `s[0..5]` = x y z u v w of each, updated in place.
template <typename TP, typename TF>
__device__ __forceinline__ void pair_move(const GridT<TP> &g, const MoveT<TP> &mv, const FieldPtrs<TF> &f,
                                          const LdsFieldNode<TP> *__restrict__ fl, const TileGeom &tg, int ox,
                                          int oy, int oz, CellCache<TP> &cca, CellCache<TP> &ccb, TP (&a)[6],
                                          TP (&b)[6]) {
    TP ua = a[3], va = a[4], wa = a[5], xa = a[0], ya = a[1], za = a[2];
    TP ub = b[3], vb = b[4], wb = b[5], xb = b[0], yb = b[1], zb = b[2];
    for (int it = 0; it < mv.niter; ++it) {
        TP Fa[6], Fb[6];
        int rba, rbb;
        Cell<TP> ca, cb;
        const bool ina = pair_locate(g, tg, ox, oy, oz, xa, ya, za, cca, rba, ca);
        const bool inb = pair_locate(g, tg, ox, oy, oz, xb, yb, zb, ccb, rbb, cb);
        if (ina & inb) {  // the common case: both gathers from LDS, one block
            gather_lds(fl, tg, rba, ca, Fa);
            gather_lds(fl, tg, rbb, cb, Fb);
        } else {
            if (ina) {
                gather_lds(fl, tg, rba, ca, Fa);
            } else {
                gather_cell_global(f, ca, Fa);
                settle(Fa);
            }
            if (inb) {
                gather_lds(fl, tg, rbb, cb, Fb);
            } else {
                gather_cell_global(f, cb, Fb);
                settle(Fb);
            }
        }
        pair_rotate(mv, Fa, a[0], a[1], a[2], a[3], a[4], a[5], ua, va, wa, xa, ya, za);
        pair_rotate(mv, Fb, b[0], b[1], b[2], b[3], b[4], b[5], ub, vb, wb, xb, yb, zb);
    }
    a[3] = TP(2) * ua - a[3]; a[4] = TP(2) * va - a[4]; a[5] = TP(2) * wa - a[5];
    b[3] = TP(2) * ub - b[3]; b[4] = TP(2) * vb - b[4]; b[5] = TP(2) * wb - b[5];
    a[0] = pwrap(a[0] + ua * mv.dt, g.L[0], g.invL[0]);
    a[1] = pwrap(a[1] + va * mv.dt, g.L[1], g.invL[1]);
    a[2] = pwrap(a[2] + wa * mv.dt, g.L[2], g.invL[2]);
    b[0] = pwrap(b[0] + ub * mv.dt, g.L[0], g.invL[0]);
    b[1] = pwrap(b[1] + vb * mv.dt, g.L[1], g.invL[1]);
    b[2] = pwrap(b[2] + wb * mv.dt, g.L[2], g.invL[2]);
}

template <typename TP, typename TF, typename TA, class GEO>
__device__ __forceinline__ void tile_body_pair(const TileJob<TP, TF, TA> &J, int t, unsigned char *smem) {
    const GridT<TP> &g = J.g;
    TileGeom tg = J.tg;
    if constexpr (GEO::fixed) {
        tg.tx = GEO::tx; tg.ty = GEO::ty; tg.tz = GEO::tz; tg.halo = GEO::halo;
        tg.rx = GEO::rx; tg.ry = GEO::ry; tg.rz = GEO::rz;
        tg.slow = GEO::slow; tg.mid = GEO::mid; tg.fast = GEO::fast;
        tg.sx = GEO::sx; tg.sy = GEO::sy; tg.sz = GEO::sz; tg.rnp = GEO::rnp;
    }
    const FieldPtrs<TF> &f = J.f;
    const PartPtrs<TP> &p = J.p;
    const PartPtrs<TP> &pin = J.in;
    TA *__restrict__ mom = J.mom;
    const int nn = J.nn;
    const uint32_t beg = J.tile_off[t], end = J.tile_off[t + 1];
    if (beg == end) return;
    const int RNP = tg.rnp;
    const size_t fbytes = (RNP * sizeof(LdsFieldNode<TP>) + 15) & ~(size_t)15;
    LdsFieldNode<TP> *fl = (LdsFieldNode<TP> *)smem;
    TA *ml = (TA *)(smem + fbytes);
    unsigned char *wstage = smem + fbytes + (((size_t)10 * RNP * sizeof(TA) + 15) & ~(size_t)15);
    const int tzi = t % tg.ntz, tyi = (t / tg.ntz) % tg.nty, txi = t / (tg.ntz * tg.nty);
    int ox = (txi * tg.tx - tg.halo) % g.nx; ox += ox < 0 ? g.nx : 0;
    int oy = (tyi * tg.ty - tg.halo) % g.ny; oy += oy < 0 ? g.ny : 0;
    int oz = (tzi * tg.tz - tg.halo) % g.nz; oz += oz < 0 ? g.nz : 0;
    const int RL = tg.rx * tg.ry * tg.rz;
    const int sx = tg.sx, sy = tg.sy, sz = tg.sz;
    for (int r = threadIdx.x; r < RL; r += blockDim.x) {
        const RegionNode rn = region_node(tg, g.nx, g.ny, g.nz, ox, oy, oz, r);
        LdsFieldNode<TP> fn;
#pragma unroll
        for (int m = 0; m < 6; ++m) fn.v[m] = (TP)f.f[m][rn.gnode];
        fl[rn.slot] = fn;
    }
    if (mom)
        for (int q = threadIdx.x; q < 10 * RNP; q += blockDim.x) ml[q] = TA(0);
    __syncthreads();

    const int coff[8] = {0, sx, sy, sx + sy, sz, sx + sz, sy + sz, sx + sy + sz};
    const int lane = threadIdx.x & 63;
    const int lcell = lane_cell(tg, g.nx, g.ny, g.nz, txi, tyi, tzi, lane);
    TP lacc[80];
#pragma unroll
    for (int q = 0; q < 80; ++q) lacc[q] = TP(0);
    unsigned char *mine = wstage + (threadIdx.x >> 6) * (64 * sizeof(StagedParticle<TP>) + sizeof(BalanceLds));
    TP *lq = (TP *)mine;
    StagedParticle<TP> *lstage = (StagedParticle<TP> *)mine;
    BalanceLds *lbal = (BalanceLds *)(mine + 64 * sizeof(StagedParticle<TP>));
    int qn = 0;
    CellCache<TP> cca, ccb;
    cca.ijk[0] = -1; ccb.ijk[0] = -1;
    cca.rb = ccb.rb = 0;
    cca.in = ccb.in = false;
    cca.ijk[1] = cca.ijk[2] = ccb.ijk[1] = ccb.ijk[2] = 0;
    const bool copy_id = J.copy_rest && pin.id;
    const uint32_t B = blockDim.x;
    constexpr uint32_t ES = sizeof(TP);

    // one particle's deposit: lane-cell registers or the queue
    auto deposit = [&](bool valid, const TP (&s)[6], TP q) {
        bool enq = false;
        if (valid && mom) {
            int rb;
            Cell<TA> c;
            const bool in = region_locate(J.ga, tg, ox, oy, oz, (TA)s[0], (TA)s[1], (TA)s[2], rb, c);
            if (in && rb == lcell) {
                TA wt8[8];
                pweights(c.fx, c.fy, c.fz, wt8);
                const TP u = s[3], v = s[4], w = s[5];
                const TP val[10] = {TP(1), u, v, w, u * u, u * v, u * w, v * v, v * w, w * w};
                const TA qa = (TA)q;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const TP qw = (TP)(qa * wt8[k]);
#pragma unroll
                    for (int m = 0; m < 10; ++m) lacc[k * 10 + m] += qw * val[m];
                }
            } else {
                enq = true;
            }
        }
        const unsigned long long vote = __ballot(enq);
        if (vote) {
            const int cnt = __popcll(vote);
            const int pos = qn + __popcll(vote & ((1ull << lane) - 1ull));
            const TP rec[7] = {s[0], s[1], s[2], s[3], s[4], s[5], q};
            if (enq && pos < 64)
#pragma unroll
                for (int a = 0; a < 7; ++a) lq[a * 64 + pos] = rec[a];
            if (qn + cnt >= 64) {
                wave_sync();
                TP r[7];
#pragma unroll
                for (int a = 0; a < 7; ++a) r[a] = lq[a * 64 + lane];
                wave_sync();
                deposit_balanced<TP, TA, GEO>(J.ga, tg, ox, oy, oz, ml, mom, nn, lstage, lbal, lane, true, r[0], r[1],
                                              r[2], r[3], r[4], r[5], r[6]);
                if (enq && pos >= 64)
#pragma unroll
                    for (int a = 0; a < 7; ++a) lq[a * 64 + pos - 64] = rec[a];
                qn += cnt - 64;
            } else {
                qn += cnt;
            }
        }
    };

    // lane l takes particles beg + l' + 2kB and beg + l' + (2k+1)B (l' = thread index)
    for (uint32_t i0 = beg + (threadIdx.x & ~63u); i0 < end; i0 += 2 * B) {
        const uint32_t ia = i0 + lane, ib = ia + B;
        const bool va = ia < end, vb = ib < end;
        TP a[6] = {TP(0), TP(0), TP(0), TP(0), TP(0), TP(0)}, b[6] = {TP(0), TP(0), TP(0), TP(0), TP(0), TP(0)};
        TP qa = TP(0), qb = TP(0);
        int64_t ida = 0, idb = 0;
        if (va) {
            const uint32_t o = ia * ES;
            a[0] = ld32(pin.x, o); a[1] = ld32(pin.y, o); a[2] = ld32(pin.z, o);
            a[3] = ld32(pin.u, o); a[4] = ld32(pin.v, o); a[5] = ld32(pin.w, o); qa = ld32(pin.q, o);
            if (copy_id) ida = pin.id[ia];
        }
        if (vb) {
            const uint32_t o = ib * ES;
            b[0] = ld32(pin.x, o); b[1] = ld32(pin.y, o); b[2] = ld32(pin.z, o);
            b[3] = ld32(pin.u, o); b[4] = ld32(pin.v, o); b[5] = ld32(pin.w, o); qb = ld32(pin.q, o);
            if (copy_id) idb = pin.id[ib];
        }
        if (va) {  // a lane past the end moves its zero slot harmlessly and stores nothing
            pair_move(g, J.mv, f, fl, tg, ox, oy, oz, cca, ccb, a, b);
            const uint32_t o = ia * ES;
            st32(p.x, o, a[0]); st32(p.y, o, a[1]); st32(p.z, o, a[2]);
            st32(p.u, o, a[3]); st32(p.v, o, a[4]); st32(p.w, o, a[5]);
            if (J.copy_rest) {
                st32(p.q, o, qa);
                if (copy_id) p.id[ia] = ida;
            }
            if (vb) {
                const uint32_t ob = ib * ES;
                st32(p.x, ob, b[0]); st32(p.y, ob, b[1]); st32(p.z, ob, b[2]);
                st32(p.u, ob, b[3]); st32(p.v, ob, b[4]); st32(p.w, ob, b[5]);
                if (J.copy_rest) {
                    st32(p.q, ob, qb);
                    if (copy_id) p.id[ib] = idb;
                }
            }
        }
        deposit(va, a, qa);
        deposit(vb, b, qb);
    }
    if (!mom) return;
    wave_sync();
    TP r[7] = {TP(0), TP(0), TP(0), TP(0), TP(0), TP(0), TP(0)};
    if (lane < qn)
#pragma unroll
        for (int a = 0; a < 7; ++a) r[a] = lq[a * 64 + lane];
    wave_sync();
    if (qn > 0)
        deposit_balanced<TP, TA, GEO>(J.ga, tg, ox, oy, oz, ml, mom, nn, lstage, lbal, lane, lane < qn, r[0], r[1],
                                      r[2], r[3], r[4], r[5], r[6]);
    settle(lacc);
    if (lcell >= 0) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            TA *dst = ml + lcell + coff[k];
#pragma unroll
            for (int m = 0; m < 10; ++m) atomicAdd(dst + m * RNP, (TA)lacc[k * 10 + m]);
        }
    }
    __syncthreads();
    for (int r2 = threadIdx.x; r2 < RL; r2 += blockDim.x) {
        const RegionNode rn = region_node(tg, g.nx, g.ny, g.nz, ox, oy, oz, r2);
#pragma unroll
        for (int m = 0; m < 10; ++m) {
            const TA val = ml[m * RNP + rn.slot];
            if (val != TA(0)) atomicAdd(mom + (size_t)m * nn + rn.gnode, val);
        }
    }
}

// Particles in flight per thread of the deposit kernel (at least 2: a
// slot is refilled after its particle is deposited), and its register
// budget in waves per SIMD.
constexpr int kDepositPrefetch = 2;
constexpr int kDepositWaves = 3;
static_assert(kDepositPrefetch >= 2, "the deposit loop refills a slot after depositing it");

// Deposit of a tile whose particles a mover-only launch has just moved
// (variant 8, the second of its two kernels): the lane-cell register sums
// and the compact queue of variant 5 (deposited bank-balanced), with only the 80 sums and one
// particle live; LDS holds the FP64 region moments (dense layout) and the
// queues only (no fields), three workgroups of 256 per CU.
template <typename TP, typename TF, typename TA, class GEO>
__device__ __forceinline__ void deposit_body(const TileJob<TP, TF, TA> &J, int t, unsigned char *smem) {
    TileGeom tg = J.tg;
    if constexpr (GEO::fixed) {
        tg.tx = GEO::tx; tg.ty = GEO::ty; tg.tz = GEO::tz; tg.halo = GEO::halo;
        tg.rx = GEO::rx; tg.ry = GEO::ry; tg.rz = GEO::rz;
        tg.slow = GEO::slow; tg.mid = GEO::mid; tg.fast = GEO::fast;
        tg.sx = GEO::sx; tg.sy = GEO::sy; tg.sz = GEO::sz; tg.rnp = GEO::rnp;
    }
    const GridT<TP> &g = J.g;
    const PartPtrs<TP> &p = J.p;
    TA *__restrict__ mom = J.mom;
    const int nn = J.nn;
    const uint32_t beg = J.tile_off[t], end = J.tile_off[t + 1];
    if (beg == end) return;
    const int RNP = tg.rnp;
    TA *ml = (TA *)smem;
    // per-wave queue (7 arrays of 64: x y z u v w q) and, beside it, the
    // balancing stage (so that the queue takes the overflow of a flush
    // before the flush deposits)
    unsigned char *mine = smem + (((size_t)10 * RNP * sizeof(TA) + 15) & ~(size_t)15) +
                          (threadIdx.x >> 6) * (64 * 7 * sizeof(TP) + 64 * sizeof(StagedParticle<TP>) +
                                                sizeof(BalanceLds));
    TP *sq = (TP *)mine;
    StagedParticle<TP> *lstage = (StagedParticle<TP> *)(mine + 64 * 7 * sizeof(TP));
    BalanceLds *lbal = (BalanceLds *)(mine + 64 * 7 * sizeof(TP) + 64 * sizeof(StagedParticle<TP>));
    const int tzi = t % tg.ntz, tyi = (t / tg.ntz) % tg.nty, txi = t / (tg.ntz * tg.nty);
    int ox = (txi * tg.tx - tg.halo) % g.nx; ox += ox < 0 ? g.nx : 0;
    int oy = (tyi * tg.ty - tg.halo) % g.ny; oy += oy < 0 ? g.ny : 0;
    int oz = (tzi * tg.tz - tg.halo) % g.nz; oz += oz < 0 ? g.nz : 0;
    const int RL = tg.rx * tg.ry * tg.rz;
    const int sx = tg.sx, sy = tg.sy, sz = tg.sz;
    for (int q = threadIdx.x; q < 10 * RNP; q += blockDim.x) ml[q] = TA(0);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int lc = lane_cell(tg, g.nx, g.ny, g.nz, txi, tyi, tzi, lane);
    const int coff[8] = {0, sx, sy, sx + sy, sz, sx + sz, sy + sz, sx + sy + sz};
    TP sacc[80];
#pragma unroll
    for (int q = 0; q < 80; ++q) sacc[q] = TP(0);
    int sqn = 0;
    const uint32_t stride = blockDim.x;
    constexpr uint32_t ES = sizeof(TP);
    uint32_t ii = beg + threadIdx.x;
    // the next PF particles of this thread load while one deposits
    constexpr int PF = kDepositPrefetch;
    // unconditional loads (past the range: the tile's last particle, read
    // and ignored), so a slot is refilled in place with no merge of old and
    // new values that would make the compiler copy it and wait for it
    auto load = [&](TP (&dst)[7], uint32_t i) __attribute__((always_inline)) {
        const uint32_t o = min(i, end - 1) * ES;
        dst[0] = ld32(p.x, o); dst[1] = ld32(p.y, o); dst[2] = ld32(p.z, o);
        dst[3] = ld32(p.u, o); dst[4] = ld32(p.v, o); dst[5] = ld32(p.w, o); dst[6] = ld32(p.q, o);
    };
    // one particle: its lane-cell sums or the queue
    auto process = [&](const TP (&rec)[7], bool valid) __attribute__((always_inline)) {
        bool enq = false;
        if (valid) {
            // the cell from the particle-precision position, the in-cell
            // offsets of the moved (already wrapped) position in the
            // accumulation precision, the terms in the particle precision
            // (as variant 5; at a face the two precisions may pick
            // neighbouring cells, where the weights agree to rounding)
            int rb, ijk[3];
            Cell<TP> c32;
            const bool in = region_locate(g, tg, ox, oy, oz, rec[0], rec[1], rec[2], rb, c32, ijk);
            if (in && rb == lc) {
                const TP u = rec[3], v = rec[4], w = rec[5];
                const TP val[10] = {TP(1), u, v, w, u * u, u * v, u * w, v * v, v * w, w * w};
                const TA qa = (TA)rec[6];
                Cell<TA> c;
                c.fx = cell_coord((TA)rec[0], J.ga.invd[0]) - (TA)ijk[0];
                c.fy = cell_coord((TA)rec[1], J.ga.invd[1]) - (TA)ijk[1];
                c.fz = cell_coord((TA)rec[2], J.ga.invd[2]) - (TA)ijk[2];
                const TA gx = TA(1) - c.fx, gy = TA(1) - c.fy, gz = TA(1) - c.fz;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    // corner weight formed as pweights forms it, one at a time
                    const TA wk = (((k & 1) ? c.fx : gx) * ((k & 2) ? c.fy : gy)) * ((k & 4) ? c.fz : gz);
                    const TP qw = (TP)(qa * wk);
#pragma unroll
                    for (int m = 0; m < 10; ++m) sacc[k * 10 + m] += qw * val[m];
                }
            } else {
                enq = true;
            }
        }
        const unsigned long long vote = __ballot(enq);
        if (vote) {
            const int cnt = __popcll(vote);
            const int pos = sqn + __popcll(vote & ((1ull << lane) - 1ull));
            if (enq && pos < 64)
#pragma unroll
                for (int a = 0; a < 7; ++a) sq[a * 64 + pos] = rec[a];
            if (sqn + cnt >= 64) {
                wave_sync();
                TP r[7];
#pragma unroll
                for (int a = 0; a < 7; ++a) r[a] = sq[a * 64 + lane];
                wave_sync();
                if (enq && pos >= 64)
#pragma unroll
                    for (int a = 0; a < 7; ++a) sq[a * 64 + pos - 64] = rec[a];
                deposit_balanced<TP, TA, GEO, true>(J.ga, tg, ox, oy, oz, ml, mom, nn, lstage, lbal, lane, true, r[0],
                                                    r[1], r[2], r[3], r[4], r[5], r[6]);
                sqn += cnt - 64;
            } else {
                sqn += cnt;
            }
        }
    };
    // PF particles of this thread are in flight: the loop is unrolled by PF
    // and each slot is deposited from and then refilled in place, so that
    // no register copy of a slot whose load is in flight (which would wait
    // for every load) is needed; a load has PF - 1 particles' time to land
    TP ring[PF][7];
#pragma unroll
    for (int k = 0; k < PF; ++k) load(ring[k], ii + k * stride);
    for (uint32_t i0 = beg + (threadIdx.x & ~63u); i0 < end; i0 += PF * stride, ii += PF * stride) {
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            process(ring[k], ii + k * stride < end);
            load(ring[k], ii + (k + PF) * stride);
        }
    }
    wave_sync();
    {
        TP r[7] = {TP(0), TP(0), TP(0), TP(0), TP(0), TP(0), TP(0)};
        if (lane < sqn)
#pragma unroll
            for (int a = 0; a < 7; ++a) r[a] = sq[a * 64 + lane];
        wave_sync();
        if (sqn > 0)
            deposit_balanced<TP, TA, GEO, true>(J.ga, tg, ox, oy, oz, ml, mom, nn, lstage, lbal, lane, lane < sqn,
                                                r[0], r[1], r[2], r[3], r[4], r[5], r[6]);
    }
    settle(sacc);
    if (lc >= 0) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            TA *dst = ml + lc + coff[k];
#pragma unroll
            for (int m = 0; m < 10; ++m) atomicAdd(dst + m * RNP, (TA)sacc[k * 10 + m]);
        }
    }
    __syncthreads();
    for (int r = threadIdx.x; r < RL; r += blockDim.x) {
        const RegionNode rn = region_node(tg, g.nx, g.ny, g.nz, ox, oy, oz, r);
#pragma unroll
        for (int m = 0; m < 10; ++m) {
            const TA val = ml[m * RNP + rn.slot];
            if (val != TA(0)) atomicAdd(mom + (size_t)m * nn + rn.gnode, val);
        }
    }
}

template <typename TP, typename TF, typename TA, class GEO>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(kDepositWaves)))
k_deposit_tiled(TileJob<TP, TF, TA> J, int chunk) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int b = blockIdx.x;
    const int t = (b & 7) * chunk + (b >> 3);
    if (t >= J.tg.ntiles) return;
    deposit_body<TP, TF, TA, GEO>(J, t, smem);
}

// Variants (register budget -> waves per SIMD):
//   0  every deposit is an LDS atomic; <= 128 VGPRs, 4 waves/SIMD
//   1  as 0, and the 48 field corners of the last cell stay in registers,
//      so gathers in a thread's cell skip LDS; <= 168 VGPRs, 3 waves/SIMD
//   2  home-cell register accumulation of the deposit (80 sums) with LDS
//      atomics for drifted particles; <= 256 VGPRs, 2 waves/SIMD
//   3  as 0, with the bank-balanced deposit (per-wave staging in LDS)
//   4  segmented wave pre-reduction of the deposit (cell-major sort order)
//   5  lane-cell sums in particle-precision registers + compact queue of
//      drifted particles, deposited bank-balanced; <= 256 VGPRs (its LDS
//      keeps it at 2 waves/SIMD at 256 threads anyway)
//   6  two-phase mover / deposit pass; <= 168 VGPRs (FP32), 3 waves/SIMD
//   7  as 5 with a second register set for one drift cell; <= 256 VGPRs
//   8  two launches: mover only (variant 1, or 0, without moments), then
//      the lane-cell deposit kernel over the moved particles
//   9  as 5 with two particles per thread in flight; <= 256 VGPRs
template <int VAR, typename TP>
struct VariantWaves {
    static constexpr int value =
        (VAR == 0 || VAR == 3 || VAR == 4) ? 4 : (VAR == 1 || (VAR == 6 && sizeof(TP) == 4)) ? 3 : 2;
};

template <typename TP, typename TF, typename TA, int VAR, class GEO>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(VariantWaves<VAR, TP>::value)))
k_fused_tiled(TileJob<TP, TF, TA> J, int chunk) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int b = blockIdx.x;
    const int t = (b & 7) * chunk + (b >> 3);
    if (t >= J.tg.ntiles) return;
    if constexpr (VAR == 9) tile_body_pair<TP, TF, TA, GEO>(J, t, smem);
    else tile_body<TP, TF, TA, VAR, GEO>(J, t, smem);
}

// Persistent work-list kernel: workgroups take (job, tile) items from an
// atomic counter until the list is drained; every workgroup exits once the
// counter passes nitems.  The counter must be zero at launch.
template <typename TP, typename TF, typename TA, int VAR, class GEO>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(VariantWaves<VAR, TP>::value)))
k_worklist(const TileJob<TP, TF, TA> *__restrict__ jobs, const uint2 *__restrict__ items, int nitems,
           unsigned *__restrict__ counter) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int cur;
    for (;;) {
        __syncthreads();  // the previous item's LDS use is over before `cur` changes
        if (threadIdx.x == 0) cur = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(cur);
        if (it >= nitems) break;
        const uint2 item = items[it];
        const TileJob<TP, TF, TA> J = jobs[item.x];
        if constexpr (VAR == 9) tile_body_pair<TP, TF, TA, GEO>(J, (int)item.y, smem);
        else tile_body<TP, TF, TA, VAR, GEO>(J, (int)item.y, smem);
    }
}

size_t tiled_lds_bytes(const TileGeom &tg, int dtype, int acc_dtype, int variant, int block) {
    const size_t fsz = (size_t)tg.rnp * 6 * (dtype == SPIC_F64 ? 8 : 4);
    const size_t msz = (size_t)tg.rnp * 10 * (acc_dtype == SPIC_F64 ? 8 : 4);
    return ((fsz + 15) & ~(size_t)15) + ((msz + 15) & ~(size_t)15) + stage_lds_bytes(variant, block, dtype);
}

// Dynamic LDS above 64 KiB must be allowed per kernel once.
template <typename K>
static void allow_lds(K kernel, size_t bytes) {
    static size_t allowed = 64 * 1024;
    if (bytes > allowed) {
        if (hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) ==
            hipSuccess)
            allowed = bytes;
    }
}

template <typename TP, typename TF, typename TA, int VAR, class GEO>
static void tiled_launch(const TileJob<TP, TF, TA> &job, int chunk, size_t lds, int block, hipStream_t s) {
    allow_lds(k_fused_tiled<TP, TF, TA, VAR, GEO>, lds);
    hipLaunchKernelGGL((k_fused_tiled<TP, TF, TA, VAR, GEO>), dim3(8 * chunk), dim3(block), lds, s, job, chunk);
}

template <int MV, typename TP, typename TF, typename TA, class G>
static void mover_launch(const TileJob<TP, TF, TA> &mv, int chunk, size_t fl, hipStream_t s) {
    allow_lds(k_fused_tiled<TP, TF, TA, MV, G>, fl);
    hipLaunchKernelGGL((k_fused_tiled<TP, TF, TA, MV, G>), dim3(8 * chunk), dim3(512), fl, s, mv, chunk);
}

// Variant 8: a mover-only launch (variant 1's or 0's tile body without
// moments, LDS for the fields only) and then the deposit kernel over the
// moved particles (LDS for the moments and queues only).
template <typename TP, typename TF, typename TA, class GEO>
static void split_launch(const TileJob<TP, TF, TA> &job, int chunk, const LaunchCfg &cfg, hipStream_t s) {
    const TileGeom &tg = job.tg;
    // the mover stages a wider field region than the deposit (fields are 6
    // values a node against the deposit's 10 FP64 moments, and a particle
    // that left the region gathers from global memory, three times)
    TileJob<TP, TF, TA> mv = job;
    mv.mom = nullptr;
    int mh = cfg.mover_halo >= 0 ? cfg.mover_halo : tg.halo + 1;
    // the layout search is memoised per thread (one tiling per run, as a rule)
    thread_local int key[5] = {-1, -1, -1, -1, -1};
    thread_local RegionLayout ml{0, 0, 0, 0};
    const int axes = tg.slow * 9 + tg.mid * 3 + tg.fast;
    if (key[0] != tg.tx || key[1] != tg.ty || key[2] != tg.tz || key[3] != mh || key[4] != axes) {
        ml = region_layout(tg.tx, tg.ty, tg.tz, mh, tg.slow, tg.mid, tg.fast, 1);
        key[0] = tg.tx; key[1] = tg.ty; key[2] = tg.tz; key[3] = mh; key[4] = axes;
    }
    // a region that does not fit the device's LDS keeps the tile's halo
    if ((size_t)ml.rnp * sizeof(LdsFieldNode<TP>) > cfg.lds_max) mh = tg.halo;
    if (mh != tg.halo) {
        mv.tg.halo = mh;
        mv.tg.rx = tg.tx + 2 * mh + 1; mv.tg.ry = tg.ty + 2 * mh + 1; mv.tg.rz = tg.tz + 2 * mh + 1;
        mv.tg.sx = ml.sx; mv.tg.sy = ml.sy; mv.tg.sz = ml.sz; mv.tg.rnp = ml.rnp;
    }
    const size_t fl = ((size_t)mv.tg.rnp * sizeof(LdsFieldNode<TP>) + 15) & ~(size_t)15;
    // the mover body: variant 1's (the last cell's 48 field values in
    // registers; in full rows a thread's particles share their sort cell, so
    // most gathers skip LDS) or variant 0's
    if (cfg.mover_cache) {
        if (mh == tg.halo) mover_launch<1, TP, TF, TA, GEO>(mv, chunk, fl, s);
        else if (cfg.fixed_geo && geo_is<GeoMover2>(mv.tg)) mover_launch<1, TP, TF, TA, GeoMover2>(mv, chunk, fl, s);
        else mover_launch<1, TP, TF, TA, GeoRuntime>(mv, chunk, fl, s);
    } else {
        if (mh == tg.halo) mover_launch<0, TP, TF, TA, GEO>(mv, chunk, fl, s);
        else if (cfg.fixed_geo && geo_is<GeoMover2>(mv.tg)) mover_launch<0, TP, TF, TA, GeoMover2>(mv, chunk, fl, s);
        else mover_launch<0, TP, TF, TA, GeoRuntime>(mv, chunk, fl, s);
    }
    if (!job.mom) return;
    // the deposit kernel's region uses the dense layout (smallest LDS: three
    // workgroups per CU)
    TileJob<TP, TF, TA> dj = job;
    const RegionLayout lay = region_layout(tg.tx, tg.ty, tg.tz, tg.halo, tg.slow, tg.mid, tg.fast, 2);
    dj.tg.sx = lay.sx; dj.tg.sy = lay.sy; dj.tg.sz = lay.sz; dj.tg.rnp = lay.rnp;
    const size_t dl = (((size_t)10 * lay.rnp * sizeof(TA) + 15) & ~(size_t)15) +
                      stage_lds_bytes(8, cfg.tile_block, sizeof(TP) == 8 ? SPIC_F64 : SPIC_F32);
    if (cfg.fixed_geo && geo_is<GeoDense>(dj.tg)) {
        allow_lds(k_deposit_tiled<TP, TF, TA, GeoDense>, dl);
        hipLaunchKernelGGL((k_deposit_tiled<TP, TF, TA, GeoDense>), dim3(8 * chunk), dim3(cfg.tile_block), dl, s, dj,
                           chunk);
    } else {
        allow_lds(k_deposit_tiled<TP, TF, TA, GeoRuntime>, dl);
        hipLaunchKernelGGL((k_deposit_tiled<TP, TF, TA, GeoRuntime>), dim3(8 * chunk), dim3(cfg.tile_block), dl, s,
                           dj, chunk);
    }
}

template <typename TP, typename TF, typename TA, class GEO>
static void tiled_variant(const TileJob<TP, TF, TA> &job, int chunk, size_t lds, const LaunchCfg &cfg,
                          hipStream_t s) {
    switch (cfg.variant) {
        case 8: split_launch<TP, TF, TA, GEO>(job, chunk, cfg, s); break;
        case 1: tiled_launch<TP, TF, TA, 1, GEO>(job, chunk, lds, cfg.tile_block, s); break;
        case 2: tiled_launch<TP, TF, TA, 2, GEO>(job, chunk, lds, cfg.tile_block, s); break;
        case 3: tiled_launch<TP, TF, TA, 3, GEO>(job, chunk, lds, cfg.tile_block, s); break;
        case 4: tiled_launch<TP, TF, TA, 4, GEO>(job, chunk, lds, cfg.tile_block, s); break;
        case 5: tiled_launch<TP, TF, TA, 5, GEO>(job, chunk, lds, cfg.tile_block, s); break;
        case 6: tiled_launch<TP, TF, TA, 6, GEO>(job, chunk, lds, cfg.tile_block, s); break;
        case 7: tiled_launch<TP, TF, TA, 7, GEO>(job, chunk, lds, cfg.tile_block, s); break;
        case 9: tiled_launch<TP, TF, TA, 9, GEO>(job, chunk, lds, cfg.tile_block, s); break;
        default: tiled_launch<TP, TF, TA, 0, GEO>(job, chunk, lds, cfg.tile_block, s);
    }
}

template <typename TP, typename TF, typename TA>
static void tiled_t(const spic_grid &g, const spic_params &prm, const spic_fields &f, const SpeciesWork &w,
                    const TileGeom &tg, const uint32_t *tile_off, const LaunchCfg &cfg, hipStream_t s) {
    const int chunk = (tg.ntiles + 7) / 8;
    const size_t lds = tiled_lds_bytes(tg, sizeof(TP) == 8 ? SPIC_F64 : SPIC_F32,
                                       sizeof(TA) == 8 ? SPIC_F64 : SPIC_F32, cfg.variant, cfg.tile_block);
    const auto job = make_tile_job<TP, TF, TA>(g, prm, f, w, tg, tile_off);
    if (geo_is_default(tg) && cfg.fixed_geo) tiled_variant<TP, TF, TA, GeoDefault>(job, chunk, lds, cfg, s);
    else if (geo_is<GeoDense>(tg) && cfg.fixed_geo && (cfg.variant == 5 || cfg.variant == 6)) {
        if (cfg.variant == 5) tiled_launch<TP, TF, TA, 5, GeoDense>(job, chunk, lds, cfg.tile_block, s);
        else tiled_launch<TP, TF, TA, 6, GeoDense>(job, chunk, lds, cfg.tile_block, s);
    }
    else tiled_variant<TP, TF, TA, GeoRuntime>(job, chunk, lds, cfg, s);
}

hipError_t launch_fused_tiled(const spic_grid &g, const spic_params &prm, const spic_fields &f,
                              const SpeciesWork &w, const TileGeom &tg, const uint32_t *tile_off,
                              const LaunchCfg &cfg, hipStream_t s) {
    if (w.n <= 0) return hipSuccess;
    const bool f64acc = (w.mom == nullptr) || w.acc_dtype == SPIC_F64;
    if (w.dtype == SPIC_F64) {
        if (f.dtype != SPIC_F64 || !f64acc) return hipErrorInvalidValue;
        tiled_t<double, double, double>(g, prm, f, w, tg, tile_off, cfg, s);
    } else if (f.dtype == SPIC_F32) {
        if (f64acc) tiled_t<float, float, double>(g, prm, f, w, tg, tile_off, cfg, s);
        else tiled_t<float, float, float>(g, prm, f, w, tg, tile_off, cfg, s);
    } else {
        if (f64acc) tiled_t<float, double, double>(g, prm, f, w, tg, tile_off, cfg, s);
        else tiled_t<float, double, float>(g, prm, f, w, tg, tile_off, cfg, s);
    }
    return hipGetLastError();
}

}  // namespace spic

// ------------------------------------------------------------ work lists
//
// The batch engine drives the persistent work-list kernel over tiles of
// many (run, species) jobs of one precision combination per launch.

namespace spic {

int job_combo(int dtype, int fdtype, int acc_dtype) {
    if (dtype == SPIC_F64) return (fdtype == SPIC_F64 && acc_dtype == SPIC_F64) ? 0 : -1;
    if (fdtype == SPIC_F32) return acc_dtype == SPIC_F64 ? 1 : 2;
    return acc_dtype == SPIC_F64 ? 3 : 4;
}

size_t tile_job_bytes(int combo) {
    switch (combo) {
        case 0: return sizeof(TileJob<double, double, double>);
        case 1: return sizeof(TileJob<float, float, double>);
        case 2: return sizeof(TileJob<float, float, float>);
        case 3: return sizeof(TileJob<float, double, double>);
        default: return sizeof(TileJob<float, double, float>);
    }
}

void write_tile_job(int combo, void *dst, const spic_grid &g, const spic_params &prm, const spic_fields &f,
                    const SpeciesWork &w, const TileGeom &tg, const uint32_t *tile_off) {
    switch (combo) {
        case 0: *(TileJob<double, double, double> *)dst = make_tile_job<double, double, double>(g, prm, f, w, tg, tile_off); break;
        case 1: *(TileJob<float, float, double> *)dst = make_tile_job<float, float, double>(g, prm, f, w, tg, tile_off); break;
        case 2: *(TileJob<float, float, float> *)dst = make_tile_job<float, float, float>(g, prm, f, w, tg, tile_off); break;
        case 3: *(TileJob<float, double, double> *)dst = make_tile_job<float, double, double>(g, prm, f, w, tg, tile_off); break;
        default: *(TileJob<float, double, float> *)dst = make_tile_job<float, double, float>(g, prm, f, w, tg, tile_off); break;
    }
}

// Workgroups of the persistent launch: resident workgroups per CU times
// CUs, capped by the item count (and by max_groups when > 0).  Also allows
// the LDS size; call before any stream capture.
template <typename TP, typename TF, typename TA, int VAR, class GEO>
static int worklist_groups_t(size_t lds, int block, int nitems, int max_groups) {
    auto k = k_worklist<TP, TF, TA, VAR, GEO>;
    allow_lds(k, lds);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, block, lds) != hipSuccess || per_cu < 1) per_cu = 1;
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    int groups = per_cu * ncu;
    if (groups > nitems) groups = nitems;
    if (max_groups > 0 && groups > max_groups) groups = max_groups;
    return groups < 1 ? 1 : groups;
}

template <typename TP, typename TF, typename TA, class GEO>
static int worklist_groups_v(int variant, size_t lds, int block, int nitems, int max_groups) {
    switch (variant) {
        case 1: return worklist_groups_t<TP, TF, TA, 1, GEO>(lds, block, nitems, max_groups);
        case 2: return worklist_groups_t<TP, TF, TA, 2, GEO>(lds, block, nitems, max_groups);
        case 3: return worklist_groups_t<TP, TF, TA, 3, GEO>(lds, block, nitems, max_groups);
        case 4: return worklist_groups_t<TP, TF, TA, 4, GEO>(lds, block, nitems, max_groups);
        case 5: return worklist_groups_t<TP, TF, TA, 5, GEO>(lds, block, nitems, max_groups);
        case 6: return worklist_groups_t<TP, TF, TA, 6, GEO>(lds, block, nitems, max_groups);
        case 7: return worklist_groups_t<TP, TF, TA, 7, GEO>(lds, block, nitems, max_groups);
        case 9: return worklist_groups_t<TP, TF, TA, 9, GEO>(lds, block, nitems, max_groups);
        default: return worklist_groups_t<TP, TF, TA, 0, GEO>(lds, block, nitems, max_groups);
    }
}

int worklist_groups(int combo, bool fixed, int variant, size_t lds, int block, int nitems, int max_groups) {
#define SPIC_WG(TP, TF, TA)                                                                  \
    return fixed ? worklist_groups_v<TP, TF, TA, GeoDefault>(variant, lds, block, nitems, max_groups) \
                 : worklist_groups_v<TP, TF, TA, GeoRuntime>(variant, lds, block, nitems, max_groups)
    switch (combo) {
        case 0: SPIC_WG(double, double, double);
        case 1: SPIC_WG(float, float, double);
        case 2: SPIC_WG(float, float, float);
        case 3: SPIC_WG(float, double, double);
        default: SPIC_WG(float, double, float);
    }
#undef SPIC_WG
}

template <typename TP, typename TF, typename TA, int VAR, class GEO>
static hipError_t worklist_t(const void *jobs, const uint2 *items, int nitems, unsigned *counter, size_t lds,
                             int block, int groups, hipStream_t s) {
    hipLaunchKernelGGL((k_worklist<TP, TF, TA, VAR, GEO>), dim3(groups), dim3(block), lds, s,
                       (const TileJob<TP, TF, TA> *)jobs, items, nitems, counter);
    return hipGetLastError();
}

template <typename TP, typename TF, typename TA, class GEO>
static hipError_t worklist_v(int variant, const void *jobs, const uint2 *items, int nitems, unsigned *counter,
                             size_t lds, int block, int groups, hipStream_t s) {
    switch (variant) {
        case 1: return worklist_t<TP, TF, TA, 1, GEO>(jobs, items, nitems, counter, lds, block, groups, s);
        case 2: return worklist_t<TP, TF, TA, 2, GEO>(jobs, items, nitems, counter, lds, block, groups, s);
        case 3: return worklist_t<TP, TF, TA, 3, GEO>(jobs, items, nitems, counter, lds, block, groups, s);
        case 4: return worklist_t<TP, TF, TA, 4, GEO>(jobs, items, nitems, counter, lds, block, groups, s);
        case 5: return worklist_t<TP, TF, TA, 5, GEO>(jobs, items, nitems, counter, lds, block, groups, s);
        case 6: return worklist_t<TP, TF, TA, 6, GEO>(jobs, items, nitems, counter, lds, block, groups, s);
        case 7: return worklist_t<TP, TF, TA, 7, GEO>(jobs, items, nitems, counter, lds, block, groups, s);
        case 9: return worklist_t<TP, TF, TA, 9, GEO>(jobs, items, nitems, counter, lds, block, groups, s);
        default: return worklist_t<TP, TF, TA, 0, GEO>(jobs, items, nitems, counter, lds, block, groups, s);
    }
}

hipError_t launch_worklist(int combo, bool fixed, int variant, const void *jobs, const uint2 *items, int nitems,
                           unsigned *counter, size_t lds, int block, int groups, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
#define SPIC_WL(TP, TF, TA)                                                                                   \
    return fixed ? worklist_v<TP, TF, TA, GeoDefault>(variant, jobs, items, nitems, counter, lds, block, groups, s) \
                 : worklist_v<TP, TF, TA, GeoRuntime>(variant, jobs, items, nitems, counter, lds, block, groups, s)
    switch (combo) {
        case 0: SPIC_WL(double, double, double);
        case 1: SPIC_WL(float, float, double);
        case 2: SPIC_WL(float, float, float);
        case 3: SPIC_WL(float, double, double);
        default: SPIC_WL(float, double, float);
    }
#undef SPIC_WL
}

// Zero many arrays in one launch: array a has counts[a] elements of
// elem_bytes (4 or 8) bytes.
__global__ void k_fill_many(void *const *__restrict__ ptrs, const int64_t *__restrict__ counts, int narr,
                            int elem_bytes) {
    const int a = blockIdx.y;
    if (a >= narr) return;
    const int64_t n = counts[a];
    if (elem_bytes == 8) {
        double *p = (double *)ptrs[a];
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
            p[i] = 0.0;
    } else {
        float *p = (float *)ptrs[a];
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
            p[i] = 0.0f;
    }
}

hipError_t launch_fill_many(void *const *ptrs, const int64_t *counts, int narr, int elem_bytes, hipStream_t s) {
    if (narr <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_many, dim3(64, narr), dim3(256), 0, s, ptrs, counts, narr, elem_bytes);
    return hipGetLastError();
}

}  // namespace spic
