// spic_tiled.hip -- tiled mover and moment gathering for a species that
// has been sorted by cell (spic_sort.hip).
//
// One workgroup per tile of cells.  The mover stages the node fields of its
// region (the tile's cells, `halo` cells around them and the +1 corner
// nodes) in LDS and moves every particle of the tile's range (Eq. 1, Eq. 2,
// Eq. 5) gathering E and B from LDS (Eq. 3, Eq. 4).  The moments of the
// moved particles (Sec. II moment equation; Sec. III-B: from the new
// position) are gathered per tile as well, into a region accumulator in
// LDS that is then added to the global moments with coalesced global
// atomics (neighbouring tiles' regions overlap).
//
// Variants (`tile_variant`):
//   0  one kernel: mover, and every deposit an FP64 LDS atomic;
//   1  as 0, with the 48 field values of a thread's last cell in registers
//      (in sort order a thread's particles share their cell, so most
//      gathers skip LDS);
//   2  two launches: variant 1's mover without moments, then the sorted
//      deposit below over the moved particles;
//   3  one launch (FP32 particles; FP64 particles run variant 2): variant
//      1's mover hands each moved particle to the sorted deposit's lane
//      sums, so only the particles that changed cell are read again.
//
// Sorted deposit.  The deposit workgroup counting-sorts the moved
// particles of its tile by their new cell in LDS (an index list), and lane
// l of every wave owns local cell l: it keeps the moments of that cell's 8
// nodes (80 sums) in registers and adds the particles the list gives it.
// Particles that moved to another cell of the tile therefore cost no more
// than those that stayed; only those that left the tile go through FP64
// LDS atomics (bank-balanced, a wave of them at a time) or, beyond the
// region, global atomics.
//
// LDS layout.  The region slot of a node is di*sx + dj*sy + dk*sz, with the
// strides of a padded layout whose slow axis is the one particles cross most
// often (region_layout) for the mover's fields, and the dense layout for
// the deposit's moments.  Fields are node-major (6 values per slot), moments
// component-major ([10][slots]).
//
// Particles whose cell lies outside the region (they drifted farther than
// the halo since the last sort) take the global path for that gather or
// deposit, so the result does not depend on the particle order; the order
// only decides how much work stays in LDS and registers.
//
// Tiles are mapped to workgroups with the 8 XCDs in mind (workgroup b runs
// on XCD b % 8): by default groups of 16 consecutive tiles are dealt to the
// XCDs in turn; the alternative gives each XCD a contiguous slab of tiles
// (tile_of_block).
#include <hip/hip_runtime.h>

#include <algorithm>

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
// sorted deposit keeps 80 lane sums live across it).
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



// Orders one wave's LDS accesses across lanes (a wave's LDS operations are
// processed in issue order; this keeps the compiler from reordering them).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A moved particle staged in LDS for the bank-balanced deposit.
template <typename TP>
struct StagedParticle {
    TP x, y, z, u, v, w, q, pad;
};

// Bank-balanced deposit of a wave's particles that lie outside the tile (in
// arbitrary region cells).  An FP64 LDS access by 16 consecutive lanes is
// conflict free when their slots differ modulo 16 (measured: 8 clk per
// atomic instruction then, 22-28 clk with 2-4-way conflicts).  Before its
// 80 atomics a wave therefore re-places its particles: the r-th particle (r < 4) whose slot is b modulo 16 goes
// to lane 16 r + b, so each group of 16 lanes holds distinct bank pairs;
// the rest fill the lanes left empty.  All 64 lanes must be active.
struct BalanceLds {
    int count[16];  // particles per bank pair
    int hole[64];   // lanes left empty, in lane order
};

// The re-placed particles are deposited with deposit_tight (few live
// registers).
template <typename TP, typename TA, class GEO>
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
        deposit_tight<TA, GEO>(ga, tg, ox, oy, oz, ml, mom, nn, (TA)s.x, (TA)s.y, (TA)s.z, (TA)s.q, (TA)s.u,
                               (TA)s.v, (TA)s.w);
    }
    wave_sync();  // the stage is rewritten by the next call
}

// Tile geometry with the compile-time values of GEO where the host launched
// a kernel specialised for one tiling.
template <class GEO>
__device__ __forceinline__ void apply_geo(TileGeom &tg) {
    if constexpr (GEO::fixed) {
        tg.tx = GEO::tx; tg.ty = GEO::ty; tg.tz = GEO::tz; tg.halo = GEO::halo;
        tg.rx = GEO::rx; tg.ry = GEO::ry; tg.rz = GEO::rz;
        tg.slow = GEO::slow; tg.mid = GEO::mid; tg.fast = GEO::fast;
        tg.sx = GEO::sx; tg.sy = GEO::sy; tg.sz = GEO::sz; tg.rnp = GEO::rnp;
        tg.cells = GEO::tx * GEO::ty * GEO::tz;
    }
}

// Where tile t sits: its first cell (c0) and the region's first node (o,
// wrapped into the grid).
struct TilePlace {
    int c0[3];
    int ox, oy, oz;
};

__device__ __forceinline__ TilePlace tile_place(const TileGeom &tg, int nx, int ny, int nz, int t) {
    TilePlace tp;
    const int tzi = t % tg.ntz, tyi = (t / tg.ntz) % tg.nty, txi = t / (tg.ntz * tg.nty);
    tp.c0[0] = txi * tg.tx;
    tp.c0[1] = tyi * tg.ty;
    tp.c0[2] = tzi * tg.tz;
    int ox = (tp.c0[0] - tg.halo) % nx; ox += ox < 0 ? nx : 0;
    int oy = (tp.c0[1] - tg.halo) % ny; oy += oy < 0 ? ny : 0;
    int oz = (tp.c0[2] - tg.halo) % nz; oz += oz < 0 ? nz : 0;
    tp.ox = ox; tp.oy = oy; tp.oz = oz;
    return tp;
}

// Stages the node fields of the region with origin (ox, oy, oz) in LDS,
// node-major, in the particle precision.
template <typename TP, typename TF>
__device__ __forceinline__ void stage_fields(const FieldPtrs<TF> &f, const TileGeom &tg, int nx, int ny, int nz,
                                             int ox, int oy, int oz, LdsFieldNode<TP> *__restrict__ fl) {
    const int RL = tg.rx * tg.ry * tg.rz;  // logical region nodes
    for (int r = threadIdx.x; r < RL; r += blockDim.x) {
        const RegionNode rn = region_node(tg, nx, ny, nz, ox, oy, oz, r);
        LdsFieldNode<TP> fn;
#pragma unroll
        for (int m = 0; m < 6; ++m) fn.v[m] = (TP)f.f[m][rn.gnode];
        fl[rn.slot] = fn;
    }
}

// Adds the region accumulator [10][rnp] to the global moments, skipping
// exact zeros (halo nodes no particle reached); consecutive threads take
// consecutive region nodes, so each moment's atomics are coalesced along
// the fast axis.
template <typename TA>
__device__ __forceinline__ void flush_region(const TileGeom &tg, int nx, int ny, int nz, int ox, int oy, int oz,
                                             const TA *__restrict__ ml, TA *__restrict__ mom, int nn) {
    const int RL = tg.rx * tg.ry * tg.rz, RNP = tg.rnp;
    for (int r = threadIdx.x; r < RL; r += blockDim.x) {
        const RegionNode rn = region_node(tg, nx, ny, nz, ox, oy, oz, r);
#pragma unroll
        for (int m = 0; m < 10; ++m) {
            const TA val = ml[m * RNP + rn.slot];
            if (val != TA(0)) atomicAdd(mom + (size_t)m * nn + rn.gnode, val);
        }
    }
}

// The first particle of thread k's slots in a tile (beg + k), loaded by the
// caller before it stages the tile's fields, so the load overlaps that
// staging and its barrier instead of following them.
template <typename TP>
struct FirstRec {
    TP x, y, z, u, v, w, q;
    int64_t id;
};

template <typename TP, typename TF, typename TA>
__device__ __forceinline__ FirstRec<TP> load_first(const TileJob<TP, TF, TA> &J, uint32_t beg, uint32_t end) {
    FirstRec<TP> r{};
    const uint32_t i = beg + threadIdx.x;
    const PartPtrs<TP> &pin = J.in;
    if (i < end) {
        const uint32_t o = i * (uint32_t)sizeof(TP);
        r.x = ld32(pin.x, o); r.y = ld32(pin.y, o); r.z = ld32(pin.z, o);
        r.u = ld32(pin.u, o); r.v = ld32(pin.v, o); r.w = ld32(pin.w, o); r.q = ld32(pin.q, o);
        if (J.copy_rest && pin.id) r.id = pin.id[i];
    }
    return r;
}

// Moves the particles [beg, end) of one tile (Eq. 1, Eq. 2, Eq. 5),
// gathering E and B (Eq. 3, Eq. 4) from the region fields `fl` staged with
// origin (ox, oy, oz), and stores the new state.  Thread k takes slots
// beg + k, beg + k + blockDim.x, ... (the first one in `first`, from
// load_first); the loop is uniform per wave, and
// after each slot every lane calls done(i, valid, x, y, z, u, v, w, q) with
// the moved particle (valid is false past the range, where the values are
// stale).
template <typename TP, typename TF, typename TA, bool CACHE, typename Done>
__device__ __forceinline__ void move_tile(const TileJob<TP, TF, TA> &J, const TileGeom &tg,
                                          const LdsFieldNode<TP> *__restrict__ fl, int ox, int oy, int oz,
                                          uint32_t beg, uint32_t end, const FirstRec<TP> &first, Done &&done) {
    const GridT<TP> &g = J.g;
    const FieldPtrs<TF> &f = J.f;
    const PartPtrs<TP> &p = J.p;
    const int sx = tg.sx, sy = tg.sy, sz = tg.sz;
    const int coff[8] = {0, sx, sy, sx + sy, sz, sx + sz, sy + sz, sx + sy + sz};
    LdsFieldNode<TP> corner[CACHE ? 8 : 1];  // field corners of the cell `cached`
    int cached = -1;

    const uint32_t stride = blockDim.x;
    constexpr uint32_t ES = sizeof(TP);
    uint32_t i = beg + threadIdx.x;
    TP nx_ = first.x, ny_ = first.y, nz_ = first.z, nu_ = first.u, nv_ = first.v, nw_ = first.w, nq_ = first.q;
    int64_t nid_ = first.id;
    const PartPtrs<TP> &pin = J.in;
    const bool copy_id = J.copy_rest && pin.id;  // ids move with the sort's copy
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
        if (valid) {
            implicit_move(
                g, J.mv,
                [&](TP px, TP py, TP pz, TP F[6]) {
                    // the cell of the point (the same arithmetic as the
                    // unsorted path's locate, so both give the same bits)
                    // and its place in the region
                    Cell<TP> c;
                    const int i = plocate(px, g.L[0], g.invL[0], g.invd[0], g.nx, c.fx);
                    const int j = plocate(py, g.L[1], g.invL[1], g.invd[1], g.ny, c.fy);
                    const int k = plocate(pz, g.L[2], g.invL[2], g.invd[2], g.nz, c.fz);
                    int di = i - ox, dj = j - oy, dk = k - oz;
                    di += di < 0 ? g.nx : 0;
                    dj += dj < 0 ? g.ny : 0;
                    dk += dk < 0 ? g.nz : 0;
                    const bool in = di < tg.rx - 1 && dj < tg.ry - 1 && dk < tg.rz - 1;
                    const int rb = di * sx + dj * sy + dk * sz;
                    if (in) {
                        if constexpr (!CACHE) {
                            gather_lds(fl, tg, rb, c, F);
                        } else {
                            // the corners of the last LDS cell stay in
                            // registers: a thread's particles share their sort cell
                            if (rb != cached) {
#pragma unroll
                                for (int q = 0; q < 8; ++q) corner[q] = fl[rb + coff[q]];
                                cached = rb;
                            }
                            TP w[8];
                            pweights(c.fx, c.fy, c.fz, w);
#pragma unroll
                            for (int m = 0; m < 6; ++m) F[m] = TP(0);
#pragma unroll
                            for (int q = 0; q < 8; ++q)
#pragma unroll
                                for (int m = 0; m < 6; ++m) F[m] += w[q] * corner[q].v[m];
                        }
                    } else {  // rare: outside the region, from global memory
                        const int nyz = g.ny * g.nz;
                        c.base = i * nyz + j * g.nz + k;
                        c.ox = (i == g.nx - 1) ? -(g.nx - 1) * nyz : nyz;
                        c.oy = (j == g.ny - 1) ? -(g.ny - 1) * g.nz : g.nz;
                        c.oz = (k == g.nz - 1) ? -(g.nz - 1) : 1;
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
        }
        done(i, valid, xn, yn, zn, un, vn, wn, qp);
    }
}

// One tile of one species: stage the region's fields, move the tile's
// particles and (unless MOVE_ONLY or J.mom is NULL) deposit each moved
// particle with FP64 LDS atomics, then flush the region's moments.  Called
// by the per-species tiled kernel and by the work-list kernels of the batch
// engine; `t` is uniform across the workgroup.
template <typename TP, typename TF, typename TA, bool CACHE, bool MOVE_ONLY, class GEO>
__device__ __forceinline__ void tile_body(const TileJob<TP, TF, TA> &J, int t, unsigned char *smem) {
    const GridT<TP> &g = J.g;
    TileGeom tg = J.tg;
    apply_geo<GEO>(tg);
    TA *__restrict__ mom = MOVE_ONLY ? nullptr : J.mom;
    const int nn = J.nn;
    const uint32_t beg = J.tile_off[t], end = J.tile_off[t + 1];
    if (beg == end) return;  // uniform: no particle in this tile

    const int RNP = tg.rnp;
    const size_t fbytes = (RNP * sizeof(LdsFieldNode<TP>) + 15) & ~(size_t)15;
    LdsFieldNode<TP> *fl = (LdsFieldNode<TP> *)smem;
    TA *ml = (TA *)(smem + fbytes);
    const TilePlace tp = tile_place(tg, g.nx, g.ny, g.nz, t);
    const int ox = tp.ox, oy = tp.oy, oz = tp.oz;

    // the first particle in flight while the region's node fields are
    // staged and its moments zeroed
    const FirstRec<TP> first = load_first(J, beg, end);
    stage_fields<TP, TF>(J.f, tg, g.nx, g.ny, g.nz, ox, oy, oz, fl);
    if (mom)
        for (int q = threadIdx.x; q < 10 * RNP; q += blockDim.x) ml[q] = TA(0);
    __syncthreads();

    move_tile<TP, TF, TA, CACHE>(J, tg, fl, ox, oy, oz, beg, end, first,
                                 [&](uint32_t, bool valid, TP xn, TP yn, TP zn, TP un, TP vn, TP wn, TP qp)
                                     __attribute__((always_inline)) {
                                         // deposit of the new state in the accumulation precision
                                         if (valid && mom)
                                             deposit_one<TA, GEO>(J.ga, tg, ox, oy, oz, ml, mom, nn, (TA)xn,
                                                                  (TA)yn, (TA)zn, (TA)qp, (TA)un, (TA)vn, (TA)wn);
                                     });
    if (!mom) return;
    __syncthreads();
    flush_region(tg, g.nx, g.ny, g.nz, ox, oy, oz, ml, mom, nn);
}

// ------------------------------------------------------- sorted deposit
//
// kDepCap indices per cell hold the particles that moved into a tile cell
// other than the one their slot belongs to; kDepOutCap those that left the
// tile or found their bin full (16-bit indices into the tile's range).  The
// bins are drained by the cell's owner lanes, so the fullest bin sets the
// length of the drain; past kDepCap a particle is cheaper in the out list,
// which is deposited 64 at a time (measured on the 128x64x32 box: 24 beats
// 48, 32, 16, 12 and 8).  In the pass over the rows kDepPrefetch particles
// per thread are in flight while one is deposited.
constexpr int kDepCap = 24;
constexpr int kDepOutCap = 2048;
constexpr int kDepPrefetch = 2;
constexpr int kDepWaves = 3;  // register budget: waves per SIMD (FP32 particles)

// LDS of the sorted deposit: [10][rnp] moments in TA (dense layout), the
// per-cell bin counts (64), the out count and the overflow flag, the bins
// (64 x kDepCap indices) and the out list, and per wave a balancing stage
// for the particles that left the tile.
inline size_t deposit_lds_bytes(int rnp, int block, int tp_bytes, int ta_bytes) {
    const size_t mom = ((size_t)10 * rnp * ta_bytes + 15) & ~(size_t)15;
    const size_t counts = 80 * sizeof(int);
    const size_t lists = (((size_t)64 * kDepCap + kDepOutCap) * sizeof(uint16_t) + 15) & ~(size_t)15;
    const size_t stage = (size_t)(block / 64) * (64 * 8 * tp_bytes + sizeof(BalanceLds));
    return mom + counts + lists + stage;
}

// Cell index and in-cell offset along one axis of a moved (already wrapped)
// position, branch free: i = min(floor(x / dx), n - 1), f = x / dx - i.  A
// position that its conversion to the accumulation precision put on L
// falls in cell n - 1 with f = 1, which deposits on node n = node 0 as the
// wrapped position would (to rounding); the clamp keeps any index in range.
template <typename T>
__device__ __forceinline__ int dep_locate(T s, T invd, int n, T &f) {
    const T t = cell_coord(s, invd);
    int i = (int)t;
    i = i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
    f = t - (T)i;
    return i;
}

// Local index of a tile cell from its offsets inside the tile: the slow
// axis slowest, the fast axis fastest (the order of spic_sort.hip's keys,
// so lane l of a row of a sorted tile holds cell l).
__device__ __forceinline__ int local_cell(const TileGeom &tg, const int d[3]) {
    const int t3[3] = {tg.tx, tg.ty, tg.tz};
    return (d[tg.slow] * t3[tg.mid] + d[tg.mid]) * t3[tg.fast] + d[tg.fast];
}

// The sorted deposit of one tile.  Lane l of every wave owns local cell l
// of the tile and keeps the moments of its 8 nodes (80 sums) in registers.
// The tile's range is taken in rows of 64 slots (after a sort in full rows
// slot (r, l) holds a particle of cell l): a particle in its slot's cell is
// added to the lane's sums at once; one that moved to another cell of the
// tile is binned by its new cell (an index in LDS), one that left the tile
// (or found its bin full) goes to the out list (dep_route).  Then lane
// (w, l) adds the entries w, w + W, ... of cell l's bin to its sums, the
// sums are added to the region, and the out list is deposited 64 at a time,
// bank-balanced, with FP64 terms and LDS atomics (global atomics beyond the
// region) (dep_drain).  A tile whose out list overflows (or of 65536
// particles or more) drops the sums and lists and deposits every particle
// with LDS atomics instead.  The region is then flushed to the global
// moments (dep_finish).
//
// DepTile holds the tile's LDS (moments [10][rnp] in the dense layout, bin
// counts, out count and overflow flag, bins, out list, the wave's
// balancing stage) and the lane's cell.
template <typename TP, typename TA>
struct DepTile {
    TileGeom tg;  // the moments' region, dense layout
    TilePlace tp;
    TA *ml;
    int *bcnt, *ocnt, *oflow;
    uint16_t *bins, *olist;
    StagedParticle<TP> *stage;
    BalanceLds *bal;
    uint32_t beg, end;
    int C, nwv, wv, lane, lslot;
    bool owner;
};

// Opens the deposit of tile t (particles [beg, end)) in smem: zeroes the
// region and the counts.  The caller synchronises before the first route.
template <typename TP, typename TA, class GEO>
__device__ __forceinline__ DepTile<TP, TA> dep_open(const GridT<TA> &ga, TileGeom tg, int t, uint32_t beg,
                                                    uint32_t end, unsigned char *smem) {
    apply_geo<GEO>(tg);
    if constexpr (!GEO::fixed) {  // the dense layout of the moments
        const int r3[3] = {tg.rx, tg.ry, tg.rz};
        int st[3];
        st[tg.fast] = 1;
        st[tg.mid] = r3[tg.fast];
        st[tg.slow] = r3[tg.fast] * r3[tg.mid];
        tg.sx = st[0]; tg.sy = st[1]; tg.sz = st[2];
        tg.rnp = tg.rx * tg.ry * tg.rz;
    }
    DepTile<TP, TA> d;
    const int RNP = tg.rnp;
    d.tg = tg;
    d.beg = beg;
    d.end = end;
    d.C = tg.cells;
    d.nwv = blockDim.x >> 6;
    d.wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
    d.lane = threadIdx.x & 63;
    d.ml = (TA *)smem;
    d.bcnt = (int *)(smem + (((size_t)10 * RNP * sizeof(TA) + 15) & ~(size_t)15));
    d.ocnt = d.bcnt + 64;
    d.oflow = d.bcnt + 65;
    d.bins = (uint16_t *)(d.bcnt + 80);
    d.olist = d.bins + 64 * kDepCap;
    unsigned char *mine = (unsigned char *)d.bins +
                          ((((size_t)64 * kDepCap + kDepOutCap) * sizeof(uint16_t) + 15) & ~(size_t)15) +
                          d.wv * (64 * sizeof(StagedParticle<TP>) + sizeof(BalanceLds));
    d.stage = (StagedParticle<TP> *)mine;
    d.bal = (BalanceLds *)(mine + 64 * sizeof(StagedParticle<TP>));
    d.tp = tile_place(tg, ga.nx, ga.ny, ga.nz, t);
    // the cell this lane owns: local index `lane` (lanes >= C own none)
    const int t3[3] = {tg.tx, tg.ty, tg.tz};
    int lc[3];
    lc[tg.fast] = d.lane % t3[tg.fast];
    lc[tg.mid] = (d.lane / t3[tg.fast]) % t3[tg.mid];
    lc[tg.slow] = d.lane / (t3[tg.fast] * t3[tg.mid]);
    d.owner = d.lane < d.C;
    d.lslot = (tg.halo + lc[0]) * tg.sx + (tg.halo + lc[1]) * tg.sy + (tg.halo + lc[2]) * tg.sz;
    for (int q = threadIdx.x; q < 10 * RNP; q += blockDim.x) d.ml[q] = TA(0);
    // the 64 bin counts, the out count and the overflow flag
    for (int q = threadIdx.x; q < 66; q += blockDim.x) d.bcnt[q] = (q == 65 && end - beg >= 65536u) ? 1 : 0;
    return d;
}

// A particle record (x, y, z, u, v, w, q) of slot i; an index past the
// range is clamped to the tile's last particle (read and ignored), so a
// prefetch slot is refilled in place.
template <typename TP, typename TA>
__device__ __forceinline__ void dep_load(const PartPtrs<TP> &p, const DepTile<TP, TA> &d, TP (&dst)[7],
                                         uint32_t i) {
    const uint32_t o = min(i, d.end - 1) * (uint32_t)sizeof(TP);
    dst[0] = ld32(p.x, o); dst[1] = ld32(p.y, o); dst[2] = ld32(p.z, o);
    dst[3] = ld32(p.u, o); dst[4] = ld32(p.v, o); dst[5] = ld32(p.w, o); dst[6] = ld32(p.q, o);
}

// A particle into the lane's sums: in-cell offsets in the accumulation
// precision, the weighted charge rounded once to the particle precision,
// the ten terms and their sums in the particle precision.  Branch free: a
// particle that is not the lane's adds its terms with zero charge (a
// conditional add would make the compiler copy all 80 sums at the join).
template <typename TP, typename TA>
__device__ __forceinline__ void dep_add_terms(TP (&sacc)[80], const TP (&rec)[7], TA fx, TA fy, TA fz,
                                              bool take) {
    const TA qa = take ? (TA)rec[6] : TA(0);
    const TA gx = TA(1) - fx, gy = TA(1) - fy, gz = TA(1) - fz;
    const TP u = rec[3], v = rec[4], w = rec[5];
    const TP val[10] = {TP(1), u, v, w, u * u, u * v, u * w, v * v, v * w, w * w};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const TA wk = (((k & 1) ? fx : gx) * ((k & 2) ? fy : gy)) * ((k & 4) ? fz : gz);
        const TP qw = (TP)(qa * wk);
#pragma unroll
        for (int m = 0; m < 10; ++m) sacc[k * 10 + m] += qw * val[m];
    }
}

// The particle's local tile cell (C when it left the tile); its terms are
// added when the cell is the lane's and mine_p holds.
template <typename TP, typename TA>
__device__ __forceinline__ int dep_add_own(const DepTile<TP, TA> &d, const GridT<TA> &ga, TP (&sacc)[80],
                                           const TP (&rec)[7], bool mine_p) {
    TA fx, fy, fz;
    int c[3];
    c[0] = dep_locate((TA)rec[0], ga.invd[0], ga.nx, fx) - d.tp.c0[0];
    c[1] = dep_locate((TA)rec[1], ga.invd[1], ga.ny, fy) - d.tp.c0[1];
    c[2] = dep_locate((TA)rec[2], ga.invd[2], ga.nz, fz) - d.tp.c0[2];
    const bool in = (unsigned)c[0] < (unsigned)d.tg.tx && (unsigned)c[1] < (unsigned)d.tg.ty &&
                    (unsigned)c[2] < (unsigned)d.tg.tz;
    const int cell = in ? local_cell(d.tg, c) : d.C;
    dep_add_terms(sacc, rec, fx, fy, fz, mine_p && d.owner && cell == d.lane);
    return cell;
}

// Routes the moved particle of slot i (valid false past the range): into
// the lane's sums, its new cell's bin, or the out list (a full bin or a
// cell outside the tile; positions counted once per wave).
template <typename TP, typename TA>
__device__ __forceinline__ void dep_route(const DepTile<TP, TA> &d, const GridT<TA> &ga, TP (&sacc)[80],
                                          const TP (&rec)[7], uint32_t i, bool valid) {
    const int cell = dep_add_own(d, ga, sacc, rec, valid);
    const bool drift = valid && !(d.owner && cell == d.lane);
    bool out = drift && cell >= d.C;
    if (drift && !out) {
        const int pos = atomicAdd(&d.bcnt[cell], 1);
        if (pos < kDepCap) d.bins[cell * kDepCap + pos] = (uint16_t)(i - d.beg);
        else out = true;
    }
    const unsigned long long om = __ballot(out);
    if (om) {
        const int lead = __ffsll((long long)om) - 1;
        int b0 = 0;
        if (d.lane == lead) b0 = atomicAdd(d.ocnt, __popcll(om));
        const int opos = __shfl(b0, lead) + __popcll(om & ((1ull << d.lane) - 1ull));
        if (out && opos < kDepOutCap) d.olist[opos] = (uint16_t)(i - d.beg);
        if (out && opos >= kDepOutCap) *d.oflow = 1;
    }
}

// After the barrier that follows the last route, when the out list has not
// overflowed: drains the bins into the sums (reloading those particles
// from p), then adds the sums and the out list to the region.
template <typename TP, typename TA, class GEO>
__device__ __forceinline__ void dep_drain(const DepTile<TP, TA> &d, const GridT<TA> &ga, const PartPtrs<TP> &p,
                                          TA *__restrict__ mom, int nn, TP (&sacc)[80]) {
    const TileGeom &tg = d.tg;
    const int RNP = tg.rnp, sx = tg.sx, sy = tg.sy, sz = tg.sz;
    // the bins: lane (wv, l) takes entries wv, wv + W, ... of cell l's
    const int mc = d.owner ? min(d.bcnt[d.lane], kDepCap) : 0;
    const int mine_n = mc > d.wv ? (mc - d.wv + d.nwv - 1) / d.nwv : 0;
    // an empty bin's first entry may be stale: it is loaded (clamped into
    // the range) and added with zero charge
    auto at = [&](int m) __attribute__((always_inline)) -> uint32_t {
        const int j = max(min(d.wv + m * d.nwv, mc - 1), 0);
        return d.beg + d.bins[(d.owner ? d.lane : 0) * kDepCap + j];
    };
    TP ring[kDepPrefetch][7];
#pragma unroll
    for (int k = 0; k < kDepPrefetch; ++k) dep_load(p, d, ring[k], at(k));
    for (int m0 = 0; __ballot(m0 < mine_n); m0 += kDepPrefetch) {
#pragma unroll
        for (int k = 0; k < kDepPrefetch; ++k) {
            (void)dep_add_own(d, ga, sacc, ring[k], m0 + k < mine_n);
            dep_load(p, d, ring[k], at(m0 + k + kDepPrefetch));
        }
    }
    // the sums stay in the particle precision until here
    settle(sacc);
    if (d.owner) {
        const int coff[8] = {0, sx, sy, sx + sy, sz, sx + sz, sy + sz, sx + sy + sz};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            TA *dst = d.ml + d.lslot + coff[k];
#pragma unroll
            for (int m = 0; m < 10; ++m) atomicAdd(dst + m * RNP, (TA)sacc[k * 10 + m]);
        }
    }
    // the particles that left the tile (or found their bin full), 64 per
    // wave at a time, bank-balanced LDS atomics (a halo cell gets too few of
    // them, and the cells next to the tile's faces too many, for lanes
    // owning halo cells to pay off)
    const int no = *d.ocnt;
    for (int b0 = d.wv * 64; b0 < no; b0 += (int)blockDim.x) {
        const int e = b0 + d.lane;
        TP rec[7];
        dep_load(p, d, rec, d.beg + d.olist[min(e, no - 1)]);
        deposit_balanced<TP, TA, GEO>(ga, tg, d.tp.ox, d.tp.oy, d.tp.oz, d.ml, mom, nn, d.stage, d.bal, d.lane,
                                      e < no, rec[0], rec[1], rec[2], rec[3], rec[4], rec[5], rec[6]);
    }
}

// Ends the deposit: after an overflow every particle of the range goes to
// the region by LDS atomics (the sums and lists are dropped); then the
// region is flushed to the global moments.
template <typename TP, typename TA, class GEO>
__device__ __forceinline__ void dep_finish(const DepTile<TP, TA> &d, const GridT<TA> &ga, const PartPtrs<TP> &p,
                                           TA *__restrict__ mom, int nn) {
    const TileGeom &tg = d.tg;
    const int ox = d.tp.ox, oy = d.tp.oy, oz = d.tp.oz;
    if (*d.oflow) {  // uniform
        for (uint32_t i0 = d.beg + (threadIdx.x & ~63u); i0 < d.end; i0 += blockDim.x) {
            const uint32_t i = i0 + d.lane;
            TP rec[7];
            dep_load(p, d, rec, i);
            deposit_balanced<TP, TA, GEO>(ga, tg, ox, oy, oz, d.ml, mom, nn, d.stage, d.bal, d.lane, i < d.end,
                                          rec[0], rec[1], rec[2], rec[3], rec[4], rec[5], rec[6]);
        }
    }
    __syncthreads();
    flush_region(tg, ga.nx, ga.ny, ga.nz, ox, oy, oz, d.ml, mom, nn);
}

// Deposit of the moved particles of tile t (the second launch of variant
// 2): the sorted deposit described above, over rows of 64 slots read
// coalesced with kDepPrefetch rows per thread in flight.  It performs the
// steps of dep_open, dep_route, dep_drain and dep_finish with its own
// locals rather than through DepTile: written through the helpers, this
// kernel keeps more values live across its bin drain, spills twice as many
// registers there, and runs about a tenth slower.
template <typename TP, typename TF, typename TA, class GEO>
__device__ __forceinline__ void deposit_body(const TileJob<TP, TF, TA> &J, int t, unsigned char *smem) {
    TileGeom tg = J.tg;
    apply_geo<GEO>(tg);
    if constexpr (!GEO::fixed) {  // the dense layout of the moments
        const int r3[3] = {tg.rx, tg.ry, tg.rz};
        int st[3];
        st[tg.fast] = 1;
        st[tg.mid] = r3[tg.fast];
        st[tg.slow] = r3[tg.fast] * r3[tg.mid];
        tg.sx = st[0]; tg.sy = st[1]; tg.sz = st[2];
        tg.rnp = tg.rx * tg.ry * tg.rz;
    }
    const GridT<TA> &ga = J.ga;
    const PartPtrs<TP> &p = J.p;
    TA *__restrict__ mom = J.mom;
    const int nn = J.nn;
    const uint32_t beg = J.tile_off[t], end = J.tile_off[t + 1];
    if (beg == end) return;
    const int RNP = tg.rnp, C = tg.cells;
    // the wave index is uniform per wave: held in a scalar register it frees
    // the vector registers the 80 sums need (fewer spills in the bin drain)
    const int nwv = blockDim.x >> 6, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    TA *ml = (TA *)smem;
    int *bcnt = (int *)(smem + (((size_t)10 * RNP * sizeof(TA) + 15) & ~(size_t)15));
    int *ocnt = bcnt + 64;
    int *oflow = bcnt + 65;
    uint16_t *bins = (uint16_t *)(bcnt + 80);
    uint16_t *olist = bins + 64 * kDepCap;
    unsigned char *mine = (unsigned char *)bins +
                          ((((size_t)64 * kDepCap + kDepOutCap) * sizeof(uint16_t) + 15) & ~(size_t)15) +
                          wv * (64 * sizeof(StagedParticle<TP>) + sizeof(BalanceLds));
    StagedParticle<TP> *stage = (StagedParticle<TP> *)mine;
    BalanceLds *bal = (BalanceLds *)(mine + 64 * sizeof(StagedParticle<TP>));

    constexpr uint32_t ES = sizeof(TP);
    // unconditional loads (an index past the range is clamped to the
    // tile's last particle, read and ignored), so a slot is refilled in place
    auto load = [&](TP (&dst)[7], uint32_t i) __attribute__((always_inline)) {
        const uint32_t o = min(i, end - 1) * ES;
        dst[0] = ld32(p.x, o); dst[1] = ld32(p.y, o); dst[2] = ld32(p.z, o);
        dst[3] = ld32(p.u, o); dst[4] = ld32(p.v, o); dst[5] = ld32(p.w, o); dst[6] = ld32(p.q, o);
    };
    // the first kDepPrefetch rows are in flight while the region and the
    // counts are zeroed (unused if the tile turns out to overflow)
    const uint32_t stride = blockDim.x;
    uint32_t ii = beg + threadIdx.x;
    TP ring[kDepPrefetch][7];
#pragma unroll
    for (int k = 0; k < kDepPrefetch; ++k) load(ring[k], ii + k * stride);

    const TilePlace tp = tile_place(tg, ga.nx, ga.ny, ga.nz, t);
    const int ox = tp.ox, oy = tp.oy, oz = tp.oz;
    const int RL = tg.rx * tg.ry * tg.rz;
    const int sx = tg.sx, sy = tg.sy, sz = tg.sz;
    for (int q = threadIdx.x; q < 10 * RNP; q += blockDim.x) ml[q] = TA(0);
    // the 64 bin counts, the out count and the overflow flag
    for (int q = threadIdx.x; q < 66; q += blockDim.x) bcnt[q] = (q == 65 && end - beg >= 65536u) ? 1 : 0;
    __syncthreads();

    // the cell this lane owns: local index `lane` (lanes >= C own none)
    const int t3[3] = {tg.tx, tg.ty, tg.tz};
    int lc[3];
    lc[tg.fast] = lane % t3[tg.fast];
    lc[tg.mid] = (lane / t3[tg.fast]) % t3[tg.mid];
    lc[tg.slow] = lane / (t3[tg.fast] * t3[tg.mid]);
    const bool owner = lane < C;
    const int lslot = (tg.halo + lc[0]) * sx + (tg.halo + lc[1]) * sy + (tg.halo + lc[2]) * sz;

    if (!*oflow) {
        TP sacc[80];
#pragma unroll
        for (int q = 0; q < 80; ++q) sacc[q] = TP(0);
        // a particle into the lane's sums: in-cell offsets in the
        // accumulation precision, the weighted charge rounded once to the
        // particle precision, the ten terms and their sums in the particle
        // precision.  Branch free: a particle that is not the lane's adds
        // its terms with zero charge (a conditional add would make the
        // compiler copy all 80 sums at the join).
        auto add_terms = [&](const TP (&rec)[7], TA fx, TA fy, TA fz, bool take) __attribute__((always_inline)) {
            const TA qa = take ? (TA)rec[6] : TA(0);
            const TA gx = TA(1) - fx, gy = TA(1) - fy, gz = TA(1) - fz;
            const TP u = rec[3], v = rec[4], w = rec[5];
            const TP val[10] = {TP(1), u, v, w, u * u, u * v, u * w, v * v, v * w, w * w};
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const TA wk = (((k & 1) ? fx : gx) * ((k & 2) ? fy : gy)) * ((k & 4) ? fz : gz);
                const TP qw = (TP)(qa * wk);
#pragma unroll
                for (int m = 0; m < 10; ++m) sacc[k * 10 + m] += qw * val[m];
            }
        };
        // the particle's local tile cell (C when it left the tile), added
        // when it is this lane's and mine_p holds
        auto add_own = [&](const TP (&rec)[7], bool mine_p) __attribute__((always_inline)) -> int {
            TA fx, fy, fz;
            int d[3];
            d[0] = dep_locate((TA)rec[0], ga.invd[0], ga.nx, fx) - tp.c0[0];
            d[1] = dep_locate((TA)rec[1], ga.invd[1], ga.ny, fy) - tp.c0[1];
            d[2] = dep_locate((TA)rec[2], ga.invd[2], ga.nz, fz) - tp.c0[2];
            const bool in = (unsigned)d[0] < (unsigned)t3[0] && (unsigned)d[1] < (unsigned)t3[1] &&
                            (unsigned)d[2] < (unsigned)t3[2];
            const int cell = in ? local_cell(tg, d) : C;
            add_terms(rec, fx, fy, fz, mine_p && owner && cell == lane);
            return cell;
        };

        // rows of 64 slots, lane l on slot l of each row (ring and ii from
        // the loads issued before the zeroing)
        {
            for (uint32_t i0 = beg + (threadIdx.x & ~63u); i0 < end; i0 += kDepPrefetch * stride,
                          ii += kDepPrefetch * stride) {
#pragma unroll
                for (int k = 0; k < kDepPrefetch; ++k) {
                    const uint32_t i = ii + k * stride;
                    const bool valid = i < end;
                    const int cell = add_own(ring[k], valid);
                    const bool drift = valid && !(owner && cell == lane);
                    // into the cell's bin; a full bin or a cell outside the
                    // tile: the out list (positions counted once per wave)
                    bool out = drift && cell >= C;
                    if (drift && !out) {
                        const int pos = atomicAdd(&bcnt[cell], 1);
                        if (pos < kDepCap) bins[cell * kDepCap + pos] = (uint16_t)(i - beg);
                        else out = true;
                    }
                    const unsigned long long om = __ballot(out);
                    if (om) {
                        const int lead = __ffsll((long long)om) - 1;
                        int b0 = 0;
                        if (lane == lead) b0 = atomicAdd(ocnt, __popcll(om));
                        const int opos = __shfl(b0, lead) + __popcll(om & ((1ull << lane) - 1ull));
                        if (out && opos < kDepOutCap) olist[opos] = (uint16_t)(i - beg);
                        if (out && opos >= kDepOutCap) *oflow = 1;
                    }
                    load(ring[k], i + kDepPrefetch * stride);
                }
            }
        }
        __syncthreads();
        if (!*oflow) {  // uniform
            // the bins: lane (wv, l) takes entries wv, wv + W, ... of cell l's
            const int mc = owner ? min(bcnt[lane], kDepCap) : 0;
            const int mine_n = mc > wv ? (mc - wv + nwv - 1) / nwv : 0;
            // an empty bin's first entry may be stale: it is loaded (clamped
            // into the range) and added with zero charge
            auto at = [&](int m) __attribute__((always_inline)) -> uint32_t {
                const int j = max(min(wv + m * nwv, mc - 1), 0);
                return beg + bins[(owner ? lane : 0) * kDepCap + j];
            };
            // one entry in flight: a second slot here costs the kernel ten
            // spilled VGPRs, whose reloads then wait for every load in flight
            TP dr[7];
            load(dr, at(0));
            for (int m0 = 0; __ballot(m0 < mine_n); ++m0) {
                (void)add_own(dr, m0 < mine_n);
                load(dr, at(m0 + 1));
            }
            // the sums stay in the particle precision until here
            settle(sacc);
            // the particles that left the tile (or found their bin full),
            // 64 per wave at a time, bank-balanced LDS atomics (a halo cell
            // gets too few of them, and the cells next to the tile's faces
            // too many, for lanes owning halo cells to pay off); the wave's
            // first 64 are loaded before the sums go to the region
            const int no = *ocnt;
            int b0 = wv * 64;
            TP rec[7];
            if (b0 < no) load(rec, beg + olist[min(b0 + lane, no - 1)]);  // uniform
            if (owner) {
                const int coff[8] = {0, sx, sy, sx + sy, sz, sx + sz, sy + sz, sx + sy + sz};
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    TA *dst = ml + lslot + coff[k];
#pragma unroll
                    for (int m = 0; m < 10; ++m) atomicAdd(dst + m * RNP, (TA)sacc[k * 10 + m]);
                }
            }
            for (; b0 < no; b0 += (int)blockDim.x) {
                const int e = b0 + lane;
                deposit_balanced<TP, TA, GEO>(ga, tg, ox, oy, oz, ml, mom, nn, stage, bal, lane, e < no, rec[0],
                                              rec[1], rec[2], rec[3], rec[4], rec[5], rec[6]);
                const int en = b0 + (int)blockDim.x;
                if (en < no) load(rec, beg + olist[min(en + lane, no - 1)]);  // uniform
            }
        }
    }
    if (*oflow) {  // uniform: every particle by LDS (or global) atomics
        for (uint32_t i0 = beg + (threadIdx.x & ~63u); i0 < end; i0 += blockDim.x) {
            const uint32_t i = i0 + lane;
            TP rec[7];
            load(rec, i);
            deposit_balanced<TP, TA, GEO>(ga, tg, ox, oy, oz, ml, mom, nn, stage, bal, lane, i < end, rec[0], rec[1],
                                          rec[2], rec[3], rec[4], rec[5], rec[6]);
        }
    }
    __syncthreads();
    for (int r = threadIdx.x; r < RL; r += blockDim.x) {
        const RegionNode rn = region_node(tg, ga.nx, ga.ny, ga.nz, ox, oy, oz, r);
#pragma unroll
        for (int m = 0; m < 10; ++m) {
            const TA val = ml[m * RNP + rn.slot];
            if (val != TA(0)) atomicAdd(mom + (size_t)m * nn + rn.gnode, val);
        }
    }
}

// One tile in one launch (variant 3): variant 1's mover (the fields of a
// region with the mover's halo in LDS, the field corners of the lane's cell
// in registers) hands each moved particle straight to the sorted deposit's
// route, so only the binned and out-listed particles are read again (after
// the barrier, from the arrays this workgroup has just written).  J.tg is
// the mover's region (GEOF), tgm the moments' (GEOM, dense layout).
template <typename TP, typename TF, typename TA, bool CACHE, class GEOF, class GEOM>
__device__ __forceinline__ void lanecell_body(const TileJob<TP, TF, TA> &J, const TileGeom &tgm, int t,
                                              unsigned char *smem) {
    const GridT<TP> &g = J.g;
    TileGeom tg = J.tg;
    apply_geo<GEOF>(tg);
    const uint32_t beg = J.tile_off[t], end = J.tile_off[t + 1];
    if (beg == end) return;
    LdsFieldNode<TP> *fl = (LdsFieldNode<TP> *)smem;
    const size_t fbytes = (tg.rnp * sizeof(LdsFieldNode<TP>) + 15) & ~(size_t)15;
    const DepTile<TP, TA> d = dep_open<TP, TA, GEOM>(J.ga, tgm, t, beg, end, smem + fbytes);
    const TilePlace tp = tile_place(tg, g.nx, g.ny, g.nz, t);
    const FirstRec<TP> first = load_first(J, beg, end);
    stage_fields<TP, TF>(J.f, tg, g.nx, g.ny, g.nz, tp.ox, tp.oy, tp.oz, fl);
    __syncthreads();
    TP sacc[80];
#pragma unroll
    for (int q = 0; q < 80; ++q) sacc[q] = TP(0);
    move_tile<TP, TF, TA, CACHE>(J, tg, fl, tp.ox, tp.oy, tp.oz, beg, end, first,
                                [&](uint32_t i, bool valid, TP x, TP y, TP z, TP u, TP v, TP w, TP q)
                                    __attribute__((always_inline)) {
                                        const TP rec[7] = {x, y, z, u, v, w, q};
                                        dep_route(d, J.ga, sacc, rec, i, valid);
                                    });
    __syncthreads();
    if (!*d.oflow) dep_drain<TP, TA, GEOM>(d, J.ga, J.p, J.mom, J.nn, sacc);  // uniform
    dep_finish<TP, TA, GEOM>(d, J.ga, J.p, J.mom, J.nn);
}

// ---------------------------------------------------------------- kernels

// Register budget of the mover-carrying kernels in waves per SIMD: the
// field-corner cache holds 48 values (96 VGPRs in FP64).
template <bool CACHE, typename TP>
struct MoverWaves {
    static constexpr int value = CACHE ? (sizeof(TP) == 8 ? 2 : 3) : 4;
};
// the sorted deposit: 80 sums (160 VGPRs in FP64)
template <typename TP>
struct DepositWaves {
    static constexpr int value = sizeof(TP) == 8 ? 2 : kDepWaves;
};

template <typename TP, typename TF, typename TA, bool CACHE, bool MOVE_ONLY, class GEO>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(MoverWaves<CACHE, TP>::value)))
k_fused_tiled(TileJob<TP, TF, TA> J, int chunk, int glog) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int b = blockIdx.x;
    const int t = tile_of_block(b, chunk, glog);
    if (t >= J.tg.ntiles) return;
    tile_body<TP, TF, TA, CACHE, MOVE_ONLY, GEO>(J, t, smem);
}

template <typename TP, typename TF, typename TA, class GEO>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(DepositWaves<TP>::value)))
k_deposit_tiled(TileJob<TP, TF, TA> J, int chunk, int glog) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int b = blockIdx.x;
    const int t = tile_of_block(b, chunk, glog);
    if (t >= J.tg.ntiles) return;
    deposit_body<TP, TF, TA, GEO>(J, t, smem);
}

// Variant 3 (FP32 particles): the deposit's 80 sums and, with CACHE, the
// mover's 48 field corners share the registers: two waves per SIMD with
// the corners, three without.
template <typename TP, typename TF, typename TA, bool CACHE, class GEOF, class GEOM>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(CACHE ? 2 : 3)))
k_lanecell_tiled(TileJob<TP, TF, TA> J, TileGeom tgm, int chunk, int glog) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int b = blockIdx.x;
    const int t = tile_of_block(b, chunk, glog);
    if (t >= J.tg.ntiles) return;
    lanecell_body<TP, TF, TA, CACHE, GEOF, GEOM>(J, tgm, t, smem);
}

// Persistent work-list kernels: workgroups take (job, tile) items from an
// atomic counter until the list is drained; every workgroup exits once the
// counter passes nitems.  The counter must be zero at launch.  KIND 0:
// variant 0/1 tile body (mover and LDS-atomic deposit), 1: mover only.
template <int KIND, typename TP, typename TF, typename TA, bool CACHE, class GEO>
__device__ __forceinline__ void worklist_loop(const TileJob<TP, TF, TA> *__restrict__ jobs,
                                              const uint2 *__restrict__ items, int nitems,
                                              unsigned *__restrict__ counter, unsigned char *smem, int *cur) {
    for (;;) {
        __syncthreads();  // the previous item's LDS use is over before `cur` changes
        if (threadIdx.x == 0) *cur = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(*cur);
        if (it >= nitems) break;
        const uint2 item = items[it];
        const TileJob<TP, TF, TA> J = jobs[item.x];
        tile_body<TP, TF, TA, CACHE, KIND == 1, GEO>(J, (int)item.y, smem);
    }
}

template <typename TP, typename TF, typename TA, bool CACHE, bool MOVE_ONLY, class GEO>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(MoverWaves<CACHE, TP>::value)))
k_worklist(const TileJob<TP, TF, TA> *__restrict__ jobs, const uint2 *__restrict__ items, int nitems,
           unsigned *__restrict__ counter) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int cur;
    worklist_loop<MOVE_ONLY ? 1 : 0, TP, TF, TA, CACHE, GEO>(jobs, items, nitems, counter, smem, &cur);
}

// The deposit list: one workgroup per (job, tile) item, the hardware
// dispatcher balancing them.  A persistent loop over the items kept its own
// state beside the deposit's 80 sums and spilled registers inside the bin
// drain.
template <typename TP, typename TF, typename TA, class GEO>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(DepositWaves<TP>::value)))
k_items_deposit(const TileJob<TP, TF, TA> *__restrict__ jobs, const uint2 *__restrict__ items) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint2 item = items[blockIdx.x];
    deposit_body<TP, TF, TA, GEO>(jobs[item.x], (int)item.y, smem);
}

// ------------------------------------------------------------- host side

static size_t fields_lds_bytes(const TileGeom &tg, int dtype) {
    return ((size_t)tg.rnp * 6 * (dtype == SPIC_F64 ? 8 : 4) + 15) & ~(size_t)15;
}

// Dense region slots of a tiling (the deposit's moment layout).
static int dense_rnp(const TileGeom &tg) { return tg.rx * tg.ry * tg.rz; }

size_t tiled_lds_bytes(const TileGeom &tg, int dtype, int acc_dtype, int variant, int block) {
    const int tb = dtype == SPIC_F64 ? 8 : 4, ab = acc_dtype == SPIC_F64 ? 8 : 4;
    if (variant == kVariantSplit) {
        // the mover launch (fields, at least the tile's halo) and the deposit launch
        return std::max(fields_lds_bytes(tg, dtype), deposit_lds_bytes(dense_rnp(tg), block, tb, ab));
    }
    if (variant == kVariantLaneCell) {
        if (dtype == SPIC_F64) return tiled_lds_bytes(tg, dtype, acc_dtype, kVariantSplit, block);
        // one launch: fields (at least the tile's halo) beside the deposit's LDS
        return fields_lds_bytes(tg, dtype) + deposit_lds_bytes(dense_rnp(tg), block, tb, ab);
    }
    return fields_lds_bytes(tg, dtype) + (((size_t)tg.rnp * 10 * ab + 15) & ~(size_t)15);
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

template <typename TP, typename TF, typename TA, bool CACHE, bool MOVE_ONLY, class GEO>
static void fused_launch(const TileJob<TP, TF, TA> &job, int chunk, int glog, size_t lds, int block,
                         hipStream_t s) {
    auto k = k_fused_tiled<TP, TF, TA, CACHE, MOVE_ONLY, GEO>;
    allow_lds(k, lds);
    hipLaunchKernelGGL(k, dim3(8 * chunk), dim3(block), lds, s, job, chunk, glog);
}

// The dense moment region of a tiling (the sorted deposit's LDS layout).
static TileGeom dense_geom(const TileGeom &tg) {
    TileGeom dg = tg;
    const RegionLayout lay = region_layout(tg.tx, tg.ty, tg.tz, tg.halo, tg.slow, tg.mid, tg.fast, 2);
    dg.sx = lay.sx; dg.sy = lay.sy; dg.sz = lay.sz; dg.rnp = lay.rnp;
    return dg;
}

// The mover launch of variant 2 stages its own field region, by default
// one cell of halo wider than the tile's (a particle that left the region
// gathers from global memory, three times); the layout search is memoised
// per thread (one tiling per run, as a rule).
static TileGeom mover_geom(const TileGeom &tg, int halo_opt, size_t lds_max, int dtype) {
    TileGeom mg = tg;
    int mh = halo_opt >= 0 ? halo_opt : tg.halo + 1;
    thread_local int key[5] = {-1, -1, -1, -1, -1};
    thread_local RegionLayout ml{0, 0, 0, 0};
    const int axes = tg.slow * 9 + tg.mid * 3 + tg.fast;
    if (key[0] != tg.tx || key[1] != tg.ty || key[2] != tg.tz || key[3] != mh || key[4] != axes) {
        ml = region_layout(tg.tx, tg.ty, tg.tz, mh, tg.slow, tg.mid, tg.fast, 1);
        key[0] = tg.tx; key[1] = tg.ty; key[2] = tg.tz; key[3] = mh; key[4] = axes;
    }
    // a region that does not fit the device's LDS keeps the tile's halo
    if ((size_t)ml.rnp * 6 * (dtype == SPIC_F64 ? 8 : 4) > lds_max) mh = tg.halo;
    if (mh != tg.halo) {
        mg.halo = mh;
        mg.rx = tg.tx + 2 * mh + 1; mg.ry = tg.ty + 2 * mh + 1; mg.rz = tg.tz + 2 * mh + 1;
        mg.sx = ml.sx; mg.sy = ml.sy; mg.sz = ml.sz; mg.rnp = ml.rnp;
    }
    return mg;
}

// Variant 2: the mover launch (variant 1's or 0's tile body without
// moments, LDS for the fields only), then the sorted deposit over the
// moved particles (LDS for the moments, counts and list only).
template <typename TP, typename TF, typename TA, class GEO>
static void split_launch(const TileJob<TP, TF, TA> &job, int chunk, const LaunchCfg &cfg, hipStream_t s) {
    const TileGeom &tg = job.tg;
    constexpr int dt = sizeof(TP) == 8 ? SPIC_F64 : SPIC_F32;
    TileJob<TP, TF, TA> mv = job;
    mv.tg = mover_geom(tg, cfg.mover_halo, cfg.lds_max, dt);
    const size_t fl = fields_lds_bytes(mv.tg, dt);
    const bool same = mv.tg.halo == tg.halo;
    const bool m2 = cfg.fixed_geo && geo_is<GeoMover2>(mv.tg);
    if (cfg.mover_cache) {
        if (same) fused_launch<TP, TF, TA, true, true, GEO>(mv, chunk, cfg.tile_group, fl, cfg.mover_block, s);
        else if (m2) fused_launch<TP, TF, TA, true, true, GeoMover2>(mv, chunk, cfg.tile_group, fl, cfg.mover_block, s);
        else fused_launch<TP, TF, TA, true, true, GeoRuntime>(mv, chunk, cfg.tile_group, fl, cfg.mover_block, s);
    } else {
        if (same) fused_launch<TP, TF, TA, false, true, GEO>(mv, chunk, cfg.tile_group, fl, cfg.mover_block, s);
        else if (m2) fused_launch<TP, TF, TA, false, true, GeoMover2>(mv, chunk, cfg.tile_group, fl, cfg.mover_block, s);
        else fused_launch<TP, TF, TA, false, true, GeoRuntime>(mv, chunk, cfg.tile_group, fl, cfg.mover_block, s);
    }
    if (!job.mom) return;
    TileJob<TP, TF, TA> dj = job;
    dj.tg = dense_geom(tg);
    const size_t dl = deposit_lds_bytes(dj.tg.rnp, cfg.tile_block, sizeof(TP), sizeof(TA));
    if (cfg.fixed_geo && geo_is<GeoDense>(dj.tg)) {
        auto k = k_deposit_tiled<TP, TF, TA, GeoDense>;
        allow_lds(k, dl);
        hipLaunchKernelGGL(k, dim3(8 * chunk), dim3(cfg.tile_block), dl, s, dj, chunk, cfg.tile_group);
    } else {
        auto k = k_deposit_tiled<TP, TF, TA, GeoRuntime>;
        allow_lds(k, dl);
        hipLaunchKernelGGL(k, dim3(8 * chunk), dim3(cfg.tile_block), dl, s, dj, chunk, cfg.tile_group);
    }
}

// Variant 3: one launch, the mover's field region (mover_geom, within the
// LDS the deposit leaves) beside the deposit's dense moment region.
template <typename TP, typename TF, typename TA>
static void lanecell_launch(const TileJob<TP, TF, TA> &job, int chunk, const LaunchCfg &cfg, hipStream_t s) {
    constexpr int dt = sizeof(TP) == 8 ? SPIC_F64 : SPIC_F32;
    const TileGeom tgm = dense_geom(job.tg);
    const size_t dl = deposit_lds_bytes(tgm.rnp, cfg.tile_block, sizeof(TP), sizeof(TA));
    TileJob<TP, TF, TA> mv = job;
    mv.tg = mover_geom(job.tg, cfg.mover_halo, cfg.lds_max > dl ? cfg.lds_max - dl : 0, dt);
    const size_t lds = fields_lds_bytes(mv.tg, dt) + dl;
    const bool fixed = cfg.fixed_geo && geo_is<GeoMover2>(mv.tg) && geo_is<GeoDense>(tgm);
    auto k = cfg.mover_cache ? (fixed ? k_lanecell_tiled<TP, TF, TA, true, GeoMover2, GeoDense>
                                      : k_lanecell_tiled<TP, TF, TA, true, GeoRuntime, GeoRuntime>)
                             : (fixed ? k_lanecell_tiled<TP, TF, TA, false, GeoMover2, GeoDense>
                                      : k_lanecell_tiled<TP, TF, TA, false, GeoRuntime, GeoRuntime>);
    allow_lds(k, lds);
    hipLaunchKernelGGL(k, dim3(8 * chunk), dim3(cfg.tile_block), lds, s, mv, tgm, chunk, cfg.tile_group);
}

template <typename TP, typename TF, typename TA, class GEO>
static void tiled_variant(const TileJob<TP, TF, TA> &job, int chunk, size_t lds, const LaunchCfg &cfg,
                          hipStream_t s) {
    switch (cfg.variant) {
        case kVariantLaneCell:
            // FP64 particles: 160 VGPRs of sums leave no room for the mover
            if constexpr (sizeof(TP) == 8) split_launch<TP, TF, TA, GEO>(job, chunk, cfg, s);
            else if (job.mom) lanecell_launch<TP, TF, TA>(job, chunk, cfg, s);
            else split_launch<TP, TF, TA, GEO>(job, chunk, cfg, s);  // no moments: the mover launch alone
            break;
        case kVariantSplit: split_launch<TP, TF, TA, GEO>(job, chunk, cfg, s); break;
        case 1:
            fused_launch<TP, TF, TA, true, false, GEO>(job, chunk, cfg.tile_group, lds, cfg.tile_block, s);
            break;
        default:
            fused_launch<TP, TF, TA, false, false, GEO>(job, chunk, cfg.tile_group, lds, cfg.tile_block, s);
    }
}

template <typename TP, typename TF, typename TA>
static void tiled_t(const spic_grid &g, const spic_params &prm, const spic_fields &f, const SpeciesWork &w,
                    const TileGeom &tg, const uint32_t *tile_off, const LaunchCfg &cfg, hipStream_t s) {
    const int chunk = tile_chunk(tg.ntiles, cfg.tile_group);
    const size_t lds = tiled_lds_bytes(tg, sizeof(TP) == 8 ? SPIC_F64 : SPIC_F32,
                                       sizeof(TA) == 8 ? SPIC_F64 : SPIC_F32, cfg.variant, cfg.tile_block);
    const auto job = make_tile_job<TP, TF, TA>(g, prm, f, w, tg, tile_off);
    if constexpr (sizeof(TP) == 8) {  // FP64 particles: the one-kernel variants in the compact layout
        if (cfg.fixed_geo && cfg.variant != kVariantSplit && geo_is<GeoCompact>(tg)) {
            if (cfg.variant == 1)
                fused_launch<TP, TF, TA, true, false, GeoCompact>(job, chunk, cfg.tile_group, lds, cfg.tile_block, s);
            else
                fused_launch<TP, TF, TA, false, false, GeoCompact>(job, chunk, cfg.tile_group, lds, cfg.tile_block,
                                                                   s);
            return;
        }
    }
    if (geo_is_default(tg) && cfg.fixed_geo) tiled_variant<TP, TF, TA, GeoDefault>(job, chunk, lds, cfg, s);
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

// ------------------------------------------------------------ work lists
//
// The batch engine drives the work-list kernels over tiles of many (run,
// species) jobs of one precision combination per launch: variants 0 and 1
// in one persistent launch, variants 2 and 3 as a persistent mover list and
// then a deposit list of one workgroup per item over the same items.

int job_combo(int dtype, int fdtype, int acc_dtype) {
    if (acc_dtype == SPIC_F32C) return -1;  // compensated FP32: the unsorted spic_mover path only
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

// The deposit list of the default tiling runs the kernel compiled for its
// dense layout.
template <class GEO>
struct DenseOf {
    using type = GeoRuntime;
};
template <>
struct DenseOf<GeoDefault> {
    using type = GeoDense;
};

static int cu_count() {
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    return ncu;
}

template <typename K>
static int resident_groups(K k, size_t lds, int block, int nitems, int max_groups) {
    allow_lds(k, lds);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, block, lds) != hipSuccess || per_cu < 1) per_cu = 1;
    int groups = per_cu * cu_count();
    if (groups > nitems) groups = nitems;
    if (max_groups > 0 && groups > max_groups) groups = max_groups;
    return groups < 1 ? 1 : groups;
}

// Workgroups of the persistent launches (the mover list at 512 threads, the
// one-launch variants at `block`): resident workgroups per CU times CUs,
// capped by the item count (and by max_groups when > 0); the deposit list
// has one workgroup (`block` threads) per item.  Also allows the LDS sizes;
// call before any stream capture.
template <typename TP, typename TF, typename TA, class GEO>
static WorklistGroups worklist_groups_t(int variant, const TileGeom &tg, int block, int nitems, int max_groups) {
    constexpr int dt = sizeof(TP) == 8 ? SPIC_F64 : SPIC_F32, at = sizeof(TA) == 8 ? SPIC_F64 : SPIC_F32;
    WorklistGroups r{};
    if (variant == kVariantLaneCell) variant = kVariantSplit;  // the lists run variant 3 as variant 2
    if (variant == kVariantSplit) {
        r.lds_mover = fields_lds_bytes(tg, dt);
        r.lds_deposit = deposit_lds_bytes(dense_rnp(tg), block, sizeof(TP), sizeof(TA));
        r.mover = resident_groups(k_worklist<TP, TF, TA, true, true, GEO>, r.lds_mover, 512, nitems, max_groups);
        allow_lds(k_items_deposit<TP, TF, TA, typename DenseOf<GEO>::type>, r.lds_deposit);
        r.deposit = nitems;  // one workgroup per item
    } else {
        r.lds_mover = tiled_lds_bytes(tg, dt, at, variant, block);
        if (variant == 1)
            r.mover = resident_groups(k_worklist<TP, TF, TA, true, false, GEO>, r.lds_mover, block, nitems, max_groups);
        else
            r.mover = resident_groups(k_worklist<TP, TF, TA, false, false, GEO>, r.lds_mover, block, nitems, max_groups);
    }
    return r;
}

WorklistGroups worklist_groups(int combo, bool fixed, int variant, const TileGeom &tg, int block, int nitems,
                               int max_groups) {
#define SPIC_WG(TP, TF, TA)                                                                           \
    return fixed ? worklist_groups_t<TP, TF, TA, GeoDefault>(variant, tg, block, nitems, max_groups) \
                 : worklist_groups_t<TP, TF, TA, GeoRuntime>(variant, tg, block, nitems, max_groups)
    switch (combo) {
        case 0: SPIC_WG(double, double, double);
        case 1: SPIC_WG(float, float, double);
        case 2: SPIC_WG(float, float, float);
        case 3: SPIC_WG(float, double, double);
        default: SPIC_WG(float, double, float);
    }
#undef SPIC_WG
}

template <typename TP, typename TF, typename TA, class GEO>
static hipError_t worklist_t(int variant, const void *jobs, const uint2 *items, int nitems, unsigned *counters,
                             const WorklistGroups &gr, int block, hipStream_t s) {
    using Job = TileJob<TP, TF, TA>;
    const Job *jb = (const Job *)jobs;
    if (variant == kVariantSplit || variant == kVariantLaneCell) {
        hipLaunchKernelGGL((k_worklist<TP, TF, TA, true, true, GEO>), dim3(gr.mover), dim3(512), gr.lds_mover, s,
                           jb, items, nitems, counters);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_items_deposit<TP, TF, TA, typename DenseOf<GEO>::type>), dim3(nitems), dim3(block),
                           gr.lds_deposit, s, jb, items);
    } else if (variant == 1) {
        hipLaunchKernelGGL((k_worklist<TP, TF, TA, true, false, GEO>), dim3(gr.mover), dim3(block), gr.lds_mover, s,
                           jb, items, nitems, counters);
    } else {
        hipLaunchKernelGGL((k_worklist<TP, TF, TA, false, false, GEO>), dim3(gr.mover), dim3(block), gr.lds_mover, s,
                           jb, items, nitems, counters);
    }
    return hipGetLastError();
}

hipError_t launch_worklist(int combo, bool fixed, int variant, const void *jobs, const uint2 *items, int nitems,
                           unsigned *counters, const WorklistGroups &gr, int block, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
#define SPIC_WL(TP, TF, TA)                                                                                 \
    return fixed ? worklist_t<TP, TF, TA, GeoDefault>(variant, jobs, items, nitems, counters, gr, block, s) \
                 : worklist_t<TP, TF, TA, GeoRuntime>(variant, jobs, items, nitems, counters, gr, block, s)
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
