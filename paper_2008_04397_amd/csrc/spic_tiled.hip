// spic_tiled.hip -- tiled fused mover + moment gathering for a species
// that has been sorted by cell (spic_sort.hip).
//
// One workgroup per tile of cells.  The workgroup stages the node fields of
// its region (the tile's cells, `halo` cells around them and the +1 corner
// nodes) in LDS, moves every particle of the tile's range (Eq. 1, Eq. 2,
// Eq. 5) gathering E and B from LDS (Eq. 3, Eq. 4), and deposits the ten
// moments of the moved particle (Sec. II moment equation; Sec. III-B:
// fused, from the new position) into an FP64 region accumulator in LDS.
// The region accumulator is then added to the global moments with
// coalesced global atomics (neighbouring tiles' regions overlap).
//
// Particles whose cell lies outside the region (they drifted farther than
// the halo since the last sort) take the global path for that gather or
// deposit, so the result does not depend on the particle order; the order
// only decides how much work stays in LDS.
//
// Rank-major order inside a tile puts consecutive particles -- the lanes of
// a wave -- in different cells, so the LDS atomics of one instruction hit
// different nodes.
//
// Tiles are mapped to workgroups so that the 8 XCDs each take a contiguous
// slab of tiles: workgroup b runs on XCD b % 8, and gets tile
// (b % 8) * chunk + b / 8, keeping a slab's fields and moments in that XCD's
// L2.
#include <hip/hip_runtime.h>

#include "spic_device.h"
#include "spic_impl.h"

namespace spic {

constexpr int MSTRIDE = 11;  // doubles per node in the LDS moment region (odd: spreads banks)

template <typename TP>
struct LdsFieldNode {
    TP v[6];
};

// Region-relative cell of a point; returns false when the cell's +1 corners
// leave the region.  `o*` is the region origin cell (periodic, in [0, n)).
template <typename T>
__device__ __forceinline__ bool region_cell(const GridT<T> &g, const TileGeom &tg, int ox, int oy, int oz,
                                            T x, T y, T z, int &rb, Cell<T> &c) {
    const int i = plocate(x, g.L[0], g.invL[0], g.invd[0], g.nx, c.fx);
    const int j = plocate(y, g.L[1], g.invL[1], g.invd[1], g.ny, c.fy);
    const int k = plocate(z, g.L[2], g.invL[2], g.invd[2], g.nz, c.fz);
    int di = i - ox, dj = j - oy, dk = k - oz;
    di += (di < 0) ? g.nx : 0;
    dj += (dj < 0) ? g.ny : 0;
    dk += (dk < 0) ? g.nz : 0;
    const int nyz = g.ny * g.nz;
    c.base = i * nyz + j * g.nz + k;
    c.ox = (i == g.nx - 1) ? -(g.nx - 1) * nyz : nyz;
    c.oy = (j == g.ny - 1) ? -(g.ny - 1) * g.nz : g.nz;
    c.oz = (k == g.nz - 1) ? -(g.nz - 1) : 1;
    rb = (di * tg.ry + dj) * tg.rz + dk;
    return di < tg.rx - 1 && dj < tg.ry - 1 && dk < tg.rz - 1;
}

template <typename TP>
__device__ __forceinline__ void gather_lds(const LdsFieldNode<TP> *__restrict__ fl, const TileGeom &tg, int rb,
                                           const Cell<TP> &c, TP out[6]) {
    TP w[8];
    pweights(c.fx, c.fy, c.fz, w);
    const int sx = tg.ry * tg.rz, sy = tg.rz;
    const int nd[8] = {rb, rb + sx, rb + sy, rb + sx + sy, rb + 1, rb + sx + 1, rb + sy + 1, rb + sx + sy + 1};
#pragma unroll
    for (int m = 0; m < 6; ++m) out[m] = TP(0);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const LdsFieldNode<TP> fn = fl[nd[k]];
#pragma unroll
        for (int m = 0; m < 6; ++m) out[m] += w[k] * fn.v[m];
    }
}

template <typename TP, typename TF, typename TA>
__global__ void __launch_bounds__(512)
k_fused_tiled(GridT<TP> g, GridT<TA> ga, FieldPtrs<TF> f, MoveT<TP> mv, PartPtrs<TP> p, TA *__restrict__ mom,
              int nn, const uint32_t *__restrict__ tile_off, TileGeom tg, int chunk) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int b = blockIdx.x;
    const int t = (b & 7) * chunk + (b >> 3);
    if (t >= tg.ntiles) return;
    const int RN = tg.rx * tg.ry * tg.rz;
    LdsFieldNode<TP> *fl = (LdsFieldNode<TP> *)smem;
    TA *ml = (TA *)(smem + ((RN * sizeof(LdsFieldNode<TP>) + 15) & ~(size_t)15));

    const int tzi = t % tg.ntz, tyi = (t / tg.ntz) % tg.nty, txi = t / (tg.ntz * tg.nty);
    int ox = (txi * tg.tx - tg.halo) % g.nx; ox += ox < 0 ? g.nx : 0;
    int oy = (tyi * tg.ty - tg.halo) % g.ny; oy += oy < 0 ? g.ny : 0;
    int oz = (tzi * tg.tz - tg.halo) % g.nz; oz += oz < 0 ? g.nz : 0;
    const int rzy = tg.ry * tg.rz;

    // stage the region's node fields, zero the region's moments
    for (int r = threadIdx.x; r < RN; r += blockDim.x) {
        const int ri = r / rzy, rj = (r / tg.rz) % tg.ry, rk = r % tg.rz;
        const int gi = (ox + ri) % g.nx, gj = (oy + rj) % g.ny, gk = (oz + rk) % g.nz;
        const int gn = (gi * g.ny + gj) * g.nz + gk;
        LdsFieldNode<TP> fn;
#pragma unroll
        for (int m = 0; m < 6; ++m) fn.v[m] = (TP)f.f[m][gn];
        fl[r] = fn;
    }
    for (int q = threadIdx.x; q < RN * MSTRIDE; q += blockDim.x) ml[q] = TA(0);
    __syncthreads();

    const uint32_t beg = tile_off[t], end = tile_off[t + 1];
    for (uint32_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
        TP xn = p.x[i], yn = p.y[i], zn = p.z[i];
        TP un = p.u[i], vn = p.v[i], wn = p.w[i];
        implicit_move(
            g, mv,
            [&](TP px, TP py, TP pz, TP F[6]) {
                int rb;
                Cell<TP> c;
                if (region_cell(g, tg, ox, oy, oz, px, py, pz, rb, c)) {
                    gather_lds(fl, tg, rb, c, F);
                } else {
                    gather_cell_global(f, c, F);
                }
            },
            xn, yn, zn, un, vn, wn);
        p.x[i] = xn; p.y[i] = yn; p.z[i] = zn;
        p.u[i] = un; p.v[i] = vn; p.w[i] = wn;
        if (!mom) continue;

        // deposit of the new state in the accumulation precision
        const TA qa = (TA)p.q[i];
        const TA ua = (TA)un, va = (TA)vn, wa = (TA)wn;
        int rb;
        Cell<TA> c;
        const bool in = region_cell(ga, tg, ox, oy, oz, (TA)xn, (TA)yn, (TA)zn, rb, c);
        TA wt8[8];
        pweights(c.fx, c.fy, c.fz, wt8);
        const TA val[10] = {TA(1), ua, va, wa, ua * ua, ua * va, ua * wa, va * va, va * wa, wa * wa};
        if (in) {
            const int sx = tg.ry * tg.rz, sy = tg.rz;
            const int nd[8] = {rb, rb + sx, rb + sy, rb + sx + sy, rb + 1, rb + sx + 1, rb + sy + 1,
                               rb + sx + sy + 1};
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const TA qw = qa * wt8[k];
                TA *dst = ml + nd[k] * MSTRIDE;
#pragma unroll
                for (int m = 0; m < 10; ++m) atomicAdd(dst + m, qw * val[m]);
            }
        } else {
            int nd[8];
            pnodes(c, nd);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const TA qw = qa * wt8[k];
#pragma unroll
                for (int m = 0; m < 10; ++m) atomicAdd(mom + (size_t)m * nn + nd[k], qw * val[m]);
            }
        }
    }
    if (!mom) return;
    __syncthreads();
    // flush: region accumulator -> global moments (skip exact zeros: halo
    // nodes no particle reached)
    for (int q = threadIdx.x; q < RN * 10; q += blockDim.x) {
        const int m = q / RN, r = q - m * RN;
        const TA val = ml[r * MSTRIDE + m];
        if (val != TA(0)) {
            const int ri = r / rzy, rj = (r / tg.rz) % tg.ry, rk = r % tg.rz;
            const int gi = (ox + ri) % g.nx, gj = (oy + rj) % g.ny, gk = (oz + rk) % g.nz;
            atomicAdd(mom + (size_t)m * nn + (gi * g.ny + gj) * g.nz + gk, val);
        }
    }
}

size_t tiled_lds_bytes(const TileGeom &tg, int dtype, int acc_dtype) {
    const size_t RN = (size_t)tg.rx * tg.ry * tg.rz;
    const size_t fsz = RN * 6 * (dtype == SPIC_F64 ? 8 : 4);
    const size_t msz = RN * MSTRIDE * (acc_dtype == SPIC_F64 ? 8 : 4);
    return ((fsz + 15) & ~(size_t)15) + msz;
}

template <typename TP, typename TF, typename TA>
static void tiled_t(const spic_grid &g, const spic_params &prm, const spic_fields &f, const SpeciesWork &w,
                    const TileGeom &tg, const uint32_t *tile_off, const LaunchCfg &cfg, hipStream_t s) {
    const int nn = g.nx * g.ny * g.nz;
    const int chunk = (tg.ntiles + 7) / 8;
    const size_t lds = tiled_lds_bytes(tg, sizeof(TP) == 8 ? SPIC_F64 : SPIC_F32,
                                       sizeof(TA) == 8 ? SPIC_F64 : SPIC_F32);
    hipLaunchKernelGGL((k_fused_tiled<TP, TF, TA>), dim3(8 * chunk), dim3(cfg.tile_block), lds, s,
                       make_grid_t<TP>(g), make_grid_t<TA>(g), field_ptrs<TF>(f), make_move<TP>(prm, w.qom),
                       part_ptrs<TP>(w), (TA *)w.mom, nn, tile_off, tg, chunk);
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
