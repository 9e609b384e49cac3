// spic_device.h -- device helpers shared by the HIP kernels of libspic.so:
// periodic wrap, cell location, linear weights (Eq. 3), gather (Eq. 4),
// the implicit mover (Eq. 1, Eq. 2, Eq. 5) and the moment deposit.
#pragma once

#include <hip/hip_runtime.h>

#include "spic_impl.h"

namespace spic {

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ float dfloor(float x) { return __builtin_floorf(x); }
__device__ __forceinline__ double dfloor(double x) { return __builtin_floor(x); }

// Periodic wrap into [0, L): a point already inside is returned as is;
// otherwise r = s - L floor(s/L), and a rounding that lands on L (or below
// 0) is the same point of the box as 0.
template <typename T>
__device__ __forceinline__ T pwrap(T s, T L, T invL) {
    T r = s;
    if (__builtin_expect(!(s >= T(0) && s < L), 0)) {
        r = s - L * dfloor(s * invL);
        r = (r >= L) ? T(0) : r;
        r = (r < T(0)) ? T(0) : r;
    }
    return r;
}

// 1 / d for d >= 1 (the denominator of Eq. 2): the hardware reciprocal in
// FP32 (1 ulp), a Newton-refined reciprocal in FP64.
__device__ __forceinline__ float recip_ge1(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double recip_ge1(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = __builtin_fma(-d, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-d, r, 1.0);
    return __builtin_fma(r, e, r);
}

// Left node index along one axis and the offset xi in [0,1] inside the cell;
// the two non-zero linear weights (Eq. 3) are 1 - xi and xi.
// s * invd, rounded on its own: never fused with a neighbouring add, so
// every kernel that locates a point (and the tiled kernel's same-cell
// shortcut) obtains the same in-cell offset bit for bit.
template <typename T>
__device__ __forceinline__ T cell_coord(T s, T invd) {
#pragma clang fp contract(off)
    return s * invd;
}

template <typename T>
__device__ __forceinline__ int plocate(T s, T L, T invL, T invd, int n, T &xi) {
    T t = cell_coord(pwrap(s, L, invL), invd);
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

// Eq. 4 from global memory, for a located cell.
template <typename T, typename TF>
__device__ __forceinline__ void gather_cell_global(const FieldPtrs<TF> &f, const Cell<T> &c, T out[6]) {
    T w[8];
    int nd[8];
    pweights(c.fx, c.fy, c.fz, w);
    pnodes(c, nd);
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < 8; ++k) acc += w[k] * (T)f.f[m][nd[k]];
        out[m] = acc;
    }
}

// Eq. 4 from global memory at a point.
template <typename T, typename TF>
__device__ __forceinline__ void gather_global(const GridT<T> &g, const FieldPtrs<TF> &f, T x, T y, T z, T out[6]) {
    gather_cell_global(f, pcell(g, x, y, z), out);
}

// One implicit step of one particle (Sec. II).  The mean velocity is
// iterated niter times; iteration k gathers E, B at the current estimate of
// the half-step position (x^n for the first), then
//   vt   = v^n + beta E                                   (Eq. 1)
//   b    = (beta/c) B
//   vbar = (vt + vt x b + (vt . b) b) / (1 + b . b)       (Eq. 2)
//   xbar = x^n + vbar dt/2
// and finally v^{n+1} = 2 vbar - v^n, x^{n+1} = x^n + vbar dt (Eq. 5),
// wrapped into the periodic box.  With a tolerance (mv.tol > 0; the count
// set by an error tolerance, Sec. II after Eq. 2) a particle stops after
// iteration k >= 2 once max_d |vbar^k - vbar^(k-1)| < tol, at niter at the
// latest (lanes leave the loop on their own).  `gather(x, y, z, F)`
// evaluates Eq. 4 at a point; the kernels differ only in where it reads the
// node fields.
template <typename T, typename Gather>
__device__ __forceinline__ void implicit_move(const GridT<T> &g, const MoveT<T> &mv, Gather &&gather, T &x, T &y,
                                              T &z, T &u, T &v, T &w) {
    const T x0 = x, y0 = y, z0 = z, u0 = u, v0 = v, w0 = w;
    T xb = x0, yb = y0, zb = z0;
    T ub = u0, vb = v0, wb = w0;
    const bool use_tol = mv.tol > T(0);
    for (int it = 0; it < mv.niter; ++it) {
        const T pu = ub, pv = vb, pw = wb;
        T F[6];
        gather(xb, yb, zb, F);
        const T ut = u0 + mv.beta * F[0];
        const T vt = v0 + mv.beta * F[1];
        const T wt = w0 + mv.beta * F[2];
        const T bx = mv.bc * F[3], by = mv.bc * F[4], bz = mv.bc * F[5];
        const T vdb = ut * bx + vt * by + wt * bz;
        const T inv = recip_ge1(T(1) + (bx * bx + by * by + bz * bz));
        ub = (ut + (vt * bz - wt * by) + vdb * bx) * inv;
        vb = (vt + (wt * bx - ut * bz) + vdb * by) * inv;
        wb = (wt + (ut * by - vt * bx) + vdb * bz) * inv;
        xb = x0 + ub * mv.hdt;
        yb = y0 + vb * mv.hdt;
        zb = z0 + wb * mv.hdt;
        if (use_tol && it >= 1) {
            const T d = __builtin_fmax(__builtin_fabs(ub - pu), __builtin_fmax(__builtin_fabs(vb - pv),
                                                                               __builtin_fabs(wb - pw)));
            if (d < mv.tol) break;
        }
    }
    u = T(2) * ub - u0;
    v = T(2) * vb - v0;
    w = T(2) * wb - w0;
    x = pwrap(x0 + ub * mv.dt, g.L[0], g.invL[0]);
    y = pwrap(y0 + vb * mv.dt, g.L[1], g.invL[1]);
    z = pwrap(z0 + wb * mv.dt, g.L[2], g.invL[2]);
}

template <typename T, typename TF>
__device__ __forceinline__ void move_global(const GridT<T> &g, const FieldPtrs<TF> &f, const MoveT<T> &mv, T &x,
                                            T &y, T &z, T &u, T &v, T &w) {
    implicit_move(g, mv, [&](T px, T py, T pz, T F[6]) { gather_global(g, f, px, py, pz, F); }, x, y, z, u, v, w);
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

}  // namespace spic
