// spic_sort.hip -- counting sort of particles by cell (Sec. III-A and
// Sec. VI: periodic ordering of particles by their cell restores the
// locality of the field and moment accesses).
//
// Key order.  Cells are grouped in tiles of TX x TY x TZ cells (at most 64
// cells), tiles in flat (tx, ty, tz) order.  Within a tile the particles are
// laid out *rank-major*: first the rank-0 particle of every non-empty cell
// (cells in local order), then the rank-1 particles, and so on.  Consecutive
// particles therefore sit in different cells, so one wave of the tiled
// fused kernel deposits into 64 different cells' nodes and its LDS atomics
// do not collide; the per-tile particle ranges are what the tiled kernel
// distributes over workgroups.
//
// Passes (all on the caller's stream):
//   1 key:     cell key of every particle; rank within its cell from a
//              wave-aggregated atomic histogram, or, for particles still in
//              an earlier sort's layout, from per-tile LDS counters in order
//   2 scan:    exclusive prefix of the per-key counts (three kernels)
//   3 tables:  per tile and rank, the start of the rank block and the mask
//              of cells holding a particle of that rank
//   4 slots:   rank-major (or cell-major) slot of every particle (an index
//              scatter), then a
//              gather of the particles into slot order in scratch; copy
//              back (or the fused kernel reads the scratch directly)
#include <hip/hip_runtime.h>

#include <algorithm>

#include "spic_device.h"
#include "spic_impl.h"

namespace spic {

// ----------------------------------------------------------------- keys

template <typename T>
__device__ __forceinline__ int sort_locate(T s, T L, T invL, T invd, int n) {
    T xi;
    return plocate(s, L, invL, invd, n, xi);
}

// Tile (flat in x, y, z order) and local cell (slow, mid, fast order) of a
// cell, as one key.
__device__ __forceinline__ uint32_t tile_key(const TileGeom &tg, int i, int j, int k) {
    const int tx = i / tg.tx, ty = j / tg.ty, tz = k / tg.tz;
    const int l[3] = {i - tx * tg.tx, j - ty * tg.ty, k - tz * tg.tz};
    const int t[3] = {tg.tx, tg.ty, tg.tz};
    const uint32_t tile = (uint32_t)((tx * tg.nty + ty) * tg.ntz + tz);
    return tile * (uint32_t)tg.cells + (uint32_t)((l[tg.slow] * t[tg.mid] + l[tg.mid]) * t[tg.fast] + l[tg.fast]);
}

// Key of every particle and its rank inside its key.  Lanes holding the
// same key as their left neighbour form a segment; the segment head adds the
// segment length to the global count and the other lanes take consecutive
// ranks.  On (nearly) sorted input this turns ~64 same-address atomics into
// one or two per wave.
template <typename T>
__global__ void __launch_bounds__(256)
k_sort_keys(GridT<T> g, TileGeom tg, const T *__restrict__ x, const T *__restrict__ y,
            const T *__restrict__ z, int64_t n, uint32_t *__restrict__ counts, uint2 *__restrict__ keyrank) {
    const int lane = threadIdx.x & 63;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = base + threadIdx.x;
        const bool valid = p < n;
        uint32_t key = 0xFFFFFFFFu;
        if (valid) {
            const int i = sort_locate(x[p], g.L[0], g.invL[0], g.invd[0], g.nx);
            const int j = sort_locate(y[p], g.L[1], g.invL[1], g.invd[1], g.ny);
            const int k = sort_locate(z[p], g.L[2], g.invL[2], g.invd[2], g.nz);
            key = tile_key(tg, i, j, k);
        }
        const uint32_t prev = __shfl_up(key, 1, 64);
        const bool head = valid && (lane == 0 || prev != key);
        const uint64_t heads = __ballot(head);
        const uint64_t validm = __ballot(valid);
        // start of my segment: highest head at or below my lane
        const uint64_t below_incl = heads & ((lane == 63) ? ~0ull : ((2ull << lane) - 1));
        const int start = below_incl ? 63 - __clzll(below_incl) : 0;
        // end of my segment: next head above me, or end of valid lanes
        const uint64_t above = (lane == 63) ? 0ull : (heads & ~((2ull << lane) - 1));
        const int vend = 64 - __clzll(validm);  // one past last valid lane
        const int end = above ? __ffsll((long long)above) - 1 : vend;
        uint32_t old = 0;
        if (head) old = atomicAdd(counts + key, (uint32_t)(end - start));
        const uint32_t seg_old = __shfl(old, start, 64);
        if (valid) keyrank[p] = make_uint2(key, seg_old + (uint32_t)(lane - start));
    }
}

// Keys and ranks of particles that are still laid out by an earlier sort
// with the same tiles (prev_off = that sort's per-tile ranges, a partition
// of [0, n)).  One workgroup walks one tile's range in order.  Particles
// whose cell is in that tile are ranked with LDS counters (own[] at the
// end), so a cell's ranks follow the earlier order up to the waves in
// flight; particles that arrived from another tile's range are ranked on a
// global counter imm[] and flagged, their final rank being own + that rank
// (k_sort_slots).  The gather below then reads long runs for the particles
// that stayed.  Correct for any partition of [0, n).
constexpr uint32_t kImmigrant = 0x80000000u;

constexpr int kKeysU = 4;

template <typename T>
__global__ void __launch_bounds__(256)
k_sort_keys_tiled(GridT<T> g, TileGeom tg, const T *__restrict__ x, const T *__restrict__ y,
                  const T *__restrict__ z, const uint32_t *__restrict__ prev_off, uint32_t *__restrict__ own,
                  uint32_t *__restrict__ imm, uint2 *__restrict__ keyrank) {
    __shared__ uint32_t lc[64];
    for (int t = blockIdx.x; t < tg.ntiles; t += gridDim.x) {
        if (threadIdx.x < 64) lc[threadIdx.x] = 0u;
        __syncthreads();
        const uint32_t b = prev_off[t], e = prev_off[t + 1];
        const uint32_t key0 = (uint32_t)t * (uint32_t)tg.cells;
        // kKeysU particles per thread: their positions are loaded together
        // (an index past the range is clamped and its result dropped)
        for (uint32_t p0 = b + threadIdx.x; p0 < e; p0 += kKeysU * blockDim.x) {
            T px[kKeysU], py[kKeysU], pz[kKeysU];
#pragma unroll
            for (int u = 0; u < kKeysU; ++u) {
                const uint32_t p = min(p0 + u * blockDim.x, e - 1);
                px[u] = x[p]; py[u] = y[p]; pz[u] = z[p];
            }
#pragma unroll
            for (int u = 0; u < kKeysU; ++u) {
                const uint32_t p = p0 + u * blockDim.x;
                if (p < e) {
                    const int i = sort_locate(px[u], g.L[0], g.invL[0], g.invd[0], g.nx);
                    const int j = sort_locate(py[u], g.L[1], g.invL[1], g.invd[1], g.ny);
                    const int k = sort_locate(pz[u], g.L[2], g.invL[2], g.invd[2], g.nz);
                    const uint32_t key = tile_key(tg, i, j, k);
                    uint32_t r;
                    if (key - key0 < (uint32_t)tg.cells) r = atomicAdd(&lc[key - key0], 1u);
                    else r = atomicAdd(imm + key, 1u) | kImmigrant;
                    keyrank[p] = make_uint2(key, r);
                }
            }
        }
        __syncthreads();
        if (threadIdx.x < tg.cells) own[key0 + threadIdx.x] = lc[threadIdx.x];
        __syncthreads();
    }
}

// counts = own + imm per key (imm becomes the total; own is kept for the
// immigrants' final ranks).
__global__ void k_sort_counts(const uint32_t *__restrict__ own, uint32_t *__restrict__ imm, int64_t nkeys) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nkeys; k += (int64_t)gridDim.x * blockDim.x)
        imm[k] += own[k];
}

// ----------------------------------------------------------------- scan

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_CHUNK = SCAN_BLOCK * SCAN_ITEMS;  // keys per block

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// Exclusive scan of one value per thread across the block; returns the
// exclusive prefix and writes the block total to *total.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *sh, uint32_t *total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint32_t incl = wave_incl_scan(v);
    if (lane == 63) sh[wv] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int w = 0; w < nw; ++w) {
            const uint32_t t = sh[w];
            sh[w] = acc;
            acc += t;
        }
        sh[nw] = acc;
    }
    __syncthreads();
    const uint32_t r = sh[wv] + incl - v;
    *total = sh[nw];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(SCAN_BLOCK)
k_scan_partials(const uint32_t *__restrict__ counts, int64_t nkeys, uint32_t *__restrict__ partial) {
    __shared__ uint32_t sh[SCAN_BLOCK / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i)
        if (base + i < nkeys) s += counts[base + i];
    uint32_t total;
    (void)block_excl_scan(s, sh, &total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// One block scans the per-chunk totals in place (exclusive).
__global__ void __launch_bounds__(1024) k_scan_top(uint32_t *__restrict__ partial, int nparts) {
    __shared__ uint32_t sh[1024 / 64 + 1];
    uint32_t carry = 0;
    for (int b = 0; b < nparts; b += blockDim.x) {
        const int i = b + threadIdx.x;
        const uint32_t v = i < nparts ? partial[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_excl_scan(v, sh, &total);
        if (i < nparts) partial[i] = carry + ex;
        carry += total;
    }
}

__global__ void __launch_bounds__(SCAN_BLOCK)
k_scan_apply(const uint32_t *__restrict__ counts, int64_t nkeys, const uint32_t *__restrict__ partial,
             uint32_t *__restrict__ offsets) {
    __shared__ uint32_t sh[SCAN_BLOCK / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        v[i] = (base + i < nkeys) ? counts[base + i] : 0u;
        s += v[i];
    }
    uint32_t total;
    uint32_t run = partial[blockIdx.x] + block_excl_scan(s, sh, &total);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (base + i < nkeys) offsets[base + i] = run;
        run += v[i];
    }
    // the thread covering the last key writes the total at offsets[nkeys]
    if (base < nkeys && base + SCAN_ITEMS >= nkeys) offsets[nkeys] = run;
}

// --------------------------------------------------------------- scatter

// Rank tables.  Inside tile t the particle of local cell l with rank r goes
// to  tile_start + base_t[r] + #{l' < l : count_l' > r},  where base_t[r] is
// the number of the tile's particles of rank < r.  One wave per tile (lane
// l = local cell l) writes, for each rank r < max count, the entry
// {base_t[r], mask of cells with count > r} at tab[tab_off[t] + r].

// Max cell count of every tile.
__global__ void __launch_bounds__(64)
k_tile_maxc(const uint32_t *__restrict__ offsets, TileGeom tg, uint32_t *__restrict__ maxc) {
    const int t = blockIdx.x;
    const int lane = threadIdx.x;
    const uint32_t key0 = (uint32_t)t * (uint32_t)tg.cells;
    uint32_t c = 0;
    if (lane < tg.cells) c = offsets[key0 + lane + 1] - offsets[key0 + lane];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t o = __shfl_xor(c, d, 64);
        c = o > c ? o : c;
    }
    if (lane == 0) maxc[t] = c;
}

__global__ void __launch_bounds__(64)
k_tile_table(const uint32_t *__restrict__ offsets, TileGeom tg, const uint32_t *__restrict__ tab_off,
             uint4 *__restrict__ tab) {
    const int t = blockIdx.x;
    const int lane = threadIdx.x;
    const uint32_t key0 = (uint32_t)t * (uint32_t)tg.cells;
    uint32_t cnt = 0;
    if (lane < tg.cells) cnt = offsets[key0 + lane + 1] - offsets[key0 + lane];
    const uint32_t t0 = tab_off[t], nr = tab_off[t + 1] - t0;
    uint32_t base = 0;
    for (uint32_t r0 = 0; r0 < nr; r0 += 64) {
        // lane j computes the entry of rank r0 + j from a wave-wide ballot per rank
        uint32_t my_base = 0;
        uint64_t my_mask = 0;
        for (int j = 0; j < 64 && r0 + j < nr; ++j) {
            const uint64_t m = __ballot(cnt > r0 + j);
            if (lane == j) { my_base = base; my_mask = m; }
            base += (uint32_t)__popcll(m);
        }
        if (r0 + lane < nr) tab[t0 + r0 + lane] = make_uint4(my_base, (uint32_t)my_mask, (uint32_t)(my_mask >> 32), 0u);
    }
}

// Rank-major slot of every particle: srcidx[slot] = particle.  Only this
// 4-byte index is written scattered; a rank change by one moves a particle
// by a whole rank block, so after a few steps nearly every lane of a wave
// writes a different cache line.
__global__ void __launch_bounds__(256)
k_sort_slots(int64_t n, const uint2 *__restrict__ keyrank, const uint32_t *__restrict__ offsets,
             const uint32_t *__restrict__ tab_off, const uint4 *__restrict__ tab, int cells,
             const uint32_t *__restrict__ own, uint32_t *__restrict__ srcidx) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const uint2 kr = keyrank[p];
        const uint32_t t = kr.x / (uint32_t)cells, l = kr.x - t * (uint32_t)cells;
        // ranked in the tiled key pass as an immigrant: after the cell's own particles
        const uint32_t rank = (own && (kr.y & kImmigrant)) ? own[kr.x] + (kr.y & ~kImmigrant) : kr.y;
        const uint4 e = tab[tab_off[t] + rank];
        const uint64_t m = ((uint64_t)e.z << 32) | e.y;
        const uint64_t below = (l == 0) ? 0ull : (m & ((1ull << l) - 1));
        const uint32_t d = offsets[t * (uint32_t)cells] + e.x + (uint32_t)__popcll(below);
        srcidx[d] = (uint32_t)p;
    }
}

// Full-row layout, per tile (one wave; lane = cell): R = n_t / C full rows;
// cell c leaves h_c = max(0, R - n_c) holes in them and has
// e_c = max(0, n_c - R) particles of rank >= R.  hx[key] = (exclusive
// prefix of h, exclusive prefix of e) over the tile's cells, rh[t] = (R,
// total holes).
__global__ void __launch_bounds__(64)
k_tile_rows(const uint32_t *__restrict__ offsets, TileGeom tg, uint2 *__restrict__ hx, uint2 *__restrict__ rh) {
    const int t = blockIdx.x;
    const int lane = threadIdx.x;
    const uint32_t C = (uint32_t)tg.cells, key0 = (uint32_t)t * C;
    const uint32_t nt = offsets[key0 + C] - offsets[key0];
    const uint32_t R = nt / C;
    uint32_t h = 0, e = 0;
    if ((uint32_t)lane < C) {
        const uint32_t nc = offsets[key0 + lane + 1] - offsets[key0 + lane];
        h = nc < R ? R - nc : 0u;
        e = nc > R ? nc - R : 0u;
    }
    // inclusive wave scans
    uint32_t H = h, E = e;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t hu = __shfl_up(H, d, 64), eu = __shfl_up(E, d, 64);
        if (lane >= d) {
            H += hu;
            E += eu;
        }
    }
    if ((uint32_t)lane < C) hx[key0 + lane] = make_uint2(H - h, E - e);
    if (lane == 63) rh[t] = make_uint2(R, H);
}

// Full-row slot of every particle (see TileGeom::rows): rank r < R of cell c
// at row r, column c; the j-th particle of rank >= R (cells in order) in the
// j-th hole (columns in order, rows upward), past the holes in the last
// partial row.
__global__ void __launch_bounds__(256)
k_sort_slots_rows(int64_t n, const uint2 *__restrict__ keyrank, const uint32_t *__restrict__ offsets,
                  const uint2 *__restrict__ hx, const uint2 *__restrict__ rh, int cells,
                  const uint32_t *__restrict__ own, uint32_t *__restrict__ srcidx) {
    const uint32_t C = (uint32_t)cells;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const uint2 kr = keyrank[p];
        const uint32_t t = kr.x / C, c = kr.x - t * C, key0 = t * C;
        const uint32_t rank = (own && (kr.y & kImmigrant)) ? own[kr.x] + (kr.y & ~kImmigrant) : kr.y;
        const uint32_t base = offsets[key0];
        const uint2 RH = rh[t];
        uint32_t d;
        if (rank < RH.x) {
            d = base + C * rank + c;
        } else {
            const uint32_t j = hx[kr.x].y + (rank - RH.x);
            if (j < RH.y) {
                // the column whose holes hold j: the last c2 with H(c2) <= j
                uint32_t lo = 0, hi = C - 1;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi + 1) >> 1;
                    if (hx[key0 + mid].x <= j) lo = mid;
                    else hi = mid - 1;
                }
                const uint32_t n2 = offsets[key0 + lo + 1] - offsets[key0 + lo];
                d = base + C * (n2 + (j - hx[key0 + lo].x)) + lo;
            } else {
                d = base + C * RH.x + (j - RH.y);
            }
        }
        srcidx[d] = (uint32_t)p;
    }
}

// Gather the particles into slot order: writes are coalesced; the reads
// are scattered over the tile's earlier range and its neighbours' (L2
// resident) wherever particles changed cell since the last sort.
template <typename T>
__global__ void __launch_bounds__(256)
k_sort_gather(PartPtrs<T> src, PartPtrs<T> dst, int64_t n, const uint32_t *__restrict__ srcidx) {
    for (int64_t d = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; d < n; d += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t p = srcidx[d];
        if (p >= (uint64_t)n) continue;  // never taken: the slots are a permutation of [0, n)
        dst.x[d] = src.x[p]; dst.y[d] = src.y[p]; dst.z[d] = src.z[p];
        dst.u[d] = src.u[p]; dst.v[d] = src.v[p]; dst.w[d] = src.w[p];
        dst.q[d] = src.q[p];
        if (src.id) dst.id[d] = src.id[p];
    }
}

// The same gather for a re-sort with the same tiling, one workgroup per new
// tile: most of a tile's particles were in the same tile at the previous
// sort, so each array's old tile range is staged in LDS with coalesced
// reads, the new order is gathered from LDS and written coalesced; a
// particle that came from another tile (or lies past the staging capacity)
// is read from global memory.  old_off holds the previous sort's tile
// ranges, offsets the new per-cell offsets.
constexpr int kGatherLdsBytes = 32768;

template <typename T, typename V>
__device__ __forceinline__ void gather_tile_array(const V *__restrict__ sa, V *__restrict__ da, V *stage, uint32_t ob,
                                                  uint32_t ocap, uint32_t nb, uint32_t ne, int64_t n,
                                                  const uint32_t *__restrict__ srcidx) {
    // batches of 8 elements per thread keep 8 loads in flight
    constexpr int U = 8;
    const uint32_t B = blockDim.x;
    for (uint32_t j0 = threadIdx.x; j0 < ocap; j0 += U * B) {
        V v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t j = j0 + u * B;
            if (j < ocap) v[u] = sa[ob + j];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t j = j0 + u * B;
            if (j < ocap) stage[j] = v[u];
        }
    }
    __syncthreads();
    for (uint32_t d0 = nb + threadIdx.x; d0 < ne; d0 += U * B) {
        uint32_t p[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t d = d0 + u * B;
            p[u] = d < ne ? srcidx[d] : 0u;
        }
        V v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t d = d0 + u * B;
            const uint32_t r = p[u] - ob;  // wraps past ocap when p < ob
            if (d < ne) {
                if (r < ocap) v[u] = stage[r];
                else if (p[u] < (uint64_t)n) v[u] = sa[p[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t d = d0 + u * B;
            const uint32_t r = p[u] - ob;
            if (d < ne && (r < ocap || p[u] < (uint64_t)n)) da[d] = v[u];
        }
    }
    __syncthreads();
}

// Pipelined re-sort gather of one tile whose new and old ranges hold at
// most kPipeU * blockDim slots: the source indices are loaded once; while
// array a is scattered from the stage, array a + 1's old range is already
// loading into registers; particles that came from another tile are moved
// in one last pass over all seven arrays (their loads in flight together).
constexpr int kPipeU = 20;
// FP64 particles take the per-array form (the pipelined one needs 147
// VGPRs for them: 3 waves per SIMD)
constexpr bool kPipeFP64 = false;

template <typename T>
__device__ __forceinline__ void gather_tile_piped(const T *const (&sa)[7], T *const (&da)[7], T *stage, uint32_t ob,
                                                  uint32_t span, uint32_t nb, uint32_t ne, int64_t n,
                                                  const uint32_t *__restrict__ srcidx) {
    constexpr int U = kPipeU;
    const uint32_t B = blockDim.x;
    uint32_t p[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t d = nb + threadIdx.x + u * B;
        p[u] = d < ne ? srcidx[d] : 0u;
    }
    T nv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t j = threadIdx.x + u * B;
        if (j < span) nv[u] = sa[0][ob + j];
    }
#pragma unroll
    for (int a = 0; a < 7; ++a) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t j = threadIdx.x + u * B;
            if (j < span) stage[j] = nv[u];
        }
        __syncthreads();
        if (a + 1 < 7)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t j = threadIdx.x + u * B;
                if (j < span) nv[u] = sa[a + 1][ob + j];
            }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t d = nb + threadIdx.x + u * B;
            const uint32_t r = p[u] - ob;  // wraps past span when p < ob
            if (d < ne && r < span) da[a][d] = stage[r];
        }
        __syncthreads();  // the stage is rewritten by the next array
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t d = nb + threadIdx.x + u * B;
        const uint32_t r = p[u] - ob;
        if (d < ne && r >= span && p[u] < (uint64_t)n) {
            T v[7];
#pragma unroll
            for (int a = 0; a < 7; ++a) v[a] = sa[a][p[u]];
#pragma unroll
            for (int a = 0; a < 7; ++a) da[a][d] = v[a];
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_sort_gather_tiled(PartPtrs<T> src, PartPtrs<T> dst, int64_t n, const uint32_t *__restrict__ srcidx,
                    const uint32_t *__restrict__ old_off, const uint32_t *__restrict__ offsets, int cells,
                    int ntiles, int chunk, int glog) {
    __shared__ __align__(16) unsigned char lds[kGatherLdsBytes];
    // tiles dealt to the XCDs in groups, as the tiled kernels do: the
    // particles that changed tile are read from neighbouring tiles' ranges,
    // which then sit in the same L2 more often
    const int t = tile_of_block(blockIdx.x, chunk, glog);
    if (t >= ntiles) return;
    const uint32_t nb = offsets[(uint32_t)t * (uint32_t)cells], ne = offsets[(uint32_t)(t + 1) * (uint32_t)cells];
    // clamped to [0, n] so that stale ranges cannot send a read out of bounds
    const uint32_t nn32 = (uint32_t)n;
    const uint32_t ob = min(old_off[t], nn32), oe = min(old_off[t + 1], nn32);
    const uint32_t span = oe > ob ? oe - ob : 0u;
    const uint32_t capT = kGatherLdsBytes / sizeof(T), cap8 = kGatherLdsBytes / 8;
    const uint32_t oc = span < capT ? span : capT;
    T *st = (T *)lds;
    const T *const sa[7] = {src.x, src.y, src.z, src.u, src.v, src.w, src.q};
    T *const da[7] = {dst.x, dst.y, dst.z, dst.u, dst.v, dst.w, dst.q};
    const uint32_t piped = (uint32_t)kPipeU * blockDim.x;
    if ((kPipeFP64 || sizeof(T) == 4) && ne - nb <= piped && span <= piped && span <= capT) {
        gather_tile_piped<T>(sa, da, st, ob, span, nb, ne, n, srcidx);
    } else {
#pragma unroll
        for (int a = 0; a < 7; ++a) gather_tile_array<T, T>(sa[a], da[a], st, ob, oc, nb, ne, n, srcidx);
    }
    if (src.id)
        gather_tile_array<T, int64_t>(src.id, dst.id, (int64_t *)lds, ob, span < cap8 ? span : cap8, nb, ne, n,
                                      srcidx);
}

template <typename T>
__global__ void __launch_bounds__(256) k_copy_parts(PartPtrs<T> src, PartPtrs<T> dst, int64_t n) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        dst.x[p] = src.x[p]; dst.y[p] = src.y[p]; dst.z[p] = src.z[p];
        dst.u[p] = src.u[p]; dst.v[p] = src.v[p]; dst.w[p] = src.w[p];
        dst.q[p] = src.q[p];
        if (src.id) dst.id[p] = src.id[p];
    }
}

// Per-tile particle ranges: tile_off[t] = offsets[t * cells].
__global__ void k_tile_offsets(const uint32_t *__restrict__ offsets, TileGeom tg, int ntiles,
                               uint32_t *__restrict__ tile_off) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t <= ntiles) tile_off[t] = offsets[(uint32_t)t * (uint32_t)tg.cells];
}

// ------------------------------------------------------------------ host

TileGeom make_tile_geom(const spic_grid &g, int tx, int ty, int tz, int halo, int layout, bool rows) {
    TileGeom t;
    t.tx = tx; t.ty = ty; t.tz = tz;
    t.cells = tx * ty * tz;
    t.ntx = (g.nx + tx - 1) / tx;
    t.nty = (g.ny + ty - 1) / ty;
    t.ntz = (g.nz + tz - 1) / tz;
    t.ntiles = t.ntx * t.nty * t.ntz;
    t.halo = halo;
    t.rx = tx + 2 * halo + 1;
    t.ry = ty + 2 * halo + 1;
    t.rz = tz + 2 * halo + 1;
    // the slow axis is the one with the finest cells (crossed most often by
    // particles moving alike in every direction); ties go to z, then y
    const double d[3] = {g.Lx / g.nx, g.Ly / g.ny, g.Lz / g.nz};
    int slow = 2;
    if (d[1] < d[slow]) slow = 1;
    if (d[0] < d[slow]) slow = 0;
    t.slow = slow;
    t.mid = slow == 0 ? 1 : 0;
    t.fast = slow == 2 ? 1 : 2;
    const RegionLayout lay = region_layout(tx, ty, tz, halo, t.slow, t.mid, t.fast, layout);
    t.sx = lay.sx;
    t.sy = lay.sy;
    t.sz = lay.sz;
    t.rnp = lay.rnp;
    t.rows = rows ? 1 : 0;
    return t;
}

size_t sort_scratch_bytes(int64_t n, int dtype, bool with_id, const TileGeom &tg) {
    const int64_t nkeys = (int64_t)tg.ntiles * tg.cells;
    const int64_t nparts = (nkeys + SCAN_CHUNK - 1) / SCAN_CHUNK;
    const size_t sp = dtype == SPIC_F64 ? 8 : 4;
    size_t b = 0;
    b += (size_t)nkeys * 4 + 256;          // counts
    b += (size_t)nkeys * 4 + 256;          // counts of a tile's own particles (ordered key pass)
    b += (size_t)(nkeys + 1) * 4 + 256;    // offsets
    b += (size_t)nparts * 4 + 256;         // partials
    b += (size_t)n * 8 + 256;              // key/rank
    b += (size_t)n * 4 + 256;              // source index of every slot
    b += (size_t)(tg.ntiles + 1) * 4 * 2 + 512;   // maxc, tab_off
    b += ((size_t)n + tg.ntiles) * 16 + 256;      // rank tables (sum of max counts <= n)
    b += (size_t)((tg.ntiles + SCAN_CHUNK) / SCAN_CHUNK) * 4 + 256;  // partials of the tile scan
    b += (size_t)nkeys * 8 + 256;                 // full rows: hole / excess prefixes per key
    b += (size_t)(tg.ntiles + 1) * 8 + 256;       // full rows: rows and holes per tile
    b += 7 * ((size_t)n * sp + 256);       // particle copy
    if (with_id) b += (size_t)n * 8 + 256;
    return b;
}

static inline char *carve(char *&cur, size_t bytes) {
    char *p = cur;
    cur += (bytes + 255) & ~(size_t)255;
    return p;
}

template <typename T>
static hipError_t sort_t(const spic_grid &g, const SpeciesWork &w, const TileGeom &tg, void *scratch,
                         uint32_t *tile_off, bool prev, hipStream_t s, SpeciesWork *sorted_out) {
    const int64_t n = w.n;
    const int64_t nkeys = (int64_t)tg.ntiles * tg.cells;
    const int nparts = (int)((nkeys + SCAN_CHUNK - 1) / SCAN_CHUNK);
    char *cur = (char *)scratch;
    uint32_t *counts = (uint32_t *)carve(cur, (size_t)nkeys * 4);
    uint32_t *own = (uint32_t *)carve(cur, (size_t)nkeys * 4);
    uint32_t *offsets = (uint32_t *)carve(cur, (size_t)(nkeys + 1) * 4);
    uint32_t *partial = (uint32_t *)carve(cur, (size_t)nparts * 4);
    uint2 *keyrank = (uint2 *)carve(cur, (size_t)n * 8);
    uint32_t *srcidx = (uint32_t *)carve(cur, (size_t)n * 4);
    uint32_t *maxc = (uint32_t *)carve(cur, (size_t)(tg.ntiles + 1) * 4);
    uint32_t *tab_off = (uint32_t *)carve(cur, (size_t)(tg.ntiles + 1) * 4);
    uint4 *tab = (uint4 *)carve(cur, ((size_t)n + tg.ntiles) * 16);
    const int tparts = (int)((tg.ntiles + SCAN_CHUNK) / SCAN_CHUNK);
    uint32_t *tpartial = (uint32_t *)carve(cur, (size_t)tparts * 4);
    uint2 *hx = (uint2 *)carve(cur, (size_t)nkeys * 8);
    uint2 *rh = (uint2 *)carve(cur, (size_t)(tg.ntiles + 1) * 8);
    PartPtrs<T> src, tmp;
    src.x = (T *)w.a[0]; src.y = (T *)w.a[1]; src.z = (T *)w.a[2];
    src.u = (T *)w.a[3]; src.v = (T *)w.a[4]; src.w = (T *)w.a[5]; src.q = (T *)w.a[6];
    src.id = w.id;
    tmp.x = (T *)carve(cur, n * sizeof(T)); tmp.y = (T *)carve(cur, n * sizeof(T));
    tmp.z = (T *)carve(cur, n * sizeof(T)); tmp.u = (T *)carve(cur, n * sizeof(T));
    tmp.v = (T *)carve(cur, n * sizeof(T)); tmp.w = (T *)carve(cur, n * sizeof(T));
    tmp.q = (T *)carve(cur, n * sizeof(T));
    tmp.id = w.id ? (int64_t *)carve(cur, (size_t)n * 8) : nullptr;

    hipError_t e;
    if ((e = launch_zero32(counts, nkeys, s)) != hipSuccess) return e;
    const int gp = (int)std::min<int64_t>((n + 255) / 256, 1 << 16);
    if (prev) {  // tile_off still holds the ranges of the current order
        hipLaunchKernelGGL((k_sort_keys_tiled<T>), dim3(std::min(tg.ntiles, 1 << 20)), dim3(256), 0, s,
                           make_grid_t<T>(g), tg, src.x, src.y, src.z, (const uint32_t *)tile_off, own, counts,
                           keyrank);
        const int gk = (int)std::min<int64_t>((nkeys + 255) / 256, 1 << 16);
        hipLaunchKernelGGL(k_sort_counts, dim3(gk > 0 ? gk : 1), dim3(256), 0, s, own, counts, nkeys);
    } else {
        hipLaunchKernelGGL((k_sort_keys<T>), dim3(gp > 0 ? gp : 1), dim3(256), 0, s, make_grid_t<T>(g), tg, src.x,
                           src.y, src.z, n, counts, keyrank);
    }
    hipLaunchKernelGGL(k_scan_partials, dim3(nparts), dim3(SCAN_BLOCK), 0, s, counts, nkeys, partial);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, partial, nparts);
    hipLaunchKernelGGL(k_scan_apply, dim3(nparts), dim3(SCAN_BLOCK), 0, s, counts, nkeys, partial, offsets);
    if (tg.rows) {
        hipLaunchKernelGGL(k_tile_rows, dim3(tg.ntiles), dim3(64), 0, s, offsets, tg, hx, rh);
        hipLaunchKernelGGL(k_sort_slots_rows, dim3(gp > 0 ? gp : 1), dim3(256), 0, s, n, keyrank, offsets, hx, rh,
                           tg.cells, prev ? (const uint32_t *)own : nullptr, srcidx);
    } else {
        // rank tables: max count per tile, exclusive scan of the max counts, fill
        hipLaunchKernelGGL(k_tile_maxc, dim3(tg.ntiles), dim3(64), 0, s, offsets, tg, maxc);
        hipLaunchKernelGGL(k_scan_partials, dim3(tparts), dim3(SCAN_BLOCK), 0, s, maxc, (int64_t)tg.ntiles,
                           tpartial);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, tpartial, tparts);
        hipLaunchKernelGGL(k_scan_apply, dim3(tparts), dim3(SCAN_BLOCK), 0, s, maxc, (int64_t)tg.ntiles, tpartial,
                           tab_off);
        hipLaunchKernelGGL(k_tile_table, dim3(tg.ntiles), dim3(64), 0, s, offsets, tg, tab_off, tab);
        hipLaunchKernelGGL(k_sort_slots, dim3(gp > 0 ? gp : 1), dim3(256), 0, s, n, keyrank, offsets, tab_off, tab,
                           tg.cells, prev ? (const uint32_t *)own : nullptr, srcidx);
    }
    if (prev)  // tile_off still holds the previous sort's tile ranges
        hipLaunchKernelGGL((k_sort_gather_tiled<T>), dim3(8 * tile_chunk(tg.ntiles, kTileGroup)), dim3(256), 0, s,
                           src, tmp, n, srcidx, (const uint32_t *)tile_off, offsets, tg.cells, tg.ntiles,
                           tile_chunk(tg.ntiles, kTileGroup), kTileGroup);
    else
        hipLaunchKernelGGL((k_sort_gather<T>), dim3(gp > 0 ? gp : 1), dim3(256), 0, s, src, tmp, n, srcidx);
    if (sorted_out) {  // the next kernel reads the reordered copy and writes w's arrays
        *sorted_out = w;
        sorted_out->from_src = true;
        sorted_out->src[0] = tmp.x; sorted_out->src[1] = tmp.y; sorted_out->src[2] = tmp.z;
        sorted_out->src[3] = tmp.u; sorted_out->src[4] = tmp.v; sorted_out->src[5] = tmp.w;
        sorted_out->src[6] = tmp.q;
        sorted_out->src_id = tmp.id;
    } else {
        hipLaunchKernelGGL((k_copy_parts<T>), dim3(gp > 0 ? gp : 1), dim3(256), 0, s, tmp, src, n);
    }
    hipLaunchKernelGGL(k_tile_offsets, dim3((tg.ntiles + 1 + 255) / 256), dim3(256), 0, s, offsets, tg, tg.ntiles,
                       tile_off);
    return hipGetLastError();
}

hipError_t launch_sort(const spic_grid &g, const SpeciesWork &w, const TileGeom &tg, void *scratch,
                       uint32_t *tile_off, bool prev, hipStream_t s, SpeciesWork *sorted_out) {
    if (w.n <= 0) {
        if (sorted_out) *sorted_out = w;
        return launch_zero32(tile_off, tg.ntiles + 1, s);
    }
    if (!scratch || !tile_off) return hipErrorInvalidValue;  // nothing is launched without scratch
    return w.dtype == SPIC_F64 ? sort_t<double>(g, w, tg, scratch, tile_off, prev, s, sorted_out)
                               : sort_t<float>(g, w, tg, scratch, tile_off, prev, s, sorted_out);
}

}  // namespace spic
