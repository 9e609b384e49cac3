// spic_noalloc.hip -- spic_mover_noalloc: the fused step with a sort of
// every species before its move, whose scratch (sort keys, ranks, slot
// indices, the reordered copy of the particles, per-tile ranges) lives in
// one fixed array of device memory instead of memory the library
// allocates, for callers that cannot allocate (code under stream capture,
// serving loops, harnesses that forbid hipMalloc).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "spic_ctx.h"
#include "spic_impl.h"

namespace {

// The fixed scratch: one copy per GPU, held until the process ends.  In
// host code its name stands for a host-side symbol, not a device address;
// kernels get the address that hipGetSymbolAddress returns for the current
// device (noalloc_scratch below).
__device__ __align__(256) unsigned char scratch[SPIC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

}  // namespace

namespace spic {

// Device address of the fixed scratch on `device` (which must be current),
// looked up once per device.  NULL with *err set when the lookup fails.
void *noalloc_scratch(int device, hipError_t *err) {
    *err = hipSuccess;
    if (device < 0 || device >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return nullptr;
        }
        g_ptr[device] = p;
    }
    return g_ptr[device];
}

}  // namespace spic

using namespace spic;

// Sizes first (host only, also on a host-only context): every species must
// fit the tiled path and its sort the fixed scratch.
int spic_ctx_s::noalloc_check(const spic_grid &g, const spic_species *sp, int32_t nsp,
                              const spic_moment_array *mom) {
    const LaunchCfg cfg = launch_cfg();
    for (int i = 0; i < nsp; ++i) {
        const TileGeom tg = tile_geom(g, sp[i].dtype);
        if (tg.cells < 1 || tg.cells > 64 || tg.halo < 0 || tg.halo > 8)
            return fail(SPIC_E_ARG, "tile shape %dx%dx%d (halo %d): a tile holds 1..64 cells, halo 0..8", tg.tx,
                        tg.ty, tg.tz, tg.halo);
        if (!tiled_fits(sp[i].n, sp[i].dtype))
            return fail(SPIC_E_UNSUPPORTED, "species %d: the fixed-scratch step needs n * element size < 4 GiB", i);
        const size_t toff = (((size_t)tg.ntiles + 1) * 4 + 255) & ~(size_t)255;
        const size_t need = toff + sort_scratch_bytes(sp[i].n, sp[i].dtype, sp[i].id != nullptr, tg);
        if (need > (size_t)SPIC_NOALLOC_SCRATCH_BYTES)
            return fail(SPIC_E_BUDGET,
                        "species %d: %lld particles need %zu bytes of scratch; the fixed scratch holds %zu "
                        "(SPIC_NOALLOC_SCRATCH_BYTES)",
                        i, (long long)sp[i].n, need, (size_t)SPIC_NOALLOC_SCRATCH_BYTES);
        const int acc = mom ? mom[i].acc_dtype : SPIC_F64;
        if (acc == SPIC_F32C)
            return fail(SPIC_E_UNSUPPORTED, "species %d: compensated FP32 moments take the unsorted path", i);
        const LaunchCfg tcfg = resolve_cfg(cfg, sp[i].dtype, acc);
        if (tiled_lds_bytes(tg, sp[i].dtype, acc, tcfg.variant, tcfg.tile_block) > lds_max &&
            tiled_lds_bytes(tg, sp[i].dtype, acc, 0, 512) > lds_max)
            return fail(SPIC_E_UNSUPPORTED, "species %d: the tile region does not fit the device's LDS", i);
    }
    return SPIC_OK;
}

// One fused step of every species with a sort before each move, all
// scratch in the fixed array (validated and sized arguments, device
// current).  Species run one after the other on the stream, so they reuse
// the same scratch.
int spic_ctx_s::mover_noalloc(const spic_grid &g, const spic_params &p, const spic_fields &f, spic_species *sp,
                              int32_t nsp, spic_moment_array *mom, hipStream_t s) {
    hipError_t e;
    char *base = (char *)noalloc_scratch(device, &e);
    if (!base) return hip(e, "fixed scratch lookup");
    const int64_t nn = (int64_t)g.nx * g.ny * g.nz;
    const LaunchCfg cfg = launch_cfg();
    for (int i = 0; i < nsp; ++i) {
        SpeciesWork w;
        w.dtype = sp[i].dtype;
        w.n = sp[i].n;
        w.qom = sp[i].qom;
        w.a[0] = sp[i].x; w.a[1] = sp[i].y; w.a[2] = sp[i].z;
        w.a[3] = sp[i].u; w.a[4] = sp[i].v; w.a[5] = sp[i].w; w.a[6] = sp[i].q;
        w.id = sp[i].id;
        w.mom = mom ? mom[i].m : nullptr;
        w.acc_dtype = mom ? mom[i].acc_dtype : SPIC_F64;
        int rc;
        if (w.mom && (rc = hip(launch_fill(w.mom, w.acc_dtype, 10 * nn, s), "zero moments"))) return rc;
        if (w.n == 0) continue;
        const TileGeom tg = tile_geom(g, w.dtype);
        const size_t toff_bytes = (((size_t)tg.ntiles + 1) * 4 + 255) & ~(size_t)255;
        uint32_t *toff = (uint32_t *)base;
        SpeciesWork sorted;
        // a sort layout an earlier spic_sort kept for this species no longer
        // matches the new order; dropping it frees no device memory
        layouts.erase(layout_key(g, sp[i]));
        if ((rc = hip(launch_sort(g, w, tg, base + toff_bytes, toff, false, s, &sorted), "sort (fixed scratch)")))
            return rc;
        sorted.mom = w.mom;
        sorted.acc_dtype = w.acc_dtype;
        LaunchCfg tcfg = resolve_cfg(cfg, w.dtype, w.mom ? w.acc_dtype : SPIC_F64);
        if (tiled_lds_bytes(tg, w.dtype, w.acc_dtype, tcfg.variant, tcfg.tile_block) > lds_max) {
            tcfg.variant = 0;
            tcfg.tile_block = 512;
        }
        if ((rc = hip(launch_fused_tiled(g, p, f, sorted, tg, toff, tcfg, s), "fused mover (fixed scratch)")))
            return rc;
    }
    return SPIC_OK;
}
