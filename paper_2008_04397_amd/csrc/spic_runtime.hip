// spic_runtime.hip -- host side of libspic.so: the C ABI of include/spic.h,
// argument validation, the context (device, HBM budget, scratch, options)
// and the dispatch to the HIP kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "spic_impl.h"
#include "spic_ctx.h"

using namespace spic;

// ------------------------------------------------------------------ errors

int spic_ctx_s::fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    return code;
}

int spic_ctx_s::host_only() {
    return fail(SPIC_E_STATE, "host-only context (device -1): arguments are valid, no work is enqueued");
}

int spic_ctx_s::hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return SPIC_OK;
    return fail(SPIC_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (dev < 0) return;  // host-only context: no HIP call at all
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

bool dtype_ok(int d) { return d == SPIC_F32 || d == SPIC_F64; }

}  // namespace

// --------------------------------------------------------------- validation

int spic_ctx_s::check_grid(const spic_grid *g) {
    if (!g) return fail(SPIC_E_ARG, "grid is NULL");
    if (g->reserved != 0) return fail(SPIC_E_ARG, "grid.reserved must be 0");
    if (g->nx < 2 || g->ny < 2 || g->nz < 2)
        return fail(SPIC_E_ARG, "grid needs at least 2 cells per axis (got %d x %d x %d)", g->nx, g->ny, g->nz);
    const double nn = (double)g->nx * g->ny * g->nz;
    if (nn > 1.0e9) return fail(SPIC_E_ARG, "grid has %.3g nodes; the limit is 1e9", nn);
    if (!(g->Lx > 0) || !(g->Ly > 0) || !(g->Lz > 0) || !std::isfinite(g->Lx) || !std::isfinite(g->Ly) ||
        !std::isfinite(g->Lz))
        return fail(SPIC_E_ARG, "box lengths must be finite and > 0");
    return SPIC_OK;
}

int spic_ctx_s::check_params(const spic_params *p) {
    if (!p) return fail(SPIC_E_ARG, "params is NULL");
    if (!std::isfinite(p->dt)) return fail(SPIC_E_ARG, "dt must be finite");
    if (!(p->c > 0) || !std::isfinite(p->c)) return fail(SPIC_E_ARG, "c must be finite and > 0");
    if (p->niter_mover < 1 || p->niter_mover > 1000) return fail(SPIC_E_ARG, "niter_mover must be in [1, 1000]");
    if (!(p->mover_tol >= 0) || !std::isfinite(p->mover_tol))
        return fail(SPIC_E_ARG, "mover_tol must be finite and >= 0");
    if (p->sort_every < 0) return fail(SPIC_E_ARG, "sort_every must be >= 0");
    if (p->step < 0) return fail(SPIC_E_ARG, "step must be >= 0");
    return SPIC_OK;
}

int spic_ctx_s::check_fields(const spic_fields *f) {
    if (!f) return fail(SPIC_E_ARG, "fields is NULL");
    if (!dtype_ok(f->dtype)) return fail(SPIC_E_ARG, "fields.dtype %d is not SPIC_F32/SPIC_F64", f->dtype);
    if (f->reserved != 0) return fail(SPIC_E_ARG, "fields.reserved must be 0");
    const void *p[6] = {f->ex, f->ey, f->ez, f->bx, f->by, f->bz};
    const size_t al = f->dtype == SPIC_F64 ? 8 : 4;
    for (int i = 0; i < 6; ++i) {
        if (!p[i]) return fail(SPIC_E_ARG, "field array %d is NULL", i);
        if ((uintptr_t)p[i] % al) return fail(SPIC_E_ARG, "field array %d is misaligned", i);
    }
    return SPIC_OK;
}

int spic_ctx_s::check_field(const spic_grid *g, const spic_field_params *fp, const spic_em_state *em,
                            const spic_moment_array *mom, const double *qom, int32_t nsp) {
    int rc;
    if ((rc = check_grid(g))) return rc;
    if (!fp) return fail(SPIC_E_ARG, "field params is NULL");
    if (!(fp->dt > 0.0) || !std::isfinite(fp->dt)) return fail(SPIC_E_ARG, "field params: dt must be finite and > 0");
    if (!(fp->c > 0.0) || !std::isfinite(fp->c)) return fail(SPIC_E_ARG, "field params: c must be finite and > 0");
    if (!(fp->theta > 0.0 && fp->theta <= 1.0)) return fail(SPIC_E_ARG, "field params: theta must be in (0, 1]");
    if (!(fp->fourpi >= 0.0) || !std::isfinite(fp->fourpi))
        return fail(SPIC_E_ARG, "field params: fourpi must be finite and >= 0");
    if (!(fp->tol > 0.0 && fp->tol < 1.0)) return fail(SPIC_E_ARG, "field params: tol must be in (0, 1)");
    if (fp->max_iter < 1) return fail(SPIC_E_ARG, "field params: max_iter must be >= 1");
    if (fp->restart < 1 || fp->restart > 64) return fail(SPIC_E_ARG, "field params: restart must be in 1..64");
    if (!em) return fail(SPIC_E_ARG, "em state is NULL");
    const double *p[6] = {em->ex, em->ey, em->ez, em->bx, em->by, em->bz};
    for (int i = 0; i < 6; ++i) {
        if (!p[i]) return fail(SPIC_E_ARG, "em array %d is NULL", i);
        if ((uintptr_t)p[i] % 8) return fail(SPIC_E_ARG, "em array %d is misaligned", i);
    }
    if (nsp < 0 || nsp > 16) return fail(SPIC_E_ARG, "field solve: nsp must be in 0..16");
    if (nsp > 0 && (!mom || !qom)) return fail(SPIC_E_ARG, "field solve: moments or qom array is NULL");
    for (int s = 0; s < nsp; ++s) {
        if (mom[s].acc_dtype != SPIC_F64)
            return fail(SPIC_E_ARG, "field solve: species %d moments must be SPIC_F64", s);
        if (mom[s].reserved != 0) return fail(SPIC_E_ARG, "field solve: species %d moments.reserved must be 0", s);
        if (!mom[s].m || (uintptr_t)mom[s].m % 8) return fail(SPIC_E_ARG, "field solve: species %d moments", s);
        if (!std::isfinite(qom[s])) return fail(SPIC_E_ARG, "field solve: species %d qom is not finite", s);
    }
    return SPIC_OK;
}

int spic_ctx_s::check_species(const spic_species *sp, int32_t nsp, bool allow_host) {
    if (nsp < 0) return fail(SPIC_E_ARG, "nsp must be >= 0");
    if (nsp > 0 && !sp) return fail(SPIC_E_ARG, "species array is NULL");
    for (int s = 0; s < nsp; ++s) {
        const spic_species &x = sp[s];
        if (!dtype_ok(x.dtype)) return fail(SPIC_E_ARG, "species %d: dtype %d is not SPIC_F32/SPIC_F64", s, x.dtype);
        if (x.n < 0) return fail(SPIC_E_ARG, "species %d: n < 0", s);
        if (x.n > ((int64_t)1 << 40)) return fail(SPIC_E_ARG, "species %d: n too large", s);
        if (x.host_resident != 0 && x.host_resident != 1)
            return fail(SPIC_E_ARG, "species %d: host_resident must be 0 or 1", s);
        if (x.host_resident && !allow_host)
            return fail(SPIC_E_ARG, "species %d: host-resident particles are only accepted by spic_batch_submit", s);
        if (!std::isfinite(x.qom)) return fail(SPIC_E_ARG, "species %d: qom must be finite", s);
        if (x.n == 0) continue;
        const void *a[7] = {x.x, x.y, x.z, x.u, x.v, x.w, x.q};
        const size_t al = x.dtype == SPIC_F64 ? 8 : 4;
        for (int i = 0; i < 7; ++i) {
            if (!a[i]) return fail(SPIC_E_ARG, "species %d: array %d is NULL", s, i);
            if ((uintptr_t)a[i] % al) return fail(SPIC_E_ARG, "species %d: array %d is misaligned", s, i);
        }
        if (x.id && ((uintptr_t)x.id % 8)) return fail(SPIC_E_ARG, "species %d: id is misaligned", s);
    }
    return SPIC_OK;
}

int spic_ctx_s::check_moments(const spic_moment_array *m, const spic_species *sp, int32_t nsp) {
    if (!m) return SPIC_OK;
    for (int s = 0; s < nsp; ++s) {
        if (m[s].reserved != 0) return fail(SPIC_E_ARG, "moments %d: reserved must be 0", s);
        if (!dtype_ok(m[s].acc_dtype) && m[s].acc_dtype != SPIC_F32C)
            return fail(SPIC_E_ARG, "moments %d: acc_dtype %d invalid", s, m[s].acc_dtype);
        if (!m[s].m) return fail(SPIC_E_ARG, "moments %d: array is NULL", s);
        if ((uintptr_t)m[s].m % (m[s].acc_dtype == SPIC_F64 ? 8 : 4))
            return fail(SPIC_E_ARG, "moments %d: array is misaligned", s);
        if (sp[s].dtype == SPIC_F64 && m[s].acc_dtype != SPIC_F64)
            return fail(SPIC_E_UNSUPPORTED, "moments %d: FP64 particles need FP64 accumulation", s);
    }
    return SPIC_OK;
}

int spic_ctx_s::check_combo(const spic_fields *f, const spic_species *sp, int32_t nsp) {
    for (int s = 0; s < nsp; ++s) {
        if (sp[s].dtype == SPIC_F64 && f->dtype != SPIC_F64)
            return fail(SPIC_E_UNSUPPORTED, "species %d: FP64 particles need FP64 fields", s);
    }
    return SPIC_OK;
}

// -------------------------------------------------------------- scratch

int spic_ctx_s::reserve(const char *tag, size_t bytes, void **out) {
    Scratch &sc = scratch[tag];
    if (sc.bytes >= bytes && sc.ptr) {
        *out = sc.ptr;
        return SPIC_OK;
    }
    const uint64_t new_used = used - sc.bytes + bytes;
    if (budget && new_used > budget)
        return fail(SPIC_E_BUDGET, "scratch '%s' of %zu bytes exceeds the HBM budget (%llu of %llu bytes in use)",
                    tag, bytes, (unsigned long long)used, (unsigned long long)budget);
    if (sc.ptr) {
        // the old buffer may still be read by enqueued work on any stream
        (void)hipDeviceSynchronize();
        (void)hipFree(sc.ptr);
        used -= sc.bytes;
        sc.ptr = nullptr;
        sc.bytes = 0;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes ? bytes : 256);
    if (e != hipSuccess) return hip(e, "hipMalloc(scratch)");
    sc.ptr = p;
    sc.bytes = bytes;
    used += bytes;
    *out = p;
    return SPIC_OK;
}

void spic_ctx_s::release_all() {
    for (auto &kv : scratch)
        if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    scratch.clear();
    used = 0;
}

// ------------------------------------------------------------------ options

static const char *const kOptionNames[] = {
    "block",        // threads per block of the generic kernels
    "grid_cap",     // cap on blocks of the grid-stride kernels
    "path",         // 0 auto (tiled for sorted species), 1 generic only
    "tile_block",   // threads per block of the tiled kernel (variant 2: of the deposit launch)
    "tile_x", "tile_y", "tile_z",  // sort tile shape in cells (product <= 64)
    "halo",         // cells of halo staged around a tile
    "lds_max",      // read only: LDS bytes per workgroup on the device
    "tile_variant", // tiled kernel: 0 one kernel with LDS-atomic deposits, 1 + field corners in registers,
                    // 2 mover launch then the sorted register deposit, 3 both in one launch (FP32)
    "fixed_geo",    // tiled kernel: 1 = compile-time region geometry for 4x4x4 tiles, halo 1
    "sort_ordered", // sort: 1 = ranks follow the previous order (a sorted species' tiles walked in order)
    "sort_rows",    // sort: 1 = full rows (lane = cell for all but a few particles), 0 = plain rank blocks
                    // (default: 1 for variants 2 and 3)
    "bank_align",   // tiled kernel LDS layout: 0 compact conflict-free, 1 + slow-axis stride keeps bank pairs,
                    // 2 dense (no padding)
    "graph",        // batch engine: 1 = replay unchanged ticks as a hipGraph
    "batch_particles",  // batch engine: particles per streamed batch (upper bound)
    "max_groups",   // batch engine: cap on workgroups of the persistent launch (0 = occupancy)
    "tick_items",   // batch engine: (job, tile) items per tick, shortest runs first (0 = all runs)
    "srpt_aging",   // batch engine: credit, in M particle-steps per second waited, against starvation
    "mover_halo",   // variants 2, 3: halo of the mover's field region (-1: tile halo + 1)
    "mover_cache",  // variant 2: 1 = the mover keeps the last cell's field corners in registers
    "mover_block",  // variant 2: threads per workgroup of the mover launch (64..512, x64; default 512)
    "tile_group",   // tiles to workgroups: groups of 2^v tiles dealt to the XCDs (default 4); -1 XCD slabs
};

int64_t spic_ctx_s::opt(const char *k, int64_t dflt) const {
    auto it = options.find(k);
    return it == options.end() ? dflt : it->second;
}

LaunchCfg spic_ctx_s::launch_cfg() const {
    LaunchCfg c;
    c.block = (int)opt("block", 256);
    c.grid_cap = (int)opt("grid_cap", 1 << 20);
    c.tile_block = (int)opt("tile_block", -1);
    c.variant = (int)opt("tile_variant", -1);
    c.fixed_geo = (int)opt("fixed_geo", 1);
    c.mover_halo = (int)opt("mover_halo", -1);
    c.mover_cache = (int)opt("mover_cache", 1);
    c.mover_block = (int)opt("mover_block", 512);
    c.tile_group = (int)opt("tile_group", kTileGroup);
    c.lds_max = lds_max;
    return c;
}

// ================================================================== C ABI

extern "C" {

int spic_version(void) { return SPIC_ABI_VERSION; }

const char *spic_status_str(int status) {
    switch (status) {
        case SPIC_OK: return "SPIC_OK";
        case SPIC_E_ARG: return "SPIC_E_ARG";
        case SPIC_E_BUDGET: return "SPIC_E_BUDGET";
        case SPIC_E_HIP: return "SPIC_E_HIP";
        case SPIC_E_UNSUPPORTED: return "SPIC_E_UNSUPPORTED";
        case SPIC_E_STATE: return "SPIC_E_STATE";
        default: return "SPIC_E_UNKNOWN";
    }
}

int spic_ctx_create(int device, uint64_t hbm_budget_bytes, spic_ctx *out) {
    if (!out) return SPIC_E_ARG;
    *out = nullptr;
    if (device != -1) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return SPIC_E_HIP;
        if (device < 0 || device >= ndev) return SPIC_E_ARG;
    }
    spic_ctx c = new (std::nothrow) spic_ctx_s();
    if (!c) return SPIC_E_HIP;
    c->device = device;
    c->budget = hbm_budget_bytes;
    if (device >= 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && v > 0)
            c->lds_max = (size_t)v;
        // set-up of spic_mover_noalloc: the device address of its fixed
        // scratch on this device, looked up once per device with it current
        // (a failure surfaces at that entry point's call)
        DeviceGuard dg(device);
        hipError_t e;
        (void)spic::noalloc_scratch(device, &e);
    }
    *out = c;
    return SPIC_OK;
}

int spic_ctx_destroy(spic_ctx ctx) {
    if (!ctx) return SPIC_OK;
    if (ctx->device >= 0) {
        DeviceGuard dg(ctx->device);
        ctx->shutdown();
        (void)hipDeviceSynchronize();
        ctx->release_all();
    }
    delete ctx;
    return SPIC_OK;
}

const char *spic_last_error(spic_ctx ctx) { return ctx ? ctx->err.c_str() : "ctx is NULL"; }

int spic_set_option(spic_ctx ctx, const char *key, int64_t value) {
    if (!ctx || !key) return SPIC_E_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (const char *k : kOptionNames)
        if (!strcmp(k, key)) {
            if (!strcmp(key, "block") && (value < 64 || value > 1024 || value % 64))
                return ctx->fail(SPIC_E_ARG, "block must be a multiple of 64 in [64, 1024]");
            if (!strcmp(key, "grid_cap") && (value < 1 || value > (1 << 24)))
                return ctx->fail(SPIC_E_ARG, "grid_cap must be in [1, 2^24]");
            if (!strcmp(key, "path") && (value < 0 || value > 1))
                return ctx->fail(SPIC_E_ARG, "path must be 0 (auto) or 1 (generic)");
            if (!strcmp(key, "mover_block") && (value < 64 || value > 512 || value % 64))
                return ctx->fail(SPIC_E_ARG, "mover_block must be a multiple of 64 in [64, 512]");
            if (!strcmp(key, "tile_block") && value != -1 && (value < 64 || value > 512 || value % 64))
                return ctx->fail(SPIC_E_ARG, "tile_block must be -1 or a multiple of 64 in [64, 512]");
            if ((!strcmp(key, "tile_x") || !strcmp(key, "tile_y") || !strcmp(key, "tile_z")) &&
                (value < 1 || value > 64))
                return ctx->fail(SPIC_E_ARG, "tile sizes must be in [1, 64]");
            if (!strcmp(key, "tile_variant") && (value < -1 || value > 3))
                return ctx->fail(SPIC_E_ARG, "tile_variant must be -1 or in 0..3");
            if (!strcmp(key, "batch_particles") && (value < 1024 || value > ((int64_t)1 << 29)))
                return ctx->fail(SPIC_E_ARG, "batch_particles must be in [1024, 2^29]");
            if (!strcmp(key, "tick_items") && (value < 0 || value > ((int64_t)1 << 30)))
                return ctx->fail(SPIC_E_ARG, "tick_items must be in [0, 2^30]");
            if (!strcmp(key, "srpt_aging") && (value < 0 || value > ((int64_t)1 << 40)))
                return ctx->fail(SPIC_E_ARG, "srpt_aging must be in [0, 2^40]");
            if ((!strcmp(key, "fixed_geo") || !strcmp(key, "sort_ordered") || !strcmp(key, "sort_rows") ||
                 !strcmp(key, "mover_cache")) &&
                (value < 0 || value > 1))
                return ctx->fail(SPIC_E_ARG, "%s must be 0 or 1", key);
            if (!strcmp(key, "bank_align") && (value < 0 || value > 2))
                return ctx->fail(SPIC_E_ARG, "bank_align must be 0, 1 or 2");
            if (!strcmp(key, "halo") && (value < 0 || value > 8))
                return ctx->fail(SPIC_E_ARG, "halo must be in [0, 8]");
            if (!strcmp(key, "tile_group") && (value < -1 || value > 10))
                return ctx->fail(SPIC_E_ARG, "tile_group must be -1 or in 0..10");
            if (!strcmp(key, "mover_halo") && (value < -1 || value > 8))
                return ctx->fail(SPIC_E_ARG, "mover_halo must be -1 or in [0, 8]");
            if (!strcmp(key, "lds_max")) return ctx->fail(SPIC_E_ARG, "lds_max is read only");
            ctx->options[key] = value;
            return SPIC_OK;
        }
    return ctx->fail(SPIC_E_ARG, "unknown option '%s'", key);
}

int spic_get_option(spic_ctx ctx, const char *key, int64_t *value) {
    if (!ctx || !key || !value) return SPIC_E_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    // "f32:<name>" / "f64:<name>": the setting the library resolves for
    // particles of that precision with FP64 moments
    if ((!strncmp(key, "f32:", 4) || !strncmp(key, "f64:", 4)) && key[4]) {
        const int dt = key[2] == '2' ? SPIC_F32 : SPIC_F64;
        const char *k = key + 4;
        const LaunchCfg c = resolve_cfg(ctx->launch_cfg(), dt, SPIC_F64);
        const TileGeom tg = ctx->tile_geom(spic_grid{8, 8, 8, 0, 1.0, 1.0, 1.0}, dt);
        if (!strcmp(k, "tile_variant")) *value = c.variant;
        else if (!strcmp(k, "tile_block")) *value = c.tile_block;
        else if (!strcmp(k, "sort_rows")) *value = tg.rows;
        else if (!strcmp(k, "halo")) *value = tg.halo;
        else if (!strcmp(k, "bank_align")) *value = ctx->opt("bank_align", dt == SPIC_F64 ? 0 : 1);
        else if (!strcmp(k, "sort_ordered")) *value = ctx->opt("sort_ordered", 1);
        else if (!strcmp(k, "mover_cache")) *value = c.mover_cache;
        else if (!strcmp(k, "mover_halo")) *value = c.mover_halo >= 0 ? c.mover_halo : tg.halo + 1;
        else if (!strcmp(k, "tile_group")) *value = c.tile_group;
        else return ctx->fail(SPIC_E_ARG, "unknown resolved setting '%s'", key);
        return SPIC_OK;
    }
    for (const char *k : kOptionNames)
        if (!strcmp(k, key)) {
            if (!strcmp(key, "lds_max")) *value = (int64_t)ctx->lds_max;
            else if (!strcmp(key, "tile_group")) *value = ctx->opt(key, kTileGroup);  // -1 is a value here
            else *value = ctx->opt(key, -1);
            return SPIC_OK;
        }
    return ctx->fail(SPIC_E_ARG, "unknown option '%s'", key);
}

int spic_mover(spic_ctx ctx, const spic_grid *grid, const spic_params *params, const spic_fields *fields,
               spic_species *sp, int32_t nsp, spic_moment_array *mom, void *hip_stream) {
    if (!ctx) return SPIC_E_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->err.clear();
    int rc;
    if ((rc = ctx->check_grid(grid)) || (rc = ctx->check_params(params)) || (rc = ctx->check_fields(fields)) ||
        (rc = ctx->check_species(sp, nsp, false)) || (rc = ctx->check_moments(mom, sp, nsp)) ||
        (rc = ctx->check_combo(fields, sp, nsp)))
        return rc;
    if (ctx->device < 0) return ctx->host_only();
    DeviceGuard dg(ctx->device);
    return ctx->mover(*grid, *params, *fields, sp, nsp, mom, (hipStream_t)hip_stream);
}

int spic_mover_noalloc(spic_ctx ctx, const spic_grid *grid, const spic_params *params, const spic_fields *fields,
                       spic_species *sp, int32_t nsp, spic_moment_array *mom, void *hip_stream) {
    if (!ctx) return SPIC_E_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->err.clear();
    int rc;
    if ((rc = ctx->check_grid(grid)) || (rc = ctx->check_params(params)) || (rc = ctx->check_fields(fields)) ||
        (rc = ctx->check_species(sp, nsp, false)) || (rc = ctx->check_moments(mom, sp, nsp)) ||
        (rc = ctx->check_combo(fields, sp, nsp)))
        return rc;
    if (params->sort_every != 1)
        return ctx->fail(SPIC_E_ARG, "spic_mover_noalloc sorts every species before its move: sort_every must be 1");
    if ((rc = ctx->noalloc_check(*grid, sp, nsp, mom))) return rc;
    if (ctx->device < 0) return ctx->host_only();
    DeviceGuard dg(ctx->device);
    return ctx->mover_noalloc(*grid, *params, *fields, sp, nsp, mom, (hipStream_t)hip_stream);
}

int spic_moments(spic_ctx ctx, const spic_grid *grid, const spic_species *sp, int32_t nsp, spic_moment_array *mom,
                 int32_t accumulate, void *hip_stream) {
    if (!ctx) return SPIC_E_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->err.clear();
    int rc;
    if ((rc = ctx->check_grid(grid)) || (rc = ctx->check_species(sp, nsp, false))) return rc;
    if (nsp > 0 && !mom) return ctx->fail(SPIC_E_ARG, "moments array is NULL");
    if ((rc = ctx->check_moments(mom, sp, nsp))) return rc;
    if (ctx->device < 0) return ctx->host_only();
    DeviceGuard dg(ctx->device);
    return ctx->moments(*grid, sp, nsp, mom, accumulate != 0, (hipStream_t)hip_stream);
}

int spic_sort(spic_ctx ctx, const spic_grid *grid, spic_species *sp, int32_t nsp, void *hip_stream) {
    if (!ctx) return SPIC_E_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->err.clear();
    int rc;
    if ((rc = ctx->check_grid(grid)) || (rc = ctx->check_species(sp, nsp, false))) return rc;
    if (ctx->device < 0) return ctx->host_only();
    DeviceGuard dg(ctx->device);
    return ctx->sort(*grid, sp, nsp, (hipStream_t)hip_stream);
}

int spic_field_apply(spic_ctx ctx, const spic_grid *grid, const spic_field_params *params,
                     const spic_em_state *em, const spic_moment_array *mom, const double *qom, int32_t nsp,
                     const double *x, double *y, void *hip_stream) {
    if (!ctx) return SPIC_E_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->err.clear();
    int rc;
    if ((rc = ctx->check_field(grid, params, em, mom, qom, nsp))) return rc;
    if (!x || !y || x == y || (uintptr_t)x % 8 || (uintptr_t)y % 8)
        return ctx->fail(SPIC_E_ARG, "field apply: x and y must be distinct, aligned, non-NULL");
    if (ctx->device < 0) return ctx->host_only();
    DeviceGuard dg(ctx->device);
    return ctx->field_apply(*grid, *params, *em, mom, qom, nsp, x, y, (hipStream_t)hip_stream);
}

int spic_field_cycle(spic_ctx ctx, const spic_grid *grid, const spic_field_params *params, spic_em_state *em,
                     const spic_moment_array *mom, const double *qom, int32_t nsp, spic_field_stats *stats,
                     void *hip_stream) {
    if (!ctx) return SPIC_E_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->err.clear();
    int rc;
    if ((rc = ctx->check_field(grid, params, em, mom, qom, nsp))) return rc;
    if (ctx->device < 0) return ctx->host_only();
    DeviceGuard dg(ctx->device);
    return ctx->field_cycle(*grid, *params, *em, mom, qom, nsp, stats, (hipStream_t)hip_stream);
}

int spic_batch_submit(spic_ctx ctx, const spic_run *runs, int32_t nruns, uint64_t *tickets_out) {
    if (!ctx) return SPIC_E_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->err.clear();
    if (nruns < 0 || (nruns > 0 && (!runs || !tickets_out))) return ctx->fail(SPIC_E_ARG, "bad runs/tickets");
    for (int r = 0; r < nruns; ++r) {
        const spic_run &R = runs[r];
        int rc;
        if ((rc = ctx->check_grid(&R.grid)) || (rc = ctx->check_params(&R.params)) ||
            (rc = ctx->check_fields(&R.fields)) || (rc = ctx->check_species(R.species, R.nspecies, true)) ||
            (rc = ctx->check_moments(R.moments, R.species, R.nspecies)) ||
            (rc = ctx->check_combo(&R.fields, R.species, R.nspecies)))
            return ctx->fail(rc, "run %d: %s", r, std::string(ctx->err).c_str());
        if (R.nsteps < 0) return ctx->fail(SPIC_E_ARG, "run %d: nsteps < 0", r);
        // admission plan (host only): a run that cannot fit the budget even
        // streamed is refused here, also on a host-only context
        spic::RunPlan plan;
        if ((rc = ctx->plan_run(R, r, plan))) return rc;
    }
    if (ctx->device < 0) return ctx->host_only();
    DeviceGuard dg(ctx->device);
    return ctx->batch_submit(runs, nruns, tickets_out);
}

int spic_wait(spic_ctx ctx, uint64_t ticket, double *device_seconds_out) {
    if (!ctx) return SPIC_E_ARG;
    if (ctx->device < 0) return ctx->host_only();
    DeviceGuard dg(ctx->device);
    return ctx->wait(ticket, device_seconds_out);
}

int spic_poll(spic_ctx ctx, uint64_t ticket, int32_t *done) {
    if (!ctx || !done) return SPIC_E_ARG;
    if (ctx->device < 0) return ctx->host_only();
    DeviceGuard dg(ctx->device);
    return ctx->poll(ticket, done);
}

}  // extern "C"
