// spic_exec.hip -- host dispatch of one fused step, the deposit-only pass
// and the sort, on validated arguments.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <string>

#include "spic_ctx.h"
#include "spic_impl.h"

using namespace spic;


static SpeciesWork work_of(const spic_species &s, const spic_moment_array *m) {
    SpeciesWork w;
    w.dtype = s.dtype;
    w.n = s.n;
    w.qom = s.qom;
    w.a[0] = s.x; w.a[1] = s.y; w.a[2] = s.z;
    w.a[3] = s.u; w.a[4] = s.v; w.a[5] = s.w; w.a[6] = s.q;
    w.id = s.id;
    w.mom = m ? m->m : nullptr;
    w.acc_dtype = m ? m->acc_dtype : SPIC_F64;
    return w;
}

std::string spic_ctx_s::layout_key(const spic_grid &g, const spic_species &s) const {
    char buf[160];
    snprintf(buf, sizeof buf, "%p/%lld/%d/%d.%d.%d", s.x, (long long)s.n, s.dtype, g.nx, g.ny, g.nz);
    return buf;
}

// The bank-preserving layout pays off for FP32 particles; FP64 particles
// keep the compact one (two workgroups per CU for the one-kernel variants)
// unless bank_align is set.  Full rows for variants 2 and 3 (the mover's
// corner cache and the deposit's lane sums want lane c on cell c); the
// LDS-atomic variants keep plain rank blocks, whose rows never hold one
// cell twice.
TileGeom spic_ctx_s::tile_geom(const spic_grid &g, int dtype) const {
    int var = (int)opt("tile_variant", -1);
    if (var < 0) var = auto_variant(dtype, SPIC_F64);
    const int dflt = dtype == SPIC_F64 ? 0 : 1;
    return make_tile_geom(g, (int)opt("tile_x", 4), (int)opt("tile_y", 4), (int)opt("tile_z", 4),
                          (int)opt("halo", 1), (int)opt("bank_align", dflt),
                          opt("sort_rows", variant_rows(var) ? 1 : 0) != 0);
}


int spic_ctx_s::mover(const spic_grid &g, const spic_params &p, const spic_fields &f, spic_species *sp,
                      int32_t nsp, spic_moment_array *mom, hipStream_t s) {
    const int64_t nn = (int64_t)g.nx * g.ny * g.nz;
    const LaunchCfg cfg = launch_cfg();
    const bool sort_now = p.sort_every > 0 && p.step % p.sort_every == 0;
    const bool generic_only = opt("path", 0) == 1;
    size_t sort_need = 0;
    if (sort_now) {
        int rc = sort_prepare(g, sp, nsp, sort_need);
        if (rc) return rc;
    }
    for (int i = 0; i < nsp; ++i) {
        SpeciesWork w = work_of(sp[i], mom ? &mom[i] : nullptr);
        if (w.mom) {
            int rc = hip(launch_fill(w.mom, w.acc_dtype, 10 * nn, s), "zero moments");
            if (rc) return rc;
        }
        // the tiled kernel runs for a sorted species whose region fits in LDS;
        // a variant whose extra LDS does not fit falls back to variant 0
        LaunchCfg tcfg = resolve_cfg(cfg, w.dtype, w.mom ? w.acc_dtype : SPIC_F64);
        auto tiled_ok = [&](const TileGeom &tg) {
            // compensated FP32 moments take the unsorted path (global atomics)
            if (generic_only || !tiled_fits(w.n, w.dtype) || (w.mom && w.acc_dtype == SPIC_F32C)) return false;
            if (tiled_lds_bytes(tg, w.dtype, w.acc_dtype, tcfg.variant, tcfg.tile_block) > lds_max) tcfg.variant = 0;
            return tiled_lds_bytes(tg, w.dtype, w.acc_dtype, tcfg.variant, tcfg.tile_block) <= lds_max;
        };
        int rc;
        if (sort_now) {
            // sort this species; the tiled kernel then reads the reordered
            // copy directly instead of it being copied back first
            const TileGeom tg_now = tile_geom(g, sp[i].dtype);
            const bool tiled = tiled_ok(tg_now);
            uint32_t *toff = nullptr;
            SpeciesWork sorted;
            if ((rc = sort_one(g, sp[i], tg_now, sort_need, s, &toff, tiled ? &sorted : nullptr))) return rc;
            if (tiled) {
                sorted.mom = w.mom;
                sorted.acc_dtype = w.acc_dtype;
                rc = hip(launch_fused_tiled(g, p, f, sorted, tg_now, toff, tcfg, s), "fused mover (tiled)");
            } else {
                rc = hip(launch_fused_generic(g, p, f, w, cfg, s), "fused mover");
            }
            if (rc) return rc;
            continue;
        }
        const Layout *lay = nullptr;
        auto it = layouts.find(layout_key(g, sp[i]));
        if (it != layouts.end() && tiled_ok(it->second.tg)) lay = &it->second;
        if (lay) {
            void *toff = nullptr;
            if ((rc = reserve(lay->slot.c_str(), (size_t)(lay->tg.ntiles + 1) * 4, &toff))) return rc;
            rc = hip(launch_fused_tiled(g, p, f, w, lay->tg, (const uint32_t *)toff, tcfg, s), "fused mover (tiled)");
        } else {
            rc = hip(launch_fused_generic(g, p, f, w, cfg, s), "fused mover");
        }
        if (rc) return rc;
    }
    return SPIC_OK;
}

int spic_ctx_s::moments(const spic_grid &g, const spic_species *sp, int32_t nsp, spic_moment_array *mom,
                        bool accumulate, hipStream_t s) {
    const int64_t nn = (int64_t)g.nx * g.ny * g.nz;
    const LaunchCfg cfg = launch_cfg();
    for (int i = 0; i < nsp; ++i) {
        SpeciesWork w = work_of(sp[i], &mom[i]);
        int rc;
        if (!accumulate && (rc = hip(launch_fill(w.mom, w.acc_dtype, 10 * nn, s), "zero moments"))) return rc;
        if ((rc = hip(launch_deposit_generic(g, w, cfg, s), "deposit"))) return rc;
    }
    return SPIC_OK;
}

// Checks the tile shape and sizes the scratch the next sort of every
// species needs (each species gets the tiling of its dtype).
int spic_ctx_s::sort_prepare(const spic_grid &g, const spic_species *sp, int32_t nsp, size_t &need) {
    const TileGeom tg = tile_geom(g, SPIC_F32);
    if (tg.cells < 1 || tg.cells > 64 || tg.halo < 0 || tg.halo > 8)
        return fail(SPIC_E_ARG, "tile shape %dx%dx%d (halo %d): a tile holds 1..64 cells, halo 0..8", tg.tx, tg.ty,
                    tg.tz, tg.halo);
    need = 0;
    for (int i = 0; i < nsp; ++i) {
        if (sp[i].n >= ((int64_t)1 << 31)) return fail(SPIC_E_UNSUPPORTED, "species %d: sort needs n < 2^31", i);
        need = std::max(need, sort_scratch_bytes(sp[i].n, sp[i].dtype, sp[i].id != nullptr, tile_geom(g, sp[i].dtype)));
    }
    return SPIC_OK;
}

// Sort one species and record its layout.  With sorted_out the reordered
// particles stay in the shared scratch for the kernel launched next.
int spic_ctx_s::sort_one(const spic_grid &g, const spic_species &sp, const TileGeom &tg, size_t need,
                         hipStream_t s, uint32_t **toff_out, SpeciesWork *sorted_out) {
    const std::string key = layout_key(g, sp);
    const std::string slot = "tileoff:" + key;
    void *toff = nullptr, *scr = nullptr;
    int rc;
    if ((rc = reserve(slot.c_str(), (size_t)(tg.ntiles + 1) * 4, &toff))) return rc;
    if ((rc = reserve("sort", need, &scr))) return rc;
    SpeciesWork w = work_of(sp, nullptr);
    auto it = layouts.find(key);
    const bool prev = opt("sort_ordered", 1) && it != layouts.end() && same_tiling(it->second.tg, tg);
    if ((rc = hip(launch_sort(g, w, tg, scr, (uint32_t *)toff, prev, s, sorted_out), "sort"))) return rc;
    layouts[key] = Layout{tg, slot};
    if (toff_out) *toff_out = (uint32_t *)toff;
    return SPIC_OK;
}

int spic_ctx_s::sort(const spic_grid &g, spic_species *sp, int32_t nsp, hipStream_t s) {
    size_t need = 0;
    int rc = sort_prepare(g, sp, nsp, need);
    if (rc) return rc;
    for (int i = 0; i < nsp; ++i)
        if ((rc = sort_one(g, sp[i], tile_geom(g, sp[i].dtype), need, s, nullptr, nullptr))) return rc;
    return SPIC_OK;
}
