// spic_ctx.h -- the library context behind the opaque spic_ctx handle.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <string>

#include "spic_impl.h"

namespace spic {
struct BatchEngine;  // spic_batch.hip

// Host-side plan of one spic_batch_submit run (spic_batch.hip): its tiling,
// the engine-owned bytes it holds while admitted, the sort scratch its
// resident species need, and whether (and in batches of how many
// particles) it is streamed from host memory.
struct RunPlan {
    TileGeom tg{};
    size_t footprint = 0;  // particle slots (host-resident runs) + tile ranges + tick tables
    size_t sort_need = 0;  // shared sort scratch for its largest resident species
    bool host = false, streamed = false;
    int dtype = SPIC_F32;  // widest particle dtype of its species
    bool with_id = false;
    int64_t batch = 0;     // streamed: particles per batch
};

// Particles per streamed batch: the largest power-of-two fraction of
// max_batch whose two device slots, batch sort scratch and per-batch tile
// ranges fit `budget` (0 = no limit: max_batch itself); 0 when even 1024
// particles do not fit.
int64_t stream_batch_size(uint64_t budget, int64_t max_batch, int dtype, bool with_id, const TileGeom &tg,
                          const int64_t *n, int nsp);

// Device address of spic_mover_noalloc's fixed scratch on `device` (which
// must be current), looked up once per device (spic_noalloc.hip); NULL with
// *err set when the lookup fails.
void *noalloc_scratch(int device, hipError_t *err);
}

struct spic_ctx_s {
    struct Scratch {
        void *ptr = nullptr;
        size_t bytes = 0;
    };

    int device = 0;        // -1: host-only context (validation only)
    size_t lds_max = 160 * 1024;  // LDS bytes one workgroup may use (gfx950: 160 KiB; queried on a device)
    uint64_t budget = 0;   // 0 = unlimited
    std::atomic<uint64_t> used{0};  // bytes of library scratch currently allocated (read by the engine)
    std::string err;
    std::mutex mu;         // serialises the ABI calls on one ctx
    std::map<std::string, int64_t> options;
    std::map<std::string, Scratch> scratch;
    std::unique_ptr<spic::BatchEngine> batch;

    // Sort layout of a species, keyed by its x array, count, dtype and
    // grid: the tile geometry and the per-tile particle ranges (a scratch
    // slot) written by the last sort.  The tiled path uses them; they only
    // steer work to workgroups, so a stale layout is still correct.
    struct Layout {
        spic::TileGeom tg;
        std::string slot;
    };
    std::map<std::string, Layout> layouts;
    std::string layout_key(const spic_grid &g, const spic_species &s) const;
    spic::TileGeom tile_geom(const spic_grid &g, int dtype) const;

    spic_ctx_s();
    ~spic_ctx_s();

    int fail(int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
    int hip(hipError_t e, const char *what);
    int host_only();

    int check_grid(const spic_grid *g);
    int check_params(const spic_params *p);
    int check_fields(const spic_fields *f);
    int check_species(const spic_species *sp, int32_t nsp, bool allow_host);
    int check_moments(const spic_moment_array *m, const spic_species *sp, int32_t nsp);
    int check_combo(const spic_fields *f, const spic_species *sp, int32_t nsp);

    // scratch owned by the library, within the budget; `tag` names a slot
    // that is grown on demand and reused across calls
    int reserve(const char *tag, size_t bytes, void **out);
    void release_all();

    int64_t opt(const char *k, int64_t dflt) const;
    spic::LaunchCfg launch_cfg() const;

    // operations (validated arguments, device already current)
    int mover(const spic_grid &g, const spic_params &p, const spic_fields &f, spic_species *sp, int32_t nsp,
              spic_moment_array *mom, hipStream_t s);
    int moments(const spic_grid &g, const spic_species *sp, int32_t nsp, spic_moment_array *mom, bool accumulate,
                hipStream_t s);
    int sort(const spic_grid &g, spic_species *sp, int32_t nsp, hipStream_t s);
    // spic_mover_noalloc (spic_noalloc.hip): the sizes (host only), then the step
    int noalloc_check(const spic_grid &g, const spic_species *sp, int32_t nsp, const spic_moment_array *mom);
    int mover_noalloc(const spic_grid &g, const spic_params &p, const spic_fields &f, spic_species *sp,
                      int32_t nsp, spic_moment_array *mom, hipStream_t s);
    // the field solve (spic_field.hip)
    int check_field(const spic_grid *g, const spic_field_params *fp, const spic_em_state *em,
                    const spic_moment_array *mom, const double *qom, int32_t nsp);
    int field_apply(const spic_grid &g, const spic_field_params &fp, const spic_em_state &em,
                    const spic_moment_array *mom, const double *qom, int32_t nsp, const double *x, double *y,
                    hipStream_t s);
    int field_cycle(const spic_grid &g, const spic_field_params &fp, spic_em_state &em,
                    const spic_moment_array *mom, const double *qom, int32_t nsp, spic_field_stats *stats,
                    hipStream_t s);
    int sort_prepare(const spic_grid &g, const spic_species *sp, int32_t nsp, size_t &need);
    int sort_one(const spic_grid &g, const spic_species &sp, const spic::TileGeom &tg, size_t need, hipStream_t s,
                 uint32_t **toff_out, spic::SpeciesWork *sorted_out);
    // the plan of run r (validated), or an error (SPIC_E_BUDGET when it
    // cannot fit the budget even streamed); makes no HIP call
    int plan_run(const spic_run &R, int r, spic::RunPlan &p);
    int batch_submit(const spic_run *runs, int32_t nruns, uint64_t *tickets);
    int wait(uint64_t ticket, double *secs);
    int poll(uint64_t ticket, int32_t *done);
    void shutdown();
};
