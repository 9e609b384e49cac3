// spic_exec.hip -- host dispatch of one fused step, the deposit-only pass
// and the sort, on validated arguments.
#include <hip/hip_runtime.h>

#include "spic_ctx.h"
#include "spic_impl.h"

using namespace spic;

namespace spic {
struct BatchEngine {};
}

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

int spic_ctx_s::mover(const spic_grid &g, const spic_params &p, const spic_fields &f, spic_species *sp,
                      int32_t nsp, spic_moment_array *mom, hipStream_t s) {
    const int64_t nn = (int64_t)g.nx * g.ny * g.nz;
    const LaunchCfg cfg = launch_cfg();
    if (p.sort_every > 0 && p.step % p.sort_every == 0) {
        int rc = sort(g, sp, nsp, s);
        if (rc) return rc;
    }
    for (int i = 0; i < nsp; ++i) {
        SpeciesWork w = work_of(sp[i], mom ? &mom[i] : nullptr);
        if (w.mom) {
            int rc = hip(launch_fill(w.mom, w.acc_dtype, 10 * nn, s), "zero moments");
            if (rc) return rc;
        }
        int rc = hip(launch_fused_generic(g, p, f, w, cfg, s), "fused mover");
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

int spic_ctx_s::sort(const spic_grid &, spic_species *, int32_t, hipStream_t) {
    return fail(SPIC_E_UNSUPPORTED, "sort is not built yet");
}

int spic_ctx_s::batch_submit(const spic_run *, int32_t, uint64_t *) {
    return fail(SPIC_E_UNSUPPORTED, "batch_submit is not built yet");
}

int spic_ctx_s::wait(uint64_t, double *) { return fail(SPIC_E_STATE, "unknown ticket"); }

int spic_ctx_s::poll(uint64_t, int32_t *) { return fail(SPIC_E_STATE, "unknown ticket"); }

void spic_ctx_s::shutdown() {}

spic_ctx_s::spic_ctx_s() {}
spic_ctx_s::~spic_ctx_s() {}
