// spic_batch.hip -- the batch engine behind spic_batch_submit: many
// independent multi-step runs on one GPU (Sec. III-B, particle batching).
//
// A scheduler thread owns three streams (compute, host->device,
// device->host) and advances all resident runs together in "ticks": one
// tick is one fused step of every active run, executed as one work-list
// launch (two for the split variants: mover, then deposit) over the (run,
// species, tile) items of all of them (plus the cell sort of the runs whose cadence is due, and one batched
// zeroing of their moments).  While the set of active runs does not change
// and no sort is due, the tick is captured once as a hipGraph and replayed.
//
// Continuous batching.  Runs submitted while others are executing wait in
// a queue and are admitted at the next tick boundary as soon as their HBM
// footprint fits the budget left by the active runs; runs that finish are
// retired (results copied back, memory released) and their tickets
// signalled at the tick they complete, so long and short runs overlap on
// the device.
//
// Host-resident species (pinned host memory) are copied into engine-owned
// device slots at admission and back at retirement.  A run whose particles
// cannot fit the budget at all is streamed instead: its species are cut
// into batches that flow through two device slots, the upload of the next
// batch and the download of the previous one overlapping the kernel on the
// current one (Sec. III-B: overlap of transfers with computation, and
// computation on data larger than device memory).
//
// Every engine run is sorted by cell at its first step (and every
// sort_every steps after), so its particle arrays are permuted; ids, when
// given, are permuted alongside.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "spic_ctx.h"
#include "spic_impl.h"

namespace spic {

namespace {

size_t elem(int dtype) { return dtype == SPIC_F64 ? 8 : 4; }

// Bytes of the 7 particle arrays (+ ids) of n particles, 256-aligned each.
size_t species_bytes(int64_t n, int dtype, bool with_id) {
    const size_t a = ((size_t)n * elem(dtype) + 255) & ~(size_t)255;
    return 7 * a + (with_id ? (((size_t)n * 8 + 255) & ~(size_t)255) : 0);
}

// Carve the 7 arrays (+ id) of n particles out of one allocation.
void carve_species(void *base, int64_t n, int dtype, bool with_id, spic_species &d) {
    char *p = (char *)base;
    const size_t a = ((size_t)n * elem(dtype) + 255) & ~(size_t)255;
    void **arr[7] = {&d.x, &d.y, &d.z, &d.u, &d.v, &d.w, &d.q};
    for (int i = 0; i < 7; ++i) {
        *arr[i] = p;
        p += a;
    }
    d.id = with_id ? (int64_t *)p : nullptr;
}

SpeciesWork work_of(const spic_species &s, const spic_moment_array *m) {
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

}  // namespace

struct SpeciesSlot {
    spic_species user{};   // the caller's descriptor
    spic_species dev{};    // device-resident view used by the kernels
    void *buf = nullptr;   // engine-owned device copy (host-resident species)
    size_t bytes = 0;
    uint32_t *tile_off = nullptr;
    int combo = -1;
};

struct RunState {
    uint64_t ticket = 0;
    spic_grid grid{};
    spic_params params{};
    spic_fields fields{};
    std::vector<SpeciesSlot> sp;
    std::vector<spic_moment_array> mom;
    int nsteps = 0, done_steps = 0;
    bool host = false, streamed = false;
    size_t footprint = 0;  // engine-owned bytes while admitted (see RunPlan)
    size_t sort_need = 0;  // shared sort scratch it needs
    int64_t batch = 0;     // streamed: particles per batch
    TileGeom tg{};
    hipEvent_t ev_start = nullptr, ev_done = nullptr;
    enum Phase { QUEUED, ACTIVE, RETIRING, DONE } phase = QUEUED;
    int status = SPIC_OK;
    std::string err;
    double secs = 0;
    std::chrono::steady_clock::time_point submitted;

    // particle-steps still to do, and (job, tile) items of one tick
    double remaining_work() const {
        double n = 0;
        for (auto &sl : sp) n += (double)sl.user.n;
        return n * (double)(nsteps - done_steps);
    }
    int64_t tick_items() const {
        int64_t k = 0;
        for (auto &sl : sp) k += sl.user.n > 0 ? tg.ntiles : 0;
        return k;
    }
};

struct BatchEngine {
    spic_ctx_s *ctx;
    int device;
    hipStream_t cs = nullptr, h2d = nullptr, d2h = nullptr;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<RunState>> queued;
    std::vector<std::shared_ptr<RunState>> active, retiring;
    std::map<uint64_t, std::shared_ptr<RunState>> all;
    uint64_t next_ticket = 1;
    uint64_t used = 0;   // engine-owned bytes of admitted runs
    bool stop = false;

    // scratch owned by the scheduler thread
    void *sort_scr = nullptr;
    size_t sort_bytes = 0;
    void *dtab = nullptr;        // device tables of the current tick
    size_t dtab_bytes = 0;
    void *htab = nullptr;        // pinned host staging of the tables
    size_t htab_bytes = 0;
    hipEvent_t tab_ev = nullptr; // the last table upload has been read
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<uint64_t> graph_key;

    // tuning, read from the ctx options when the engine starts
    int tile_block = -1, variant = -1, use_graph = 1, max_groups = 0, fixed_geo = 1, sort_ordered = 1;
    int64_t tick_items = 4096;  // 0: every active run steps at every tick
    double srpt_aging = 1e10;   // particle-steps of credit per second waited
    int64_t batch_particles = (int64_t)1 << 26;
    LaunchCfg lcfg;

    explicit BatchEngine(spic_ctx_s *c) : ctx(c), device(c->device) {}

    int start() {
        hipError_t e;
        if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipStreamCreateWithFlags(&h2d, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipStreamCreateWithFlags(&d2h, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&tab_ev, hipEventDisableTiming)) != hipSuccess)
            return ctx->hip(e, "batch engine streams");
        th = std::thread([this] { loop(); });
        return SPIC_OK;
    }

    void shutdown() {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv_work.notify_all();
        if (th.joinable()) th.join();
        (void)hipDeviceSynchronize();
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
        for (auto &kv : all) release(*kv.second);
        if (sort_scr) (void)hipFree(sort_scr);
        if (dtab) (void)hipFree(dtab);
        if (htab) (void)hipHostFree(htab);
        if (tab_ev) (void)hipEventDestroy(tab_ev);
        if (cs) (void)hipStreamDestroy(cs);
        if (h2d) (void)hipStreamDestroy(h2d);
        if (d2h) (void)hipStreamDestroy(d2h);
        cs = h2d = d2h = nullptr;
    }

    // ------------------------------------------------------------ submit

    // Called under ctx->mu with validated runs.
    int submit(const spic_run *runs, int32_t nruns, uint64_t *tickets) {
        std::vector<std::shared_ptr<RunState>> made;
        for (int r = 0; r < nruns; ++r) {
            const spic_run &R = runs[r];
            RunPlan plan;
            int rc = ctx->plan_run(R, r, plan);
            if (rc) return rc;
            auto st = std::make_shared<RunState>();
            st->grid = R.grid;
            st->params = R.params;
            st->fields = R.fields;
            st->nsteps = R.nsteps;
            st->tg = plan.tg;
            st->host = plan.host;
            st->streamed = plan.streamed;
            st->footprint = plan.footprint;
            st->sort_need = plan.sort_need;
            st->batch = plan.batch;
            for (int s = 0; s < R.nspecies; ++s) {
                SpeciesSlot sl;
                sl.user = R.species[s];
                sl.combo = job_combo(sl.user.dtype, R.fields.dtype, R.moments ? R.moments[s].acc_dtype : SPIC_F64);
                st->sp.push_back(sl);
            }
            if (R.moments) st->mom.assign(R.moments, R.moments + R.nspecies);
            made.push_back(st);
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            for (size_t i = 0; i < made.size(); ++i) {
                made[i]->ticket = next_ticket++;
                made[i]->submitted = std::chrono::steady_clock::now();
                tickets[i] = made[i]->ticket;
                all[made[i]->ticket] = made[i];
                queued.push_back(made[i]);
            }
        }
        cv_work.notify_all();
        return SPIC_OK;
    }

    int wait(uint64_t ticket, double *secs) {
        std::unique_lock<std::mutex> lk(mu);
        auto it = all.find(ticket);
        if (it == all.end()) return SPIC_E_STATE;
        auto st = it->second;
        cv_done.wait(lk, [&] { return st->phase == RunState::DONE; });
        if (secs) *secs = st->secs;
        if (st->status != SPIC_OK) {
            ctx->err = st->err;
            return st->status;
        }
        return SPIC_OK;
    }

    int poll(uint64_t ticket, int32_t *done) {
        std::lock_guard<std::mutex> lk(mu);
        auto it = all.find(ticket);
        if (it == all.end()) return SPIC_E_STATE;
        *done = it->second->phase == RunState::DONE ? 1 : 0;
        return SPIC_OK;
    }

    // --------------------------------------------------------- scheduler

    void fail_run(RunState &r, hipError_t e, const char *what) {
        if (r.status == SPIC_OK) {
            r.status = SPIC_E_HIP;
            r.err = std::string(what) + ": " + hipGetErrorString(e);
        }
    }

    void release(RunState &r) {
        for (auto &sl : r.sp) {
            if (sl.buf) (void)hipFree(sl.buf);
            if (sl.tile_off) (void)hipFree(sl.tile_off);
            sl.buf = nullptr;
            sl.tile_off = nullptr;
        }
        if (r.ev_start) (void)hipEventDestroy(r.ev_start);
        if (r.ev_done) (void)hipEventDestroy(r.ev_done);
        r.ev_start = r.ev_done = nullptr;
    }

    // Engine-owned bytes (admitted runs and the shared sort scratch) plus
    // the ctx's own scratch stay within the ctx's budget.
    bool fits(const RunState &r) const {
        if (!ctx->budget) return true;
        const uint64_t sort_after = std::max<uint64_t>(sort_bytes, r.sort_need);
        return used + r.footprint + sort_after + ctx->used.load() <= ctx->budget;
    }

    // Allocate and upload a resident run (scheduler thread, engine lock held).
    void admit(RunState &r) {
        hipError_t e;
        if ((e = hipEventCreate(&r.ev_start)) != hipSuccess || (e = hipEventCreate(&r.ev_done)) != hipSuccess) {
            fail_run(r, e, "events");
            return;
        }
        bool uploads = false;
        for (auto &sl : r.sp) {
            sl.dev = sl.user;
            sl.dev.host_resident = 0;
            if ((e = hipMalloc(&sl.tile_off, (size_t)(r.tg.ntiles + 1) * 4)) != hipSuccess) {
                fail_run(r, e, "hipMalloc(tile ranges)");
                return;
            }
            if (!sl.user.host_resident || sl.user.n == 0) continue;
            sl.bytes = species_bytes(sl.user.n, sl.user.dtype, sl.user.id != nullptr);
            if ((e = hipMalloc(&sl.buf, sl.bytes)) != hipSuccess) {
                fail_run(r, e, "hipMalloc(run particles)");
                return;
            }
            carve_species(sl.buf, sl.user.n, sl.user.dtype, sl.user.id != nullptr, sl.dev);
            const size_t b = (size_t)sl.user.n * elem(sl.user.dtype);
            const void *src[7] = {sl.user.x, sl.user.y, sl.user.z, sl.user.u, sl.user.v, sl.user.w, sl.user.q};
            void *dst[7] = {sl.dev.x, sl.dev.y, sl.dev.z, sl.dev.u, sl.dev.v, sl.dev.w, sl.dev.q};
            for (int i = 0; i < 7; ++i)
                if ((e = hipMemcpyAsync(dst[i], src[i], b, hipMemcpyHostToDevice, h2d)) != hipSuccess)
                    fail_run(r, e, "upload");
            if (sl.user.id &&
                (e = hipMemcpyAsync(sl.dev.id, sl.user.id, (size_t)sl.user.n * 8, hipMemcpyHostToDevice, h2d)) !=
                    hipSuccess)
                fail_run(r, e, "upload ids");
            uploads = true;
        }
        if (uploads) {
            hipEvent_t up;
            if (hipEventCreateWithFlags(&up, hipEventDisableTiming) == hipSuccess) {
                (void)hipEventRecord(up, h2d);
                (void)hipStreamWaitEvent(cs, up, 0);
                (void)hipEventDestroy(up);
            }
        }
        used += r.footprint;
        (void)hipEventRecord(r.ev_start, cs);
        r.phase = RunState::ACTIVE;
    }

    void retire(RunState &r) {
        hipError_t e;
        bool downloads = false;
        for (auto &sl : r.sp) {
            if (!sl.buf) continue;
            if (!downloads) {
                hipEvent_t ready;
                if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) == hipSuccess) {
                    (void)hipEventRecord(ready, cs);
                    (void)hipStreamWaitEvent(d2h, ready, 0);
                    (void)hipEventDestroy(ready);
                }
                downloads = true;
            }
            const size_t b = (size_t)sl.user.n * elem(sl.user.dtype);
            const void *src[7] = {sl.dev.x, sl.dev.y, sl.dev.z, sl.dev.u, sl.dev.v, sl.dev.w, sl.dev.q};
            void *dst[7] = {sl.user.x, sl.user.y, sl.user.z, sl.user.u, sl.user.v, sl.user.w, sl.user.q};
            for (int i = 0; i < 7; ++i)
                if ((e = hipMemcpyAsync(dst[i], src[i], b, hipMemcpyDeviceToHost, d2h)) != hipSuccess)
                    fail_run(r, e, "download");
            if (sl.user.id &&
                (e = hipMemcpyAsync(sl.user.id, sl.dev.id, (size_t)sl.user.n * 8, hipMemcpyDeviceToHost, d2h)) !=
                    hipSuccess)
                fail_run(r, e, "download ids");
        }
        (void)hipEventRecord(r.ev_done, downloads ? d2h : cs);
        r.phase = RunState::RETIRING;
    }

    // Grow the shared sort scratch to `need` bytes.  On failure no scratch
    // is held (sort_scr == nullptr) and the error is returned: the caller
    // fails the run before launching anything on it.
    hipError_t ensure_sort_scratch(size_t need) {
        if (need <= sort_bytes && sort_scr) return hipSuccess;
        (void)hipStreamSynchronize(cs);
        if (sort_scr) (void)hipFree(sort_scr);
        sort_scr = nullptr;
        sort_bytes = 0;
        const hipError_t e = hipMalloc(&sort_scr, need ? need : 256);
        if (e != hipSuccess) {
            sort_scr = nullptr;
            return e;
        }
        sort_bytes = need;
        return hipSuccess;
    }

    void ensure_tables(size_t need) {
        if (need > dtab_bytes) {
            (void)hipStreamSynchronize(cs);
            if (dtab) (void)hipFree(dtab);
            dtab = nullptr;
            dtab_bytes = 0;
            if (hipMalloc(&dtab, need) == hipSuccess) dtab_bytes = need;
        }
        if (need > htab_bytes) {
            (void)hipEventSynchronize(tab_ev);
            if (htab) (void)hipHostFree(htab);
            htab = nullptr;
            htab_bytes = 0;
            if (hipHostMalloc(&htab, need, hipHostMallocDefault) == hipSuccess) htab_bytes = need;
        }
    }

    // One fused step of every active run.
    void tick(std::vector<std::shared_ptr<RunState>> &act) {
        // 1. sorts that are due (first step, then every sort_every)
        bool sorted_now = false;
        for (auto &rp : act) {
            RunState &r = *rp;
            const int64_t step = r.params.step + r.done_steps;
            const bool due = r.done_steps == 0 || (r.params.sort_every > 0 && step % r.params.sort_every == 0);
            if (!due) continue;
            for (auto &sl : r.sp) {
                if (sl.dev.n == 0) {
                    (void)launch_zero32(sl.tile_off, r.tg.ntiles + 1, cs);
                    continue;
                }
                hipError_t e = ensure_sort_scratch(sort_scratch_bytes(sl.dev.n, sl.dev.dtype, sl.dev.id != nullptr, r.tg));
                if (e != hipSuccess) {
                    fail_run(r, e, "sort scratch");
                    break;
                }
                e = launch_sort(r.grid, work_of(sl.dev, nullptr), r.tg, sort_scr, sl.tile_off,
                                sort_ordered && r.done_steps > 0, cs);
                if (e != hipSuccess) {
                    fail_run(r, e, "sort");
                    break;
                }
            }
            sorted_now = true;
        }
        // a run whose sort could not run is retired without a kernel touching
        // its (possibly never written) tile ranges
        {
            std::vector<std::shared_ptr<RunState>> ok, bad;
            for (auto &rp : act) (rp->status == SPIC_OK ? ok : bad).push_back(rp);
            if (!bad.empty()) {
                advance(bad);
                act.swap(ok);
                if (act.empty()) return;
            }
        }
        // 2. tables: moment arrays to zero, jobs and items per combo
        std::vector<uint64_t> key;
        for (auto &rp : act) key.push_back(rp->ticket);
        const bool same = !sorted_now && gexec && key == graph_key;
        if (same) {
            hipError_t e = hipGraphLaunch(gexec, cs);
            if (e == hipSuccess) return advance(act);
            (void)hipGraphExecDestroy(gexec);
            gexec = nullptr;
        }
        struct Combo {
            std::vector<unsigned char> jobs;
            std::vector<uint2> items;
            TileGeom tg{};             // the job tiling with the largest region
            int var = 0, var_cfg = -1, block = 512;
            int dtype = SPIC_F32, acc = SPIC_F64;
        };
        std::map<int, Combo> combos;
        std::vector<void *> mptr[2];
        std::vector<int64_t> mcnt[2];
        for (auto &rp : act) {
            RunState &r = *rp;
            const int64_t nn = (int64_t)r.grid.nx * r.grid.ny * r.grid.nz;
            for (size_t s = 0; s < r.sp.size(); ++s) {
                SpeciesSlot &sl = r.sp[s];
                const spic_moment_array *m = r.mom.empty() ? nullptr : &r.mom[s];
                if (m) {
                    const int which = m->acc_dtype == SPIC_F64 ? 0 : 1;
                    mptr[which].push_back(m->m);
                    mcnt[which].push_back(10 * nn);
                }
                if (sl.dev.n == 0) continue;
                // launch key: precision combination, +8 for the compile-time default tiling
                Combo &c = combos[sl.combo + (fixed_geo && geo_is_default(r.tg) ? 8 : 0)];
                const int acc = m ? m->acc_dtype : SPIC_F64;
                if (c.var_cfg < 0) {  // variant and block of this precision combination
                    LaunchCfg rc = lcfg;
                    rc.variant = variant;
                    rc.tile_block = tile_block;
                    rc = resolve_cfg(rc, sl.dev.dtype, acc);
                    c.var_cfg = rc.variant;
                    c.dtype = sl.dev.dtype;
                    c.acc = acc;
                    c.tg = r.tg;
                    c.block = rc.tile_block;
                }
                const size_t jb = tile_job_bytes(sl.combo);
                const uint32_t jidx = (uint32_t)(c.jobs.size() / jb);
                c.jobs.resize(c.jobs.size() + jb);
                spic_params prm = r.params;
                write_tile_job(sl.combo, c.jobs.data() + jidx * jb, r.grid, prm, r.fields, work_of(sl.dev, m), r.tg,
                               sl.tile_off);
                for (int t = 0; t < r.tg.ntiles; ++t) c.items.push_back(make_uint2(jidx, (uint32_t)t));
                if (r.tg.rnp > c.tg.rnp || r.tg.rx * r.tg.ry * r.tg.rz > c.tg.rx * c.tg.ry * c.tg.rz) c.tg = r.tg;
            }
        }
        // layout of the device table: [ptrs f64][cnt f64][ptrs f32][cnt f32][counters x16] then per launch key jobs, items
        size_t off = 0;
        auto reserve = [&](size_t b) { size_t o = off; off += (b + 255) & ~(size_t)255; return o; };
        const size_t o_p0 = reserve(mptr[0].size() * 8), o_c0 = reserve(mcnt[0].size() * 8);
        const size_t o_p1 = reserve(mptr[1].size() * 8), o_c1 = reserve(mcnt[1].size() * 8);
        const size_t o_ctr = reserve(32 * 4);  // two per launch key
        std::map<int, std::pair<size_t, size_t>> co;
        for (auto &kv : combos) {
            const size_t oj = reserve(kv.second.jobs.size());
            const size_t oi = reserve(kv.second.items.size() * sizeof(uint2));
            co[kv.first] = {oj, oi};
        }
        // the previous tick's tables may still be in use by a replayed graph
        if (gexec) {
            (void)hipStreamSynchronize(cs);
            (void)hipGraphExecDestroy(gexec);
            gexec = nullptr;
        }
        ensure_tables(off);
        if (!dtab || !htab) {
            for (auto &rp : act) fail_run(*rp, hipErrorOutOfMemory, "tick tables");
            return advance(act);
        }
        (void)hipEventSynchronize(tab_ev);
        char *h = (char *)htab;
        memcpy(h + o_p0, mptr[0].data(), mptr[0].size() * 8);
        memcpy(h + o_c0, mcnt[0].data(), mcnt[0].size() * 8);
        memcpy(h + o_p1, mptr[1].data(), mptr[1].size() * 8);
        memcpy(h + o_c1, mcnt[1].data(), mcnt[1].size() * 8);
        memset(h + o_ctr, 0, 32 * 4);
        for (auto &kv : combos) {
            memcpy(h + co[kv.first].first, kv.second.jobs.data(), kv.second.jobs.size());
            memcpy(h + co[kv.first].second, kv.second.items.data(), kv.second.items.size() * sizeof(uint2));
        }
        (void)hipMemcpyAsync(dtab, htab, off, hipMemcpyHostToDevice, cs);
        (void)hipEventRecord(tab_ev, cs);
        char *d = (char *)dtab;

        // 3. the step itself (captured as a graph when enabled); launch sizes
        // are settled before the capture starts
        std::map<int, WorklistGroups> groups;
        for (auto &kv : combos) {
            // a variant whose LDS does not fit falls back to variant 0
            Combo &c = kv.second;
            c.var = tiled_lds_bytes(c.tg, c.dtype, c.acc, c.var_cfg, c.block) <= ctx->lds_max ? c.var_cfg : 0;
            groups[kv.first] = worklist_groups(kv.first & 7, kv.first >= 8, c.var, c.tg, c.block,
                                               (int)c.items.size(), max_groups);
        }
        bool capturing = false;
        if (use_graph && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) capturing = true;
        hipError_t e = hipSuccess;
        if (!mptr[0].empty())
            e = launch_fill_many((void *const *)(d + o_p0), (const int64_t *)(d + o_c0), (int)mptr[0].size(), 8, cs);
        if (e == hipSuccess && !mptr[1].empty())
            e = launch_fill_many((void *const *)(d + o_p1), (const int64_t *)(d + o_c1), (int)mptr[1].size(), 4, cs);
        if (e == hipSuccess) e = launch_zero32(d + o_ctr, 32, cs);
        int ci = 0;
        for (auto &kv : combos) {
            if (e != hipSuccess) break;
            e = launch_worklist(kv.first & 7, kv.first >= 8, kv.second.var, d + co[kv.first].first,
                                (const uint2 *)(d + co[kv.first].second), (int)kv.second.items.size(),
                                (unsigned *)(d + o_ctr) + 2 * ci++, groups[kv.first], kv.second.block, cs);
        }
        if (capturing) {
            hipGraph_t g = nullptr;
            const hipError_t ce = hipStreamEndCapture(cs, &g);
            if (e == hipSuccess && ce == hipSuccess && g) {
                if (graph) (void)hipGraphDestroy(graph);
                graph = g;
                if (hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0) == hipSuccess &&
                    hipGraphLaunch(gexec, cs) == hipSuccess) {
                    graph_key = key;
                } else {
                    if (gexec) (void)hipGraphExecDestroy(gexec);
                    gexec = nullptr;
                    e = hipErrorUnknown;
                }
            } else {
                if (g) (void)hipGraphDestroy(g);
                if (e == hipSuccess) e = ce;
            }
        }
        if (e != hipSuccess)
            for (auto &rp : act) fail_run(*rp, e, "tick");
        advance(act);
    }

    void advance(std::vector<std::shared_ptr<RunState>> &act) {
        std::lock_guard<std::mutex> lk(mu);
        for (auto &rp : act) {
            rp->done_steps++;
            if (rp->done_steps >= rp->nsteps || rp->status != SPIC_OK) retire(*rp);
        }
        active.erase(std::remove_if(active.begin(), active.end(),
                                    [](const std::shared_ptr<RunState> &r) { return r->phase != RunState::ACTIVE; }),
                     active.end());
        for (auto &rp : act)
            if (rp->phase == RunState::RETIRING) retiring.push_back(rp);
    }

    void reap(bool block) {
        std::vector<std::shared_ptr<RunState>> done;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (auto &rp : retiring) {
                hipError_t q = block ? hipEventSynchronize(rp->ev_done) : hipEventQuery(rp->ev_done);
                if (q == hipErrorNotReady) continue;
                if (q != hipSuccess) fail_run(*rp, q, "run completion");
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, rp->ev_start, rp->ev_done) == hipSuccess) rp->secs = ms / 1e3;
                done.push_back(rp);
                block = false;
            }
        }
        if (done.empty()) return;
        for (auto &rp : done) release(*rp);
        {
            std::lock_guard<std::mutex> lk(mu);
            for (auto &rp : done) {
                used -= rp->footprint;
                rp->phase = RunState::DONE;
            }
            retiring.erase(std::remove_if(retiring.begin(), retiring.end(),
                                          [](const std::shared_ptr<RunState> &r) {
                                              return r->phase == RunState::DONE;
                                          }),
                           retiring.end());
        }
        cv_done.notify_all();
        cv_work.notify_all();
    }

    // Streamed run: batches of at most nb particles through two slots.
    void stream_run(RunState &r);

    // The runs the next tick steps: least remaining work first, until the
    // tick holds tick_items (job, tile) items -- enough to fill the GPU -- so
    // that short requests finish first instead of being slowed down by every
    // long run they share the GPU with.  Pure shortest-first starves a long
    // run for as long as shorter ones keep arriving, so each run's remaining
    // work is credited srpt_aging particle-steps per second since it was
    // submitted: with the credit rate near the engine's throughput, a run
    // that has waited about as long as it takes to serve alone overtakes any
    // newcomer.  Returned in ticket order, so an unchanged set replays its
    // graph.
    std::vector<std::shared_ptr<RunState>> pick(const std::vector<std::shared_ptr<RunState>> &all) const {
        if (tick_items <= 0 || all.size() <= 1) return all;
        const auto now = std::chrono::steady_clock::now();
        std::vector<std::pair<double, std::shared_ptr<RunState>>> v;
        v.reserve(all.size());
        for (auto &r : all) {
            const double waited = std::chrono::duration<double>(now - r->submitted).count();
            v.emplace_back(r->remaining_work() - srpt_aging * waited, r);
        }
        std::stable_sort(v.begin(), v.end(), [](const std::pair<double, std::shared_ptr<RunState>> &a,
                                                const std::pair<double, std::shared_ptr<RunState>> &b) {
            return a.first < b.first;
        });
        std::vector<std::shared_ptr<RunState>> out;
        int64_t items = 0;
        for (auto &e : v) {
            if (!out.empty() && items >= tick_items) break;
            out.push_back(e.second);
            items += e.second->tick_items();
        }
        std::sort(out.begin(), out.end(), [](const std::shared_ptr<RunState> &a, const std::shared_ptr<RunState> &b) {
            return a->ticket < b->ticket;
        });
        return out;
    }

    void loop() {
        (void)hipSetDevice(device);
        for (;;) {
            std::vector<std::shared_ptr<RunState>> act;
            std::shared_ptr<RunState> streamed;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait_for(lk, std::chrono::milliseconds(retiring.empty() ? 50 : 1), [&] {
                    return stop || !queued.empty() || !active.empty() || !retiring.empty();
                });
                if (stop && active.empty() && retiring.empty()) {
                    for (auto &q : queued) {
                        q->status = SPIC_E_STATE;
                        q->err = "context destroyed before the run started";
                        q->phase = RunState::DONE;
                    }
                    queued.clear();
                    cv_done.notify_all();
                    break;
                }
                // admission at the tick boundary: every queued run that fits
                for (auto it = queued.begin(); it != queued.end();) {
                    RunState &r = **it;
                    if (r.streamed) {
                        if (active.empty() && retiring.empty() && !streamed) {
                            streamed = *it;
                            it = queued.erase(it);
                        } else {
                            ++it;
                        }
                        continue;
                    }
                    if (!fits(r)) {
                        ++it;
                        continue;
                    }
                    admit(r);
                    if (r.status != SPIC_OK) {
                        (void)hipStreamSynchronize(cs);
                        release(r);
                        used -= std::min<uint64_t>(used, r.phase == RunState::ACTIVE ? r.footprint : 0);
                        r.phase = RunState::DONE;
                        cv_done.notify_all();
                    } else if (r.nsteps == 0) {
                        retire(r);  // nothing to step: round-trip the data and finish
                        retiring.push_back(*it);
                    } else {
                        active.push_back(*it);
                    }
                    it = queued.erase(it);
                }
                act = pick(active);
            }
            if (streamed) {
                stream_run(*streamed);
                std::lock_guard<std::mutex> lk(mu);
                streamed->phase = RunState::DONE;
                cv_done.notify_all();
                continue;
            }
            if (!act.empty()) tick(act);
            reap(act.empty());
        }
    }
};

// ----------------------------------------------------------- streaming

void BatchEngine::stream_run(RunState &r) {
    hipError_t e;
    int dt = SPIC_F32;
    bool with_id = false;
    for (auto &sl : r.sp) {
        if (sl.user.dtype == SPIC_F64) dt = SPIC_F64;
        with_id = with_id || sl.user.id;
    }
    const int64_t nb = r.batch;
    int64_t total_batches = 0;
    for (auto &sl : r.sp) total_batches += (sl.user.n + nb - 1) / nb;
    void *slot[2] = {nullptr, nullptr};
    void *tiles = nullptr;
    hipEvent_t loaded[2], computed[2], freed[2], t0, t1;
    for (int i = 0; i < 2; ++i) {
        (void)hipEventCreateWithFlags(&loaded[i], hipEventDisableTiming);
        (void)hipEventCreateWithFlags(&computed[i], hipEventDisableTiming);
        (void)hipEventCreateWithFlags(&freed[i], hipEventDisableTiming);
    }
    (void)hipEventCreate(&t0);
    (void)hipEventCreate(&t1);
    const size_t sb = species_bytes(nb, dt, with_id);
    if ((e = hipMalloc(&slot[0], sb)) != hipSuccess || (e = hipMalloc(&slot[1], sb)) != hipSuccess ||
        (e = hipMalloc(&tiles, (size_t)std::max<int64_t>(total_batches, 1) * (r.tg.ntiles + 1) * 4)) != hipSuccess) {
        fail_run(r, e, "streaming slots");
    } else if ((e = ensure_sort_scratch(sort_scratch_bytes(nb, dt, with_id, r.tg))) != hipSuccess) {
        fail_run(r, e, "sort scratch");
    } else {
        (void)hipEventRecord(t0, cs);
        int use = 0;  // which slot the next batch goes to
        for (int step = 0; step < r.nsteps && r.status == SPIC_OK; ++step) {
            spic_params prm = r.params;
            prm.step = r.params.step + step;
            const bool sort_due = step == 0 || (prm.sort_every > 0 && prm.step % prm.sort_every == 0);
            int64_t bidx = 0;
            for (size_t s = 0; s < r.sp.size(); ++s) {
                const SpeciesSlot &sl = r.sp[s];
                const spic_moment_array *m = r.mom.empty() ? nullptr : &r.mom[s];
                const int64_t nn = (int64_t)r.grid.nx * r.grid.ny * r.grid.nz;
                if (m && (e = launch_fill(m->m, m->acc_dtype, 10 * nn, cs)) != hipSuccess) fail_run(r, e, "zero");
                const size_t es = elem(sl.user.dtype);
                for (int64_t off = 0; off < sl.user.n; off += nb, ++bidx) {
                    const int64_t cnt = std::min<int64_t>(nb, sl.user.n - off);
                    const int k = use;
                    use ^= 1;
                    spic_species dv = sl.user;
                    dv.host_resident = 0;
                    dv.n = cnt;
                    carve_species(slot[k], nb, sl.user.dtype, sl.user.id != nullptr, dv);
                    const void *hsrc[7] = {sl.user.x, sl.user.y, sl.user.z, sl.user.u, sl.user.v, sl.user.w,
                                           sl.user.q};
                    void *ddst[7] = {dv.x, dv.y, dv.z, dv.u, dv.v, dv.w, dv.q};
                    // upload batch -> slot k once its previous download is done
                    (void)hipStreamWaitEvent(h2d, freed[k], 0);
                    for (int i = 0; i < 7; ++i)
                        (void)hipMemcpyAsync(ddst[i], (const char *)hsrc[i] + off * es, cnt * es,
                                             hipMemcpyHostToDevice, h2d);
                    if (sl.user.id)
                        (void)hipMemcpyAsync(dv.id, sl.user.id + off, cnt * 8, hipMemcpyHostToDevice, h2d);
                    (void)hipEventRecord(loaded[k], h2d);
                    // compute on the slot
                    (void)hipStreamWaitEvent(cs, loaded[k], 0);
                    uint32_t *toff = (uint32_t *)tiles + bidx * (r.tg.ntiles + 1);
                    SpeciesWork w = work_of(dv, m);
                    if (sort_due &&
                        (e = launch_sort(r.grid, w, r.tg, sort_scr, toff, sort_ordered && step > 0, cs)) != hipSuccess)
                        fail_run(r, e, "batch sort");
                    // variant 0 when the configured one's LDS does not fit
                    LaunchCfg bcfg = resolve_cfg(lcfg, w.dtype, w.mom ? w.acc_dtype : SPIC_F64);
                    if (tiled_lds_bytes(r.tg, w.dtype, w.acc_dtype, bcfg.variant, bcfg.tile_block) > ctx->lds_max)
                        bcfg.variant = 0;
                    if ((e = launch_fused_tiled(r.grid, prm, r.fields, w, r.tg, toff, bcfg, cs)) != hipSuccess)
                        fail_run(r, e, "batch kernel");
                    (void)hipEventRecord(computed[k], cs);
                    // download slot -> batch
                    (void)hipStreamWaitEvent(d2h, computed[k], 0);
                    for (int i = 0; i < 7; ++i)
                        (void)hipMemcpyAsync((char *)hsrc[i] + off * es, ddst[i], cnt * es, hipMemcpyDeviceToHost,
                                             d2h);
                    if (sl.user.id)
                        (void)hipMemcpyAsync(sl.user.id + off, dv.id, cnt * 8, hipMemcpyDeviceToHost, d2h);
                    (void)hipEventRecord(freed[k], d2h);
                }
            }
        }
        (void)hipEventRecord(t1, d2h);
        (void)hipEventSynchronize(t1);
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t0, t1) == hipSuccess) r.secs = ms / 1e3;
        e = hipGetLastError();
        if (e != hipSuccess) fail_run(r, e, "streamed run");
    }
    (void)hipStreamSynchronize(cs);
    (void)hipStreamSynchronize(h2d);
    (void)hipStreamSynchronize(d2h);
    if (slot[0]) (void)hipFree(slot[0]);
    if (slot[1]) (void)hipFree(slot[1]);
    if (tiles) (void)hipFree(tiles);
    for (int i = 0; i < 2; ++i) {
        (void)hipEventDestroy(loaded[i]);
        (void)hipEventDestroy(computed[i]);
        (void)hipEventDestroy(freed[i]);
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
}

}  // namespace spic

// ------------------------------------------------------------ planning

namespace spic {

int64_t stream_batch_size(uint64_t budget, int64_t max_batch, int dtype, bool with_id, const TileGeom &tg,
                          const int64_t *n, int nsp) {
    auto need = [&](int64_t b) {
        int64_t nbatches = 0;
        for (int s = 0; s < nsp; ++s) nbatches += (n[s] + b - 1) / b;
        return 2 * species_bytes(b, dtype, with_id) + sort_scratch_bytes(b, dtype, with_id, tg) +
               (size_t)nbatches * (tg.ntiles + 1) * 4;
    };
    int64_t nb = max_batch;
    if (budget == 0) return nb;
    while (nb > 1024 && need(nb) > budget) nb /= 2;
    return need(nb) <= budget ? nb : 0;
}

}  // namespace spic

int spic_ctx_s::plan_run(const spic_run &R, int r, spic::RunPlan &p) {
    using namespace spic;
    p = RunPlan{};
    // one tiling per run, for the dtype of its first species
    p.tg = tile_geom(R.grid, R.nspecies > 0 ? R.species[0].dtype : SPIC_F32);
    if (p.tg.cells < 1 || p.tg.cells > 64) return fail(SPIC_E_ARG, "run %d: tile shape must hold 1..64 cells", r);
    std::vector<int64_t> ns;
    for (int s = 0; s < R.nspecies; ++s) {
        const spic_species &sp = R.species[s];
        const int acc = R.moments ? R.moments[s].acc_dtype : SPIC_F64;
        if (job_combo(sp.dtype, R.fields.dtype, acc) < 0)
            return fail(SPIC_E_UNSUPPORTED, "run %d species %d: dtype combination", r, s);
        if (tiled_lds_bytes(p.tg, sp.dtype, acc, 0, 64) > lds_max)
            return fail(SPIC_E_UNSUPPORTED, "run %d species %d: the tile region (tile_x/y/z, halo) does not fit in LDS",
                        r, s);
        const bool big = !tiled_fits(sp.n, sp.dtype);
        if (big && !sp.host_resident)
            return fail(SPIC_E_UNSUPPORTED,
                        "run %d species %d: device-resident species need n * element size < 4 GiB", r, s);
        if (sp.dtype == SPIC_F64) p.dtype = SPIC_F64;
        p.with_id = p.with_id || sp.id;
        if (sp.host_resident) {
            p.host = true;
            p.streamed = p.streamed || big;  // streamed in batches that fit
            p.footprint += species_bytes(sp.n, sp.dtype, sp.id != nullptr);
        }
        // tile ranges, and the species' share of the tick tables (one job, one item per tile)
        p.footprint += (size_t)(p.tg.ntiles + 1) * 4 + 256 + (size_t)p.tg.ntiles * 8 + 512;
        if (!big) p.sort_need = std::max(p.sort_need, sort_scratch_bytes(sp.n, sp.dtype, sp.id != nullptr, p.tg));
        ns.push_back(sp.n);
    }
    if (budget && p.host && p.footprint + p.sort_need > budget) p.streamed = true;
    if (p.streamed) {
        p.batch = stream_batch_size(budget, opt("batch_particles", (int64_t)1 << 26), p.dtype, p.with_id, p.tg,
                                    ns.data(), (int)ns.size());
        if (p.batch <= 0) return fail(SPIC_E_BUDGET, "run %d cannot fit the HBM budget even streamed", r);
        p.footprint = 0;  // a streamed run runs alone and owns its slots for its duration
        p.sort_need = 0;
        return SPIC_OK;
    }
    if (budget && p.footprint + p.sort_need > budget)
        return fail(SPIC_E_BUDGET, "run %d needs %zu bytes of engine memory and %zu of sort scratch; the budget is %llu",
                    r, p.footprint, p.sort_need, (unsigned long long)budget);
    return SPIC_OK;
}

// ------------------------------------------------------------ ctx hooks

using spic::BatchEngine;

int spic_ctx_s::batch_submit(const spic_run *runs, int32_t nruns, uint64_t *tickets) {
    if (nruns == 0) return SPIC_OK;
    if (!batch) {
        batch.reset(new BatchEngine(this));
        batch->tile_block = (int)opt("tile_block", -1);
        batch->variant = (int)opt("tile_variant", -1);
        batch->fixed_geo = (int)opt("fixed_geo", 1);
        batch->sort_ordered = (int)opt("sort_ordered", 1);
        batch->use_graph = (int)opt("graph", 1);
        batch->batch_particles = opt("batch_particles", (int64_t)1 << 26);
        batch->max_groups = (int)opt("max_groups", 0);
        batch->tick_items = opt("tick_items", 4096);
        batch->srpt_aging = 1e6 * (double)opt("srpt_aging", 10000);
        batch->lcfg = launch_cfg();
        int rc = batch->start();
        if (rc) {
            batch.reset();
            return rc;
        }
    }
    return batch->submit(runs, nruns, tickets);
}

int spic_ctx_s::wait(uint64_t ticket, double *secs) {
    if (!batch) return fail(SPIC_E_STATE, "unknown ticket %llu", (unsigned long long)ticket);
    int rc = batch->wait(ticket, secs);
    if (rc == SPIC_E_STATE) return fail(SPIC_E_STATE, "unknown ticket %llu", (unsigned long long)ticket);
    return rc;
}

int spic_ctx_s::poll(uint64_t ticket, int32_t *done) {
    if (!batch) return fail(SPIC_E_STATE, "unknown ticket %llu", (unsigned long long)ticket);
    int rc = batch->poll(ticket, done);
    if (rc == SPIC_E_STATE) return fail(SPIC_E_STATE, "unknown ticket %llu", (unsigned long long)ticket);
    return rc;
}

void spic_ctx_s::shutdown() {
    if (batch) batch->shutdown();
    batch.reset();
}

spic_ctx_s::spic_ctx_s() {}
spic_ctx_s::~spic_ctx_s() {}
