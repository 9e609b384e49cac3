/*
 * spic.h -- C ABI of the MI355X (gfx950) implicit particle-in-cell mover and
 * moment gathering library (libspic.so).
 *
 * The method is the implicit PIC particle stage of sputniPIC
 * (arXiv 2008.04397, Sec. II and Sec. III):
 *   - per particle, a fixed number of predictor-corrector iterations of the
 *     implicit mean velocity (Eq. 1, Eq. 2), each gathering E and B at the
 *     current half-step position with linear weights (Eq. 3, Eq. 4), then the
 *     update of velocity and position (Eq. 5) in a periodic box;
 *   - the particle-to-grid moments rho, J and the pressure tensor P of each
 *     species (Sec. II, moment equation), deposited from the updated state in
 *     the same pass as the move (Sec. III-B, fused mover and gathering).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every call returns an int status: SPIC_OK (0) or a negative error code.
 *    No call throws or aborts.  On error, spic_last_error(ctx) returns a
 *    human-readable message (valid until the next call on that ctx).
 *  - Argument validation happens on the host before anything is enqueued: a
 *    call that returns an error has enqueued no work.
 *  - Device pointers are HIP device addresses on the ctx's device.  All
 *    particle, field and moment buffers are owned by the caller and must stay
 *    valid until the enqueued work completes.  The library owns only its
 *    scratch (sort keys and offsets, staging slots, work lists), allocated
 *    within the ctx's HBM budget and freed by spic_ctx_destroy.
 *  - Work is enqueued on the caller's HIP stream (hip_stream, a hipStream_t;
 *    NULL means the null stream) and the call returns without waiting.
 *    Faults inside kernels surface at the next synchronisation.
 *  - Grid: a periodic box [0,Lx) x [0,Ly) x [0,Lz) with nx, ny, nz cells and
 *    as many distinct nodes per axis, node (i,j,k) at (i*Lx/nx, j*Ly/ny,
 *    k*Lz/nz) and flat index (i*ny + j)*nz + k.  n_d >= 2 on every axis.
 *  - Particles (Sec. III-D: structure-of-arrays): one array per coordinate
 *    x, y, z, velocity u, v, w and charge q, each of n elements of the
 *    species' dtype, contiguous.  x, y, z, u, v, w are updated in place;
 *    q is only read by the mover; sorts permute all seven arrays together.
 *    Positions may lie anywhere; they are wrapped into the box by the mover.
 *  - Moments: [10][nodes] of the accumulation dtype, in the order rho, Jx,
 *    Jy, Jz, Pxx, Pxy, Pxz, Pyy, Pyz, Pzz; each entry is the plain sum
 *    sum_p q {1, v, v (x) v} W over the particles (no volume factor).
 *  - Units are normalised (Sec. III-C), c = 1 unless the caller says
 *    otherwise; qom is the species' charge-to-mass ratio q/m.
 *  - NaN inputs propagate; they are not checked.
 */
#ifndef SPIC_H
#define SPIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPIC_ABI_VERSION 2

/* status codes */
#define SPIC_OK             0
#define SPIC_E_ARG         -1  /* NULL pointer, bad size, bad dtype, misalignment     */
#define SPIC_E_BUDGET      -2  /* the request cannot fit the ctx's HBM budget          */
#define SPIC_E_HIP         -3  /* HIP runtime error (text in spic_last_error)          */
#define SPIC_E_UNSUPPORTED -4  /* valid but unsupported combination (e.g. dtypes)      */
#define SPIC_E_STATE       -5  /* unknown ticket, or a call that does not fit the state */

/* element types */
#define SPIC_F32 1
#define SPIC_F64 2
#define SPIC_F32C 3  /* moment accumulation only: compensated FP32 (see spic_moment_array) */

typedef struct spic_ctx_s *spic_ctx;

/* Periodic box (see conventions above). */
typedef struct {
    int32_t nx, ny, nz;
    int32_t reserved;   /* must be 0 */
    double Lx, Ly, Lz;
} spic_grid;

/* Time step and mover controls.
 *  dt           time step (Eq. 1, Eq. 2, Eq. 5)
 *  c            speed of light in the normalised units (Eq. 2); > 0
 *  niter_mover  predictor-corrector iterations (three in the paper); >= 1.
 *               With mover_tol > 0 it is the cap on the iterations.
 *  sort_every   re-sort the particles by cell every sort_every steps
 *               (Sec. III-A, Sec. VI: sorting restores locality); 0 = never.
 *               Sorting permutes the particle arrays (and id, if given).
 *  step         the caller's step counter: a sort runs before the move when
 *               sort_every > 0 and step % sort_every == 0.
 *  mover_tol    0 (default): exactly niter_mover iterations.  > 0: the
 *               iteration count is set by this error tolerance instead
 *               (Sec. II, after Eq. 2): each particle stops after its k-th
 *               iteration (k >= 2) once the change of its mean velocity over
 *               that iteration, max over x, y, z of |vbar^k - vbar^(k-1)|,
 *               is below mover_tol (velocity units), and after niter_mover
 *               iterations at the latest.  Finite, >= 0. */
typedef struct {
    double dt;
    double c;
    int32_t niter_mover;
    int32_t sort_every;
    int64_t step;
    double mover_tol;
} spic_params;

/* Node-centred E and B (Sec. II, Eq. 4): six device arrays of `nodes`
 * elements of `dtype`, read only. */
typedef struct {
    int32_t dtype;
    int32_t reserved;   /* must be 0 */
    const void *ex, *ey, *ez, *bx, *by, *bz;
} spic_fields;

/* One particle species (Sec. III-B: species are independent streams).
 *  dtype          SPIC_F32 or SPIC_F64 for x, y, z, u, v, w, q
 *  host_resident  0: arrays are device memory.  1: arrays are pinned host
 *                 memory (hipHostMalloc); only spic_batch_submit accepts
 *                 this, streaming the species through HBM in batches
 *                 (Sec. III-B, particle batching).
 *  n              particle count (>= 0; 0 is a no-op)
 *  qom            charge-to-mass ratio q/m
 *  id             optional int64 particle ids (may be NULL), permuted
 *                 together with the particles when they are sorted. */
typedef struct {
    int32_t dtype;
    int32_t host_resident;
    int64_t n;
    double qom;
    void *x, *y, *z, *u, *v, *w;
    void *q;            /* read by the mover, permuted by sorts */
    int64_t *id;
} spic_species;

/* Moment output of one species: a device array [10][nodes].
 *  acc_dtype  SPIC_F64 (default; accumulation in FP64), SPIC_F32 (plain
 *             single precision accumulation, for precision studies) or
 *             SPIC_F32C (compensated FP32, FP32 particles only): m is then
 *             [2][10][nodes] FP32, a high and a low plane whose sum is the
 *             moment.  Every term is formed in FP32 (cell offsets from an
 *             FMA with a two-float 1/dx, so a position's cell-relative
 *             coordinate keeps its precision) and added to the high plane
 *             with an atomic that returns the old value; the exact rounding
 *             error of that addition (Knuth's two-sum, in FP32) is added to
 *             the low plane.  No FP64 arithmetic; the species takes the
 *             unsorted path (global atomics). */
typedef struct {
    int32_t acc_dtype;
    int32_t reserved;   /* must be 0 */
    void *m;
} spic_moment_array;

/* One multi-step run for spic_batch_submit: nsteps fused steps of every
 * species with fixed fields; the moments written are those of the last
 * step.  params.step is the step counter of the first step. */
typedef struct {
    spic_grid grid;
    spic_params params;
    spic_fields fields;
    spic_species *species;
    spic_moment_array *moments;   /* nspecies entries, or NULL for no moments */
    int32_t nspecies;
    int32_t nsteps;
} spic_run;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device` whose library-owned scratch never
 * exceeds hbm_budget_bytes (0 = no limit).  *out receives the handle.
 * device = -1 creates a host-only context that makes no HIP call: every
 * entry point validates its arguments as usual and then, instead of
 * enqueuing work, returns SPIC_E_STATE (used to check arguments, and for
 * admission decisions, on machines without a GPU). */
int spic_ctx_create(int device, uint64_t hbm_budget_bytes, spic_ctx *out);

/* Wait for the ctx's own streams, free all library-owned memory and the
 * handle.  NULL is accepted. */
int spic_ctx_destroy(spic_ctx ctx);

/* Message of the last error on ctx (never NULL; "" when none). */
const char *spic_last_error(spic_ctx ctx);

/* Name of a status code. */
const char *spic_status_str(int status);

/* SPIC_ABI_VERSION of the library. */
int spic_version(void);

/* Tuning knobs, keyed by name; none changes results beyond rounding order.
 * Out-of-range values and unknown keys return SPIC_E_ARG.
 *   block          threads per block of the unsorted-path kernels (64..1024, x64)
 *   grid_cap       cap on blocks of grid-stride kernels
 *   path           0 = tiled kernel for sorted species, 1 = unsorted path only
 *   tile_block     threads per block of the tiled kernel (64..512, x64; -1 =
 *                  by variant: 512 for variant 0, else 256)
 *   tile_x/y/z     sort tile shape in cells (product <= 64)
 *   halo           cells of halo staged around a tile in LDS (0..8)
 *   lds_max        read only: LDS bytes a workgroup may use on the device
 *   tile_variant   tiled-kernel variant (0..3; -1 = by precision): 0 one
 *                  kernel, every deposit an FP64 LDS atomic; 1 as 0 with
 *                  the 48 field values of a thread's last cell in registers
 *                  (default for FP64 particles); 2 a mover launch, then
 *                  a deposit launch into per-lane register sums of sorted
 *                  cells (default for FP32 particles); 3 the mover of 1 and
 *                  the register deposit of 2 in one launch (FP32
 *                  particles; FP64 particles run 2)
 *   mover_cache    variant 2: 1 = the mover launch keeps the 48 field
 *                  values of a thread's last cell in registers (default), 0 =
 *                  every gather reads LDS
 *   mover_block    variant 2: threads per workgroup of the mover launch
 *                  (64..512, x64; default 512)
 *   mover_halo     variants 2 and 3: cells of halo of the mover's field
 *                  region (-1..8; -1 = the tile halo + 1; a region too large
 *                  for the device's LDS falls back to the tile halo)
 *   tile_group     mapping of tiles to workgroups of a tiled launch: groups
 *                  of 2^value consecutive tiles dealt to the 8 XCDs in turn
 *                  (0..10, default 4); -1 = XCD slabs, each XCD taking a
 *                  contiguous eighth of the tiles (a launch whose particles
 *                  occupy a contiguous fraction of the tiles, as a streamed
 *                  batch does, then runs on few XCDs)
 *   fixed_geo      1 = kernels compiled for 4x4x4 tiles with halo 1 (and
 *                  the variant-2 mover's halo 2) are used when that tiling
 *                  is in effect
 *   bank_align     1 = LDS region layout that keeps a particle's bank pair
 *                  when it drifts along the most-crossed axis (more LDS);
 *                  0 = the most compact conflict-free layout; 2 = dense,
 *                  no padding (default: 1 for FP32 particles, 0 for FP64)
 *   sort_ordered   1 = a re-sort walks each tile of the current order in
 *                  order, so ranks inside a cell keep that order (0/1)
 *   sort_rows      1 = full rows: a tile of n particles and C cells gets
 *                  n / C rows of C slots, slot (r, c) holding rank r of cell
 *                  c where that exists and the particles of higher ranks
 *                  filling the rest; 0 = plain rank blocks (default 1 for
 *                  tile variants 2 and 3, else 0)
 *   graph          batch engine: replay unchanged ticks as a hipGraph (0/1)
 *   batch_particles  batch engine: particles per streamed batch
 *   max_groups     batch engine: cap on workgroups of the persistent
 *                  (mover) launch
 *   tick_items     batch engine: a tick steps the runs with the least
 *                  remaining work until it holds this many (run, species,
 *                  tile) items (default 4096; 0 = every active run)
 *   srpt_aging     batch engine: remaining work is credited this many
 *                  million particle-steps per second since submission, so
 *                  long runs are not starved by a stream of short ones
 *                  (default 10000; 0 = pure least-remaining-work) */
int spic_set_option(spic_ctx ctx, const char *key, int64_t value);
/* The value of an option: the value set, or -1 when unset (the library then
 * decides; tile_group reads 4, its default, and lds_max the device's limit).
 * "f32:<key>" / "f64:<key>" read the launch setting the library resolves for
 * FP32 / FP64 particles with FP64 moments (keys tile_variant, tile_block,
 * sort_rows, halo, bank_align, sort_ordered, mover_cache, mover_halo,
 * tile_group).  Unknown keys return SPIC_E_ARG. */
int spic_get_option(spic_ctx ctx, const char *key, int64_t *value);

/* ------------------------------------------------------------- hot path */

/* One implicit step of nsp species (Sec. II: Eq. 1-5), fused with the
 * moment gathering of the moved particles when mom != NULL (Sec. III-B).
 *  grid, params, fields  as above; fields.dtype must equal the particles'
 *                        dtype, or be SPIC_F64 with SPIC_F32 particles
 *  sp[nsp]               species, device resident, updated in place (and
 *                        permuted when a sort runs, see spic_params)
 *  mom                   NULL (move only) or nsp moment outputs; each is
 *                        overwritten with the moments of the new state
 *  hip_stream            stream to enqueue on
 * Errors: SPIC_E_ARG (validation), SPIC_E_UNSUPPORTED (dtype combination),
 * SPIC_E_BUDGET (sort scratch does not fit), SPIC_E_HIP (launch failure). */
int spic_mover(spic_ctx ctx, const spic_grid *grid, const spic_params *params,
               const spic_fields *fields, spic_species *sp, int32_t nsp,
               spic_moment_array *mom, void *hip_stream);

/* Moments of nsp species from their current state (Sec. II, moment
 * equation), without moving them.  Overwrites mom[s] unless accumulate != 0,
 * in which case the moments are added to what mom[s] holds. */
int spic_moments(spic_ctx ctx, const spic_grid *grid, const spic_species *sp, int32_t nsp,
                 spic_moment_array *mom, int32_t accumulate, void *hip_stream);

/* Sort the particles of nsp species by cell (Sec. III-A: ordering particles
 * by position restores the locality of the field and moment accesses).
 * Permutes x, y, z, u, v, w, q and id (when given) together; the
 * per-particle state is unchanged, only its order. */
int spic_sort(spic_ctx ctx, const spic_grid *grid, spic_species *sp, int32_t nsp,
              void *hip_stream);

/* Bytes of device memory spic_mover_noalloc's fixed scratch holds on each
 * GPU the library runs on (from the first context on that GPU until the
 * process ends). */
#define SPIC_NOALLOC_SCRATCH_BYTES (256u * 1024u * 1024u)

/* For callers that cannot allocate device memory: code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc.  One
 * fused step (spic_mover) with a sort of every species before its move:
 * params->sort_every must be 1, and the particles end up permuted into
 * sorted order (id with them, when given), as spic_mover leaves them with
 * sort_every = 1.  All scratch -- sort keys, ranks and slot indices, the
 * reordered copy of the particles, per-tile particle ranges -- lives in one
 * fixed array of SPIC_NOALLOC_SCRATCH_BYTES per GPU instead of memory the
 * library allocates; the call makes no hipMalloc, hipFree or other
 * allocating call.  The caller passes and owns the particles, fields and
 * moments as for spic_mover.
 *  - A species whose sort needs more scratch than the array holds (about
 *    4 million FP32 particles with ids) is refused with SPIC_E_BUDGET
 *    before anything is enqueued.
 *  - Every call on one GPU, from any context, shares that GPU's array and
 *    finds the last call's contents in it (nothing is carried over; each
 *    call clears what it uses).  Calls that overlap on one GPU (two
 *    streams, threads or contexts) race on the array: serialise them.
 *  - The sort layout an earlier spic_sort or spic_mover kept for a species
 *    is dropped (its particles were reordered).
 * Errors: as spic_mover, plus SPIC_E_ARG for sort_every != 1. */
int spic_mover_noalloc(spic_ctx ctx, const spic_grid *grid, const spic_params *params,
                       const spic_fields *fields, spic_species *sp, int32_t nsp,
                       spic_moment_array *mom, void *hip_stream);

/* ---------------------------------------------------------------- batches */

/* Submit nruns independent multi-step runs (Sec. III-B, particle batching).
 * Queued runs are admitted, in submission order, as soon as their HBM
 * footprint fits the ctx's budget (host_resident species are uploaded on
 * admission and copied back on completion).  Each tick advances admitted
 * runs by one step -- those with the least remaining work (less the
 * `srpt_aging` credit for time waited) first, until the tick holds
 * `tick_items` (run, species, tile) items -- in one launch per
 * precision combination.  A host_resident run larger than the budget, or
 * with a species of 4 GiB or more per array, is streamed through HBM in
 * batches on two streams (copy of the next batch overlapping the kernel on
 * the current one).  Device-resident species need n * element size < 4 GiB.
 * Work runs on the ctx's own streams; tickets_out[i] identifies run i.  The
 * caller's arrays must stay valid until the ticket completes.
 * Errors: SPIC_E_ARG, SPIC_E_BUDGET (a run cannot fit even when streamed),
 * SPIC_E_UNSUPPORTED, SPIC_E_HIP. */
int spic_batch_submit(spic_ctx ctx, const spic_run *runs, int32_t nruns, uint64_t *tickets_out);

/* Block until the ticket's run is complete; device_seconds_out (may be
 * NULL) receives the device time of the run.  SPIC_E_STATE for an unknown
 * ticket. */
int spic_wait(spic_ctx ctx, uint64_t ticket, double *device_seconds_out);

/* *done = 1 when the ticket's run is complete, else 0. */
int spic_poll(spic_ctx ctx, uint64_t ticket, int32_t *done);

/* ------------------------------------------------------------ field solve */

/* The implicit field solve that closes the cycle (Sec. II, step 3: a linear
 * system from the implicit-in-time discretisation of Maxwell's equations,
 * solved with GMRes, and a Poisson equation solved with CG each cycle so
 * that the continuity equation holds -- "divergence cleaning"; Sec. VI
 * names the solver's residual as the next GPU port).  The paper prints no
 * discretisation; the one used (FP64 throughout) is:
 *   grid      the periodic node grid of the particle step; vectors are
 *             [3][nodes] FP64 device arrays (x, y, z components);
 *   D_d       central differences (f(+e_d) - f(-e_d)) / (2 dx_d); curl,
 *             div and grad are built from them; the Poisson operator is
 *             div grad;
 *   mu        susceptibility at a node: sum over species s of
 *             (fourpi / 2) theta dt^2 qom_s rho_s R(b_s), b_s =
 *             qom_s dt B / (2 c), R(b) the rotation of the mover's Eq. 2
 *             (R v solves vhat = v + vhat x b);
 *   Jhat      implicit current: sum_s R(b_s) (J_s - dt/2 div P_s),
 *             (div P)_a = sum_b D_b P_ab, from the species' moments
 *             (rho, J, P as spic_moment_array orders them);
 *   equation  (I + mu) E' + (c theta dt)^2 curl curl E'
 *                 = E + theta dt (c curl B - fourpi Jhat)
 *             for E' = E^{n+theta};
 *   update    E <- (E' - (1 - theta) E) / theta, B <- B - c dt curl E';
 *   cleaning  before the solve, E <- E - grad phi with
 *             div grad phi = div E - fourpi rho_bar (CG), rho_bar the total
 *             charge density without its components along the null space
 *             of div grad (the modes constant or alternating along each
 *             axis; alternating only where the node count is even). */
typedef struct {
    double dt;
    double c;
    double theta;      /* time centring, in (0, 1] */
    double fourpi;     /* 4 pi of the unit system (>= 0) */
    double tol;        /* relative residual target of both solves, in (0, 1) */
    int32_t max_iter;  /* cap on the iterations of each solve, >= 1 */
    int32_t restart;   /* GMRes Krylov basis size, 1..64 */
} spic_field_params;

/* E and B of the field cycle: six FP64 device arrays of `nodes` elements
 * (flat node index (i * ny + j) * nz + k), read and overwritten in place by
 * spic_field_cycle, read only by spic_field_apply. */
typedef struct {
    double *ex, *ey, *ez, *bx, *by, *bz;
} spic_em_state;

/* Iterations and final relative residuals of one field cycle: clean_resid
 * is the CG recurrence residual |r| / |r0|, solve_resid the true residual
 * |b - A E'| / |b| of the GMRes result. */
typedef struct {
    int32_t clean_iters;
    int32_t solve_iters;
    double clean_resid;
    double solve_resid;
} spic_field_stats;

/* y = (I + mu) x + (c theta dt)^2 curl curl x: the field operator (the
 * residual's matrix-vector product) for the susceptibility of the given
 * moments and B.
 *  em           B is read (E is not used); FP64 device arrays
 *  mom[nsp]     SPIC_F64 moment arrays of the species ([10][nodes])
 *  qom[nsp]     host array of the species' charge-to-mass ratios
 *  x, y         [3][nodes] FP64 device arrays (distinct)
 * Enqueued on hip_stream; library scratch of 12 nodes doubles.
 * Errors: SPIC_E_ARG (validation; nsp in 0..16), SPIC_E_BUDGET, SPIC_E_HIP. */
int spic_field_apply(spic_ctx ctx, const spic_grid *grid, const spic_field_params *params,
                     const spic_em_state *em, const spic_moment_array *mom, const double *qom, int32_t nsp,
                     const double *x, double *y, void *hip_stream);

/* One field cycle: clean E (CG), solve the field equation for E' (GMRes,
 * restarted every params->restart iterations, from the cleaned E), update E
 * and B in place.  Synchronous: the host drives both solves and the call
 * returns when the update is done (stats, when not NULL, are filled).
 * Library scratch: about (9 + 6 x 3 + 5 + 3 (restart + 1)) nodes doubles.
 * Errors: SPIC_E_ARG (validation), SPIC_E_BUDGET, SPIC_E_HIP. */
int spic_field_cycle(spic_ctx ctx, const spic_grid *grid, const spic_field_params *params, spic_em_state *em,
                     const spic_moment_array *mom, const double *qom, int32_t nsp, spic_field_stats *stats,
                     void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* SPIC_H */
