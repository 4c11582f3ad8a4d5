/*
 * grlbm.h -- C ABI of the MI355X (gfx950) five-field gradient-reconstruction
 * lattice Boltzmann solver for the compressible Navier-Stokes-Fourier equations
 * (Kummerlaender, Bukreev, Krause).
 *
 * What the library computes.  Each call of lbm_step advances the populations of
 * the five conserved fields Q = (rho, rho u_x, rho u_y, rho u_z, E) (eq. 2) by one
 * collide-and-stream update per step, exactly as Algorithm 1 lists it: conserved
 * and first moments, floored primitives, the direct gradient from the
 * non-equilibrium first moment (eq. 3), the reconstruction operator R of eq. 4
 * evaluated as the block forward solve of eqs. 5-7, the chain rule to grad u and
 * grad T, the compression sensor (Sec. 2.5, Listing 2), Newtonian stress and
 * Fourier flux in the equilibrium flux, a regularized (or BGK) collision, and exact
 * on-lattice streaming on D3Q7 (c_s^2 = 1/4, 7 populations per field, 35 per cell).
 *
 * Units.  Every quantity crossing this ABI is in lattice units: cell size 1, time
 * step 1.  The solver does not convert units.
 *
 * Storage.  One device buffer holds 35 population arrays (structure of arrays,
 * x fastest), updated in place with the AA access pattern, so a single copy of the
 * state suffices: 140 bytes per cell in FP32, 70 in FP16.  On grids of more than
 * one x-row, each row is padded to whole 128-byte lines when that adds at most a
 * sixteenth of its length (and keeps the padded grid in the 32-bit index range), so
 * that the rows a cell's +-y and +-z neighbours sit in start on a line too; the
 * padding is never read or written.  lbm_state_bytes accounts for it.  The stored value is the
 * deviation f - w_i Q_ref from the equilibrium of a uniform reference state
 * (Sec. 2.2), Q_ref = (rho_ref, 0, 0, 0, E_ref).
 *
 * Threading.  A context is not internally locked: use one context per host thread
 * at a time.  lbm_last_error is thread-local.
 *
 * Errors.  Every call returns an lbm_status; on failure lbm_last_error() describes
 * it.  No call aborts the process.
 */
#ifndef GRLBM_H
#define GRLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,     /* invalid argument (message names it)                         */
  LBM_ENOMEM = -2,     /* device or host allocation failed                            */
  LBM_EDEVICE = -3,    /* a HIP runtime call failed (message keeps the HIP error)     */
  LBM_EDIVERGED = -4,  /* a diagnostic reduction saw a non-finite population          */
  LBM_ESTATE = -5      /* call out of order (e.g. step before init)                    */
} lbm_status;

typedef enum { LBM_BC_PERIODIC = 0, LBM_BC_ZERO_GRADIENT = 1 } lbm_bc;
/* Sec. 2.2 / 2.5: the regularized collision with the compression sensor is used
 * for the shock cases, BGK for smooth ones. */
typedef enum { LBM_COLL_RLB_SENSOR = 0, LBM_COLL_BGK = 1 } lbm_collision;
typedef enum { LBM_STORE_F32 = 0, LBM_STORE_F16 = 1 } lbm_storage;
/* Initial populations (the paper states none).  FIRST_ORDER: the first moment the
 * update holds a resolved field at, from central differences of the initial fields
 * (lbm_init_fields); EQUILIBRIUM: the equilibrium of the fields with their advective
 * flux, for initial data with jumps (a Riemann problem), where differences across a
 * jump are no gradient and would start negative densities. */
typedef enum { LBM_START_FIRST_ORDER = 0, LBM_START_EQUILIBRIUM = 1 } lbm_start;
/* Listing 1: mu(T) = mu_ref (1+T_S) (T/T_ref)^(3/2) / (T/T_ref + T_S). */
typedef enum { LBM_MU_CONSTANT = 0, LBM_MU_SUTHERLAND = 1 } lbm_mu_law;

typedef struct {
  int32_t nx, ny, nz;          /* cells; x is the fastest index of every array        */
  int32_t bc[3];               /* lbm_bc per axis (x, y, z)                            */
  int32_t collision;           /* lbm_collision                                        */
  int32_t storage;             /* lbm_storage of the populations                       */
  int32_t mu_law;              /* lbm_mu_law                                           */
  int32_t layout_pad;          /* extra elements between population arrays (>= 0);
                                  arrays always start on 256-byte boundaries          */
  int32_t start;               /* lbm_start: how the initial fields become populations */
  double gamma;                /* ratio of specific heats (eq. 2 equation of state)    */
  double mu_ref, kappa_ref;    /* viscosity and conductivity at T_ref; both scale with
                                  the same law: mu = mu_ref r(T), kappa = kappa_ref r(T),
                                  r = 1 (constant) or the Sutherland factor            */
  double T_ref, T_S;           /* Sutherland reference temperature and constant        */
  double omega[5];             /* relaxation frequency per field (rho, mx, my, mz, E);
                                  each in (0, 2]; the three momentum values must be
                                  equal (the closed-form momentum block needs it)      */
  double sensor_gain;          /* g of the compression sensor                           */
  double J_min;                /* dead band of the sensor                               */
  double omega_min;            /* rate the sensor relaxes towards                       */
  double rho_min, p_min;       /* positivity floors (Algorithm 1, primitives)          */
  double rho_ref, E_ref;       /* reference state of the equilibrium shift              */
} lbm_params;

/* One diagnostic record (the channels of Sec. 3.3), reduced over all cells at the
 * start of step `step` (the state after `step` completed steps): volume sums of the
 * kinetic energy density
 * rho|u|^2/2, the solenoidal dissipation mu|curl u|^2 and the dilatational
 * dissipation (4/3) mu (div u)^2 (velocity gradient from the reconstruction), the
 * totals of the five conserved fields minus N Q_ref, and the number of cells whose
 * updated populations are not finite. */
typedef struct {
  int64_t step;
  double Ek, eps_s, eps_d;
  double dtotal[5];
  int64_t nonfinite;
} lbm_diag;

typedef struct lbm_ctx lbm_ctx; /* opaque */

/* Bytes of device memory the populations of `p` need (35 arrays, padded).
 * Returns 0 if p is invalid. */
size_t lbm_state_bytes(const lbm_params* p);

/* Validate p, allocate the population buffer on the current HIP device and bind the
 * context to `hip_stream` (a hipStream_t; NULL creates a private stream, which the
 * context destroys).  EINVAL: dims < 1, a zero-gradient axis with fewer than 2
 * cells, omega outside (0, 2], unequal momentum omegas, non-finite or non-positive
 * gamma-1, mu_ref, T_ref, rho_min, or negative p_min, layout_pad < 0, unknown enum.
 * ENOMEM: device allocation failed.  On failure *out is NULL. */
lbm_status lbm_create(const lbm_params* p, void* hip_stream, lbm_ctx** out);

/* As lbm_create, but the populations live in the caller's device buffer
 * `dev_buf` of `bytes` bytes (>= lbm_state_bytes(p), 256-byte aligned), e.g. the
 * storage of a torch tensor; the caller keeps ownership and must keep it alive
 * until lbm_destroy. */
lbm_status lbm_create_in(const lbm_params* p, void* dev_buf, size_t bytes, void* hip_stream,
                         lbm_ctx** out);

/* Set the state from the conserved fields Q and reset the step counter to 0.  The
 * paper states no initialisation.  With params.start = LBM_START_FIRST_ORDER the
 * populations get zeroth moment Q, the equilibrium second moment and the first
 * moment J_k = Phi_k - (c_s^2/omega_k) grad Q_k that the update holds a resolved
 * field at to first order (the fixed point of the relaxation of the first moment
 * followed by streaming), with grad Q from central differences of Q (periodic wrap;
 * beyond a zero-gradient face the cell itself) and Phi the flux of eq. 2 with the
 * Newtonian stress and Fourier flux of that gradient.  The reconstruction of eq. 4
 * returns that gradient at step 0, and no step-to-step oscillation of the
 * non-equilibrium is started (omega -> 2 would leave it undamped).  With
 * LBM_START_EQUILIBRIUM they are the equilibrium of Q with the advective flux.  A
 * uniform state starts at its equilibrium either way.  Q: host array
 * [5][nz][ny][nx] of doubles, lattice units, field order (rho, rho u_x, rho u_y,
 * rho u_z, E).  EINVAL (state unchanged) if a value is not finite or the density
 * or the pressure (gamma - 1)(E - |rho u|^2 / (2 rho)) of a cell is not positive.
 * Synchronises the stream before returning. */
lbm_status lbm_init_fields(lbm_ctx* ctx, const double* Q);

/* Same, with Q already in device memory (float64, same layout); asynchronous for
 * FP32 storage.  FP16 storage keeps each field's shifted populations times a power
 * of two chosen here from the initial state (largest |value| mapped into
 * [32, 64), leaving 1024x headroom for populations that grow during the run),
 * which keeps the values in FP16's normal range; choosing it synchronises the
 * stream.  The scale is invisible through this ABI. */
lbm_status lbm_init_fields_device(lbm_ctx* ctx, const double* Q_dev);

/* Enqueue n >= 0 collide-and-stream steps on the context's stream (asynchronous).
 * If diag_every > 0, every step whose index t (completed steps before it) satisfies
 * t % diag_every == 0 also produces a diagnostic record (see lbm_diagnostics).
 * ESTATE before initialisation. */
lbm_status lbm_step(lbm_ctx* ctx, int64_t n, int32_t diag_every);

/* Conserved fields of the current state (post-streaming, i.e. the state after the
 * completed steps) into the host array Q_out [5][nz][ny][nx] (doubles).
 * Synchronises the stream. */
lbm_status lbm_moments(lbm_ctx* ctx, double* Q_out);

/* Same into device memory (float64, same layout); asynchronous. */
lbm_status lbm_moments_device(lbm_ctx* ctx, double* Q_dev);

/* Copy out, oldest first, up to `max` diagnostic records produced since the last
 * call and discard them; *count receives the number written.  Synchronises the
 * stream.  Returns EDIVERGED (after filling the records) if any returned record
 * has nonfinite > 0. */
lbm_status lbm_diagnostics(lbm_ctx* ctx, lbm_diag* out, int32_t max, int32_t* count);

/* Checkpoint: the 35 populations of every cell in canonical order (the stored
 * shifted value of direction i of field k at cell x after the completed steps,
 * independent of the AA parity) into the host array f[35][nz][ny][nx] (floats),
 * and the step counter.  Synchronises the stream. */
lbm_status lbm_get_populations(lbm_ctx* ctx, float* f, int64_t* step);

/* Restore a checkpoint written by lbm_get_populations (same params).  FP16 storage
 * rounds to nearest even.  Synchronises the stream. */
lbm_status lbm_set_populations(lbm_ctx* ctx, const float* f, int64_t step);

/* Launch shape of the collide-and-stream kernels: `block` threads per block (a
 * multiple of 64 in [64, 1024]; default 256), nontemporal loads/stores on or off
 * (default on, except for population states of 24 MiB up to 320 MiB, which the
 * 256 MB Infinity Cache partly keeps between steps), and an occupancy cap of `blocks_per_cu` resident blocks per compute
 * unit (1..32, enforced by reserving LDS; 0 = no cap; default 4 for FP32 storage and
 * no cap for FP16).  With `odd_lds` = 1 (the default) the odd AA step
 * moves the +-x populations through LDS so that all its HBM accesses are aligned.
 * It runs blocks of two or more whole x-rows where they fill at most 512 lanes
 * exactly (nx not a multiple of 64, rows unpadded; FP16 two rows only), else one
 * block per x-row when nx <= 1024 and nx is a multiple of 32 (64 for FP16), else
 * tiles of 512 consecutive cells (256 for FP16).  Where a row is not a whole
 * number of 128-byte lines it loads the y slots without the nontemporal hint.
 * `block` and `blocks_per_cu` then apply to the even step only.  With FP16 storage on grids of
 * 2^23 cells and more, a lane takes two consecutive cells (4-byte accesses) in the
 * even step when `block` <= 256 and the cell count is even, and in the LDS odd step
 * when nx is 384 or 512.
 * Results do not depend on any of these settings.  EINVAL otherwise. */
lbm_status lbm_set_launch(lbm_ctx* ctx, int32_t block, int32_t nontemporal, int32_t blocks_per_cu,
                          int32_t odd_lds);

/* A launch shape as lbm_set_launch takes it. */
typedef struct {
  int32_t block, nontemporal, blocks_per_cu, odd_lds;
} lbm_launch;

/* The context's current launch shape. */
lbm_status lbm_get_launch(lbm_ctx* ctx, lbm_launch* out);

/* Time candidate launch shapes on the context's live state and keep the fastest:
 * even-step blocks of 256 (capped at 4, 2 or no blocks per CU), 512 (2 or none) and
 * 1024 threads, each with nontemporal access on and off, the LDS odd step on.  Each
 * trial runs 2 warm-up steps and trial_steps timed steps (rounded up to even) with
 * no diagnostics; the populations and the step count are restored from a device
 * snapshot after each trial, so the state after the call is bitwise the state
 * before it.  The fastest shape differs with the grid (the nontemporal hint costs
 * up to a third of the rate on some states of a few hundred MB and gains 3-8% on
 * larger ones).  best/best_us receive it and its time per step; up to max_tried
 * (shape, time) pairs go to tried/tried_us (may be NULL), their number to ntried.
 * Needs a second buffer of the population size (ENOMEM if it cannot be had);
 * synchronises the stream; ESTATE before initialisation, EINVAL if trial_steps < 2. */
lbm_status lbm_autotune(lbm_ctx* ctx, int32_t trial_steps, lbm_launch* best, float* best_us, lbm_launch* tried,
                        float* tried_us, int32_t max_tried, int32_t* ntried);

/* Source term S of eq. 1 for the following steps: S_dev points to device memory
 * S[5][nz][ny][nx] (FP32, lattice units per step, field order rho, rho u_x,
 * rho u_y, rho u_z, E), projected onto the lattice weights and added to the
 * post-collision populations of every step (the collision of Algorithm 1:
 * f*_ki += w_i S_k).  The caller owns the array, keeps it alive while steps that
 * use it are in flight, and may rewrite it between steps in stream order (a
 * time-dependent source is evaluated once per step).  NULL switches the source
 * off (the default; no extra traffic).  FP32 storage only: EINVAL for FP16.  Steps
 * with a source always use nontemporal access. */
lbm_status lbm_set_source(lbm_ctx* ctx, const float* S_dev);

/* Completed steps. */
lbm_status lbm_get_step(lbm_ctx* ctx, int64_t* step);

/* Release the context (waits for its stream first).  NULL is a no-op. */
lbm_status lbm_destroy(lbm_ctx* ctx);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): lbm_step without a
 * context and without any allocation.  Advances the caller's populations F_dev
 * (device, FP32 storage, the layout and lbm_state_bytes(p) of a context with the
 * same params, holding the state after `step` completed steps, e.g. the buffer of
 * an lbm_create_in context) by n steps with the kernels and the default launch
 * shape of lbm_step, asynchronously on hip_stream (a hipStream_t, NULL = the null
 * stream).  With diag_every > 0 each step t in [step, step + n) with
 * t % diag_every == 0 writes one record of 9 floats to rec_dev (device, caller-
 * owned, rec_max records): E_k, eps_s, eps_d, the five dtotal and the non-finite
 * count, as lbm_diag holds them.  The per-block partials of those reductions live
 * in one fixed device array of the library per GPU (2^18 blocks x 9 floats, 9 MiB,
 * held until the process ends); every call on a GPU shares it and it keeps the last
 * call's contents, so calls that overlap on one GPU race.  EINVAL: invalid params,
 * FP16 storage, a NULL or misaligned buffer, negative step, n or diag_every, too
 * few records in rec_max, or a grid whose launches need more than 2^18 partial
 * blocks (more than about 67 M cells) when diag_every > 0.  Calls no hipMalloc or
 * hipFree. */
lbm_status lbm_step_noalloc(const lbm_params* p, void* F_dev, int64_t step, int64_t n, int32_t diag_every,
                            float* rec_dev, int32_t rec_max, void* hip_stream);

/* ------------------------------------------------------------------ batches
 * Many independent instances (different sizes, boundaries, parameters, storage
 * types and start times) advanced together: one persistent kernel per (collision,
 * storage) group walks a tile work-list (a tile is one block-width range of
 * consecutive cells of one instance), and time loops of `graph_steps` steps replay one captured
 * HIP graph.  Every instance keeps its own step count: it is at its step 0 when
 * added, advances with each lbm_batch_run step until it has made the number of
 * steps it was added with, then stays frozen until removed.  Results are bitwise
 * those of the same instance run alone in a context (lbm_create/lbm_step).  All
 * calls use the batch's stream; calls that touch host memory synchronise it. */
typedef struct lbm_batch lbm_batch; /* opaque */

typedef struct {
  int32_t block;          /* threads per block = cells per tile (64..1024)         */
  int32_t nontemporal;    /* nontemporal loads and stores (the odd step still loads
                             its y and z slots without the hint)                  */
  int32_t blocks_per_cu;  /* occupancy cap enforced by an LDS reservation (0 = off) */
  int32_t grid;           /* blocks that loop over the tiles (persistent), or 0 for
                             one block per tile                                     */
} lbm_batch_tuning;

typedef struct {
  int64_t clock;               /* steps run so far by the batch                    */
  size_t arena_bytes, arena_free_bytes, arena_largest_free;
  int32_t live_instances;      /* added and not removed                            */
  int32_t active_instances;    /* live and not yet finished                        */
  int64_t active_cells;
  lbm_batch_tuning tuning;
  int32_t graph_steps;
} lbm_batch_stats;

/* Create a batch: one device arena of arena_bytes for the populations of all its
 * instances, room for max_instances descriptors and max_tiles tiles per group, and
 * time loops captured in graphs of graph_steps steps (1..4096; 1 = no graph).
 * hip_stream as for lbm_create.  The launch shape starts as one 256-cell tile per
 * block with plain (not nontemporal) access and at most 2 blocks per CU (block
 * 256, nontemporal 0, blocks_per_cu 2, grid 0).  EINVAL on bad sizes, ENOMEM if the arena does not
 * fit. */
lbm_status lbm_batch_create(size_t arena_bytes, int32_t max_instances, int32_t max_tiles,
                            int32_t graph_steps, void* hip_stream, lbm_batch** out);

/* Add an instance (params as for lbm_create, validated the same way) initialised
 * like lbm_init_fields from the host array Q [5][nz][ny][nx] (checked the same
 * way: EINVAL for a non-finite value or a cell whose density or pressure is not
 * positive), to make `steps` steps.  *id receives its handle.  ENOMEM when the arena has no free run large
 * enough, the descriptor table is full or its tiles exceed max_tiles. */
lbm_status lbm_batch_add(lbm_batch* b, const lbm_params* p, const double* Q, int64_t steps,
                         int32_t* id);

/* Advance the batch by n >= 0 steps (asynchronous). */
lbm_status lbm_batch_run(lbm_batch* b, int64_t n);

/* Steps an instance has completed and whether it has finished (both may be NULL). */
lbm_status lbm_batch_query(lbm_batch* b, int32_t id, int64_t* done_steps, int32_t* finished);

/* Conserved fields of an instance, as lbm_moments (synchronises). */
lbm_status lbm_batch_moments(lbm_batch* b, int32_t id, double* Q_out);

/* Canonical populations of an instance and its completed steps, as
 * lbm_get_populations (synchronises). */
lbm_status lbm_batch_populations(lbm_batch* b, int32_t id, float* f_out, int64_t* step);

/* Divergence check for early retirement (the failure of a time-marching scheme
 * is a state that is no longer finite; a diverged instance otherwise occupies the
 * device until its step count).  Reports the live instances whose rest
 * population of some field (slot 0 of each of the five fields, every cell) holds
 * an infinity or a NaN.  Slot 0 of field k after a step sums all of the cell's
 * field-k populations (the collision of Algorithm 1), so a non-finite population of any
 * field appears there one step later.  Up to max ids go to ids in ascending order
 * (ids may be NULL when max is 0); *count receives the number of such instances,
 * which may exceed max.  Reads 5 of the 35 arrays of every live instance;
 * synchronises the stream.  EINVAL on a NULL batch or count, or a bad id buffer. */
lbm_status lbm_batch_nonfinite(lbm_batch* b, int32_t* ids, int32_t max, int32_t* count);

/* Release an instance's arena space and descriptor (synchronises first). */
lbm_status lbm_batch_remove(lbm_batch* b, int32_t id);

/* Occupancy and tuning summary. */
lbm_status lbm_batch_info(lbm_batch* b, lbm_batch_stats* out);

/* Set the launch shape (invalidates the captured graph).  grid 0 launches one block
 * per tile of each group (rounded up to a multiple of 256).  EINVAL on bad values,
 * ENOMEM if the tile width needs more tiles than the capacity. */
lbm_status lbm_batch_set_tuning(lbm_batch* b, const lbm_batch_tuning* t);

/* Time every candidate launch shape on the batch's live instances for trial_steps
 * steps each, restoring the populations and the clock after each trial (results do
 * not depend on the shape), and keep the fastest.  The candidates are blocks of
 * 128, 256, 512 and 1024 threads, each with and without nontemporal access, as
 * persistent grids of 8, 16 or 32 resident waves per CU and as one block per tile,
 * uncapped or (256- and 512-thread blocks) capped at 8 or 16 resident waves per CU
 * (36 shapes).  best/best_us receive it and its
 * time per step; up to max_tried (shape, time) pairs go to tried/tried_us (may be
 * NULL), their number to *ntried.  Needs device memory for one copy of the used
 * arena. */
lbm_status lbm_batch_autotune(lbm_batch* b, int32_t trial_steps, lbm_batch_tuning* best,
                              float* best_us, lbm_batch_tuning* tried, float* tried_us,
                              int32_t max_tried, int32_t* ntried);

/* Release the batch (waits for its stream).  NULL is a no-op. */
lbm_status lbm_batch_destroy(lbm_batch* b);

/* Achievable HBM bandwidth: a streaming copy of `bytes` bytes (read + write)
 * repeated `iters` times on a private stream; *gbps receives (2 * bytes) / time of
 * the fastest repetition in GB/s.  Allocates and frees its own buffers. */
lbm_status lbm_bw_probe(size_t bytes, int32_t iters, double* gbps);

/* Description of the last failure on this thread ("" if none). */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GRLBM_H */
