/*
 * pic.h - C ABI of the MI355X (gfx950) 2D electrostatic particle-in-cell
 * library for the trench geometry of Lin & Nishimura (arXiv:1610.03918).
 *
 * One step of the method (Sec. II, eqs. 1-5):
 *   deposit   area-weighted charge of electrons and one ion species (int64
 *             fixed point, 2^32 units per particle, exact and order-free)
 *   solve     eq. (5), -lap(phi) = n_i - n_e on a 5-point grid, with the
 *             grounded plate, the RF plate V = amp*sin(omega*t) (Sec. III.B)
 *             and the trench conductor (Sec. III.C) as Dirichlet nodes
 *   field     E = -grad(phi), central inside, two-point at walls (Sec. II)
 *   push      leapfrog of eqs. (1)-(4), absorption at walls and conductors,
 *             hit classification, ion charge build-up on the trench bottom
 *             (Sec. III.D)
 *
 * Units are the paper's normalised ones: length lambda_e (mesh spacing 1),
 * time 1/omega_e, potential T_e/e, density n_0, velocity lambda_e*omega_e.
 *
 * Layout (all arrays row-major in x, the plate-normal axis):
 *   cells  nx * ny, cell (i, j) at i*ny + j
 *   nodes  NX * NY, NX = nx (periodic x) or nx + 1, NY likewise; node (i, j)
 *          at i*NY + j; cell (i, j) spans nodes i..i+1, j..j+1 (wrapping)
 *   particles, one structure-of-arrays per species and per storage set:
 *          cell int32 = (i << 16) | j, negative once removed (-1 - class);
 *          ox, oy float32 in-cell offsets in [0, 1); vx, vy float32
 *
 * Ownership: the caller allocates every device buffer (particles, charge,
 * potential, right-hand side and one workspace block whose size
 * pic_workspace_size reports) and keeps it alive until pic_destroy.  The
 * library never allocates or frees device memory; it owns only the context.
 *
 * Streams: every call is enqueued on the stream given to pic_init and
 * returns without waiting, except where stated (pic_solve, pic_step and
 * pic_diagnostics wait for the convergence test / copy-back).  The library
 * also owns two streams of default priority: one to capture HIP graphs, and
 * one on which pic_step runs a re-binning beside the next solve (joined to
 * the context's stream before pic_step returns, see there).
 *
 * Errors: every call returns a pic_status; on failure pic_last_error gives
 * a message.  No exception or abort crosses this boundary.  A context is not
 * thread safe.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pic_ctx pic_ctx;

typedef enum {
    PIC_OK = 0,
    PIC_ERR_ARG = -1,            /* invalid configuration or argument */
    PIC_ERR_HIP = -3,            /* a HIP runtime call failed */
    PIC_ERR_NOT_CONVERGED = -4,  /* solver hit max_iter (phi still written), or a batched
                                    step pushed a potential above rtol */
    PIC_ERR_CFL = -5,            /* pic_init / pic_batch_init: omega_pe dt >= 2 at the loaded
                                    mean electron density (the leapfrog of eqs. 1-4 is
                                    unstable for the plasma oscillation) */
    PIC_ERR_OVERFLOW = -6,       /* a capacity above 2^31 - 1 particles per species: the int64
                                    fixed-point charge of a node (2^32 units per particle)
                                    could overflow */
    PIC_ERR_STATE = -7,          /* call out of order (e.g. step before init), or a device
                                    error bit was seen; the context then refuses every call */
    PIC_ERR_CAPACITY = -8        /* particle count exceeds buffer capacity */
} pic_status;
/* Not an error: a particle that drifts farther from its tile than the
 * deposit halo between two re-binnings adds its charge with global atomics
 * instead of the tile's LDS window (same integers; counted in
 * pic_diag.deposit_fallbacks).  Class-8 removals (non-finite or runaway
 * displacements) are tallied, not reported as errors. */

#define PIC_MAX_COND 8           /* conductor ids 1..7; 0 = plasma / free */
#define PIC_NCLASS 9             /* hit classes, see pic_diag */
#define PIC_IAD_BINS 90          /* ion angular distribution bins (2 degrees each) */

typedef struct {
    int32_t nx, ny;              /* cells along x (plate normal) and y */
    int32_t periodic_x, periodic_y;
    double dt;                   /* time step (Sec. III.A: 0.1) */
    const uint8_t *cell_cond;    /* host nx*ny: 0 plasma, k>0 solid conductor k; copied */
    int32_t edge_cond[4];        /* conductor of the x-low, x-high, y-low, y-high edges (bounded axes) */
    double v_amp[PIC_MAX_COND];  /* V_k(t) = v_amp[k] * sin(v_omega[k] * t)  (Sec. III.B) */
    double v_omega[PIC_MAX_COND];
    double weight;               /* density carried by one particle (1/ppc, n_0 units) */
    double alpha[2];             /* eqs. (1)-(2): species 0 electrons (-1), 1 ions (m_e/m_i) */
    int32_t box_i_top, box_j_lo, box_j_hi; /* trench box (cells) for hit classes 4..7 */
    int32_t charge_mode;         /* 0 none, 1 static extra ion density, 2 accumulate ion bottom hits */
    int32_t charge_row;          /* node row receiving the build-up charge */
    double static_density;       /* mode 1: extra n_i on charge_row, static_j_lo..static_j_hi */
    int32_t static_j_lo, static_j_hi;
    double rtol;                 /* relative residual ||b - A phi|| / ||b|| of the solve */
    int32_t max_iter;            /* cap on iterations per solve (CG iterations, or sweeps) */
    int32_t solver;              /* 0 multigrid-preconditioned CG, 1 plain CG, and the paper's own
                                    iterations (Sec. II) in float64: 2 Jacobi sweeps, 3 red-black
                                    Gauss-Seidel sweeps (a periodic axis needs an even node count);
                                    a batch mixes no CG and sweep instances, and pic_batch_step
                                    needs CG */
    int32_t sort_interval[2];    /* steps between re-binnings per species (0 = at init only) */
    int32_t tile_x, tile_y;      /* particle tile in cells (powers of two; 0 = 16) */
    int32_t halo;                /* cells of drift a tile absorbs before a global fallback (0 = 4) */
    int32_t chunk;               /* particles per thread block (0 = 8192; at most 8192) */
    int32_t push_unroll;         /* particles per thread per pass of the push loop: 1, 2, 4 (0 = 4;
                                    4 moves 4 consecutive particles with 16-byte accesses) */
    int32_t push_merge;          /* distinct cells summed per wavefront before LDS atomics: 0, 2, 4 */
    int64_t hitlog_capacity;     /* ring of wall-hit records in the workspace (0 = none) */
    int32_t hitlog_species_mask; /* bit s logs species s */
    int32_t warm_start;          /* start of pic_step's solves: 0 previous phi, 1 linear extrapolation */
    /* ion recycling (Sec. III.A, III.C): an ion removed at a wall or conductor
     * (classes 0..7) is replaced in the same slot, within the same pic_push,
     * by a thermal ion in a cell of the bulk rows 0 .. recycle_rows-1 (which
     * must hold no solid cell): cell, offsets and Gaussian velocity from
     * Philox4x32-10 with key recycle_key, counter (step, bits of the lost
     * ion's v_x after the kick, bits of its offsets before the move).
     * 0 = off. */
    int32_t recycle_rows;
    uint32_t recycle_key[2];
    double recycle_vth;          /* Gaussian sigma of each velocity component of a new ion */
    /* secondary electron emission at the trench surfaces (Sec. IV names it as
     * future work, through ion and through electron bombardment, and gives no
     * yield model; the reading here is a constant yield per impact).  A
     * particle of species s removed at the trench bottom or a sidewall
     * (classes 4, 6, 7) frees one electron with probability see_yield[s]:
     * the electron starts in the cell the particle last occupied, on the
     * struck face (offset along it uniform), with a flux-weighted
     * half-Maxwellian of thermal speed see_vth away from the wall (normal
     * speed see_vth sqrt(-2 ln u), tangential velocity Gaussian), taken as
     * the half-step velocity of the step that freed it.  Draws: Philox4x32-10
     * with key see_key, counter (step, packed cell, bits of the removed
     * particle's kicked velocity); emitted iff (r0 >> 8) < floor(yield 2^24).
     * The new electrons are appended to species 0 (up to its capacity; the
     * excess is counted in pic_diag.see_dropped) within the same pic_push,
     * their charge added to rho[0], and pushed from the next step on.  The
     * emission reads the removals from the hit ring, so hitlog_capacity must
     * hold one step's removals of the logged species (at least 65536) and
     * hitlog_species_mask must log every species with a yield > 0.
     * 0 = off. */
    double see_yield[2];         /* electrons freed per impact of species s (0 .. 1) */
    double see_vth;              /* thermal speed of the emitted electrons (> 0 with a yield) */
    uint32_t see_key[2];
} pic_config;

typedef struct {
    int64_t capacity;            /* slots in each storage set */
    int64_t count;               /* particles loaded in set 0 at pic_init */
    int32_t *cell[2];            /* device, two storage sets (re-binning ping-pong) */
    float *ox[2], *oy[2], *vx[2], *vy[2];
} pic_species_buffers;

typedef struct {
    pic_species_buffers sp[2];   /* 0 electrons, 1 ions */
    int64_t *rho[2];             /* device NX*NY per species: charge of the current positions */
    double *phi;                 /* device NX*NY potential (float64) */
    double *b;                   /* device NX*NY right-hand side; Dirichlet nodes hold V(t) */
    void *workspace;             /* device, pic_workspace_size bytes, 256-byte aligned */
    size_t workspace_bytes;
} pic_buffers;

typedef struct {
    int32_t iterations;          /* preconditioned CG iterations (one V-cycle each) */
    int32_t outer;               /* float64 refinement passes */
    int32_t converged;
    int32_t iterations_first;    /* of those, the iterations of the first refinement pass */
    double relres0;              /* relative residual of the start */
    double relres;               /* final relative residual (float64) */
    int32_t unconverged_pushes;  /* since pic_init: pushes whose potential had not met rtol
                                    (its last residual test failed) */
    int32_t pad;
    double worst_relres;         /* the largest relative residual among those pushes (0 if none) */
} pic_solve_info;

typedef struct {
    int64_t step;                /* completed pushes */
    double t;                    /* step * dt */
    int64_t alive[2];            /* particles per species: loaded minus removals not recycled */
    int64_t loaded[2];
    int64_t charge[2];           /* sum of rho over all nodes (2^-32 particle units / 2^32) */
    int64_t tally[2][PIC_NCLASS];/* removals: class = direction (0 +x, 1 -x, 2 +y, 3 -y)
                                    + 4 inside the trench box; 8 = non-finite/runaway */
    int64_t surf_hits;           /* ions absorbed by the trench bottom (charge mode 2 sum) */
    int64_t hits_logged;         /* records written to the hit ring (total) */
    int64_t deposit_fallbacks;   /* particles deposited outside their tile window */
    pic_solve_info last_solve;
    double kinetic[2];           /* 0.5 (m_s/m_e) w sum(v_x^2 + v_y^2) over live particles
                                    (n_0 T_e per unit area; leapfrog velocities v^{n-1/2}) */
    double field_energy;         /* 0.5 sum over nodes of |E|^2 (node field of the current phi) */
    int64_t iad[PIC_IAD_BINS];   /* ions absorbed by the trench bottom per 2-degree bin of the
                                    impact angle atan2(v_y, v_x) in [-90, 90) degrees (Sec. III.C) */
    int64_t see_emitted;         /* secondary electrons appended so far (counted in alive[0]) */
    int64_t see_dropped;         /* freed electrons beyond species 0's capacity, plus removal records
                                    overwritten in the hit ring before the emission read them */
} pic_diag;

typedef struct {
    int32_t species_class;       /* species << 8 | class */
    int32_t cell;                /* packed code of the last cell occupied */
    float vx, vy;                /* velocity at the hit */
    int32_t step;                /* step index of the push */
    int32_t pad;
} pic_hit;

/* Bytes of device workspace a configuration needs for the given per-species
 * particle capacities.  Pure host computation; validates the configuration.
 * capacity: host int64[2]. */
pic_status pic_workspace_size(const pic_config *cfg, const int64_t *capacity, size_t *bytes);

/* Validates the configuration, derives the Dirichlet node map from the cell
 * conductor map (Sec. II boundary conditions), builds the multigrid
 * hierarchy, bins the loaded particles of set 0 into tiles and deposits
 * them (state: t = 0, rho and b valid, phi Dirichlet nodes set).  The
 * caller must have copied particles into set 0 of each species and zeroed
 * nothing else.  stream: a hipStream_t (NULL = default stream). */
pic_status pic_init(const pic_config *cfg, const pic_buffers *buf, void *stream, pic_ctx **out);

/* Re-deposits every live particle (area weighting) into rho and assembles b
 * at the current time (eq. 5 source plus Dirichlet lifts and build-up
 * charge).  Idempotent; needed only after particles were changed outside. */
pic_status pic_deposit(pic_ctx *ctx);

/* Solves eq. (5) for phi from b.  guess_kind 0: start from zero on the free
 * nodes; 1: from the current phi (previous step); 2: from the device float64
 * array guess (NX*NY, free nodes used); 3: from 2 phi - phi_prev, the linear
 * extrapolation of the last two kind-3 or kind-4 solutions (the current phi
 * on the first call); 4: from guess as kind 2, keeping the time history of
 * kind 3 (the current phi becomes phi_prev first).  Kinds 2 and 4 need a
 * single instance.  Waits for the stream.  info may be NULL.  Returns
 * PIC_ERR_NOT_CONVERGED (phi written) at max_iter. */
pic_status pic_solve(pic_ctx *ctx, int32_t guess_kind, const double *guess, pic_solve_info *info);

/* Leapfrog start: v <- v - (alpha dt / 2) E(x) with E from the current phi
 * (velocities become v^{-1/2}).  Call once after the first pic_solve. */
pic_status pic_rewind(pic_ctx *ctx);

/* One push of both species with the field of the current phi (eqs. 1-4),
 * wall/conductor absorption and classification, deposit of the new
 * positions, t += dt, assembly of b at the new time, and re-binning when the
 * species' sort interval is due. */
pic_status pic_push(pic_ctx *ctx);

/* nsteps x (pic_solve started as cfg.warm_start selects; pic_push).  Stops
 * at the first failing solve and returns its status.  A re-binning that falls
 * due inside the loop runs on a stream the library owns (default priority),
 * beside the next step's solve; the next push waits for it, and on return
 * the context's stream is ordered after it (no host wait), so work the caller
 * queues on that stream, particle reads included, sees the re-binned state. */
pic_status pic_step(pic_ctx *ctx, int32_t nsteps);

/* Waits for the stream and copies counters to the host. */
pic_status pic_diagnostics(pic_ctx *ctx, pic_diag *out);

/* Which storage set (0/1) currently holds species s and how many slots of it
 * are in use (live particles first after a re-binning).  Waits. */
pic_status pic_particles(pic_ctx *ctx, int32_t species, int32_t *set, int64_t *slots);

/* Copies up to max of the most recent wall-hit records (oldest first) into
 * host memory out; *n receives the number copied.  Waits. */
pic_status pic_read_hits(pic_ctx *ctx, pic_hit *out, int64_t max, int64_t *n);

/* Changes the schedule of a running context (all instances): the push
 * variant (push_unroll 1, 2 or 4; push_merge 0, 2 or 4, as in pic_config)
 * and the re-binning intervals of electrons and ions (steps; 0 = never).
 * Results do not depend on any of them (integer deposit, independent
 * particles); only the time per step does.  Waits for the stream and drops
 * the captured step graphs. */
pic_status pic_tune(pic_ctx *ctx, int32_t push_unroll, int32_t push_merge, int32_t sort_e,
                    int32_t sort_i);

/* Chooses whether the fine multigrid levels below level 0 run two per launch
 * (on = 1, the default: one block per tile of the coarser level recomputes
 * the finer one on the window it needs) or one per launch (on = 0).  The
 * paired kernels perform the same operations in the same order, so the
 * potential is the same bit for bit; only the time per iteration differs.
 * Waits for the stream and drops every captured graph.  PIC_ERR_ARG for on
 * outside {0, 1}. */
pic_status pic_set_level_pairs(pic_ctx *ctx, int32_t on);

/* Re-bins species s now (tile sort; drops removed particles). */
pic_status pic_sort(pic_ctx *ctx, int32_t species);

/* Average device time per launch of the push kernel over the pushes since
 * the last call, measured with HIP events on the library stream (ms), and
 * the number of particles it processed per launch.  Resets the counters. */
pic_status pic_push_timing(pic_ctx *ctx, double *avg_ms, double *avg_particles, int32_t *launches);

/* Enables or disables HIP event timing of the push kernels (default off). */
pic_status pic_set_timing(pic_ctx *ctx, int32_t on);

/* ---- batched form: several independent instances (e.g. a sweep of trench
 * widths, Sec. III.C) advanced together; every kernel launch covers all of
 * them.  Instances may differ in grid size, geometry and particle count but
 * share one push variant (push_unroll, push_merge) and the sort intervals
 * of instance 0.  The single-instance calls above act on every instance of
 * a batch (pic_solve / pic_step converge every instance; pic_diagnostics,
 * pic_particles and pic_read_hits report instance 0). */

/* Workspace bytes for n (1..16) instances; capacity: host int64[2 n]. */
pic_status pic_batch_workspace_size(int32_t n, const pic_config *cfgs, const int64_t *capacity,
                                    size_t *bytes);

/* As pic_init for n instances: cfgs[n], bufs[n] (their workspace fields are
 * ignored), one caller-owned workspace of pic_batch_workspace_size bytes. */
pic_status pic_batch_init(int32_t n, const pic_config *cfgs, const pic_buffers *bufs,
                          void *workspace, size_t workspace_bytes, void *stream, pic_ctx **out);

/* nsteps steps of every instance as captured HIP graphs, one launch per
 * re-binning period of species 0 (its sort_interval, or 8; at most 510
 * steps, the device window of conductor potentials): each step solves
 * from the extrapolated potential with a fixed schedule of `passes`
 * float64 refinement passes, the first of `iters` preconditioned CG
 * iterations and the later ones of `iters_later` (0: `iters`), every
 * instance leaving the schedule as soon as it meets its rtol, then pushes.
 * Waits at the end; per-instance results in pic_batch_solve_info.  Returns
 * PIC_ERR_NOT_CONVERGED (after all nsteps ran) when any step of any
 * instance pushed a potential whose last residual test failed, i.e. the
 * schedule was too short for it (pic_solve_info.unconverged_pushes counts
 * them).  If no earlier extrapolated solve exists, the first step runs as
 * pic_step(1).  nsteps = 0 does nothing. */
pic_status pic_batch_step(pic_ctx *ctx, int32_t nsteps, int32_t passes, int32_t iters, int32_t iters_later);

/* Per-instance counters, particle set and last solve (i in 0..n-1). */
pic_status pic_batch_diagnostics(pic_ctx *ctx, int32_t i, pic_diag *out);
pic_status pic_batch_particles(pic_ctx *ctx, int32_t i, int32_t species, int32_t *set, int64_t *slots);
pic_status pic_batch_solve_info(pic_ctx *ctx, int32_t i, pic_solve_info *out);

/* Node map of instance i (NX*NY bytes: 0 free node, k > 0 Dirichlet node
 * held by conductor k; the boundary conditions of Sec. II).  node_cond
 * receives the device copy, owned by the context and valid until
 * pic_destroy; host_copy (caller memory of NX*NY bytes) receives a host
 * copy; NX and NY receive the node counts.  Every output may be NULL.  No
 * device work. */
pic_status pic_node_map(pic_ctx *ctx, int32_t i, const uint8_t **node_cond, uint8_t *host_copy,
                        int32_t *NX, int32_t *NY);

/* For tests of the error path only: what = 1 moves the device step counter
 * past the window of conductor potentials, as a runtime that lost track of
 * it would.  The next assembly (pic_push, pic_deposit) sets the device
 * error bit instead of reading outside the table, the next call that looks
 * at the device flags (pic_solve, pic_step, pic_batch_step,
 * pic_diagnostics) returns PIC_ERR_STATE, and every later call does too. */
pic_status pic_inject_fault(pic_ctx *ctx, int32_t what);

/* Waits for the context's stream and the library's own streams, then frees
 * the context's host objects and graphs.  The caller frees the buffers and
 * workspace it passed in afterwards.  NULL is ignored. */
void pic_destroy(pic_ctx *ctx);
const char *pic_last_error(const pic_ctx *ctx);
const char *pic_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PIC_H */
