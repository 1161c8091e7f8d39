/*
 * lbdps.h - C ABI of the MI355X (gfx950) library for the lattice-Boltzmann-based
 * discrete particle simulation of gas-solid fluidization (Wang, Zhang, Wang, Ge
 * & Li, Chem. Eng. Sci.).
 *
 * One library call advances the coupled method of Sec. 2.4 (the seven-step
 * procedure): particle statistics per cell (Eqs. 8, 10, 11), the modified
 * lattice Boltzmann collision and streaming (Eqs. 7, 9, 23-25), EMMS drag with
 * bilinear grid-to-particle interpolation and the Newton-third-law correction
 * (Eqs. 19-22, 26-28), integration of the particle equation of motion (Eq. 16)
 * and the time-driven hard-sphere collisions (Eqs. 17-18).
 *
 * Conventions
 *  - Lattice units: cell size h = 1, time step dt = 1 (Sec. 2.1).
 *  - Every function returns lbdps_status (0 = OK, < 0 = error).  Nothing throws
 *    or aborts across the ABI.  lbdps_last_error() returns a thread-local
 *    message for the last failure on the calling thread.
 *  - Pointers named d_* are device pointers (HIP device memory of the GPU the
 *    context was created on); h_* are host pointers.  The library never
 *    allocates device memory: the caller passes one workspace buffer of
 *    lbdps_workspace_bytes() bytes that must outlive the context.  Host-side
 *    context memory is allocated by lbdps_create and freed by lbdps_destroy.
 *    No pointer passed in is kept after a call returns, except the workspace.
 *  - Boundary layouts are canonical FP64 whatever the internal precision:
 *    populations f as [9][ny][nx] (direction-major, D2Q9 numbering below),
 *    node fields as [ny][nx] (vectors [ny][nx][2]), particles as [n][2] in
 *    particle-index order.  Internal layouts are private.
 *  - D2Q9 numbering: 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1)
 *    6:(-1,1) 7:(-1,-1) 8:(1,-1); weights 4/9, 1/9 (1-4), 1/36 (5-8).
 *  - Work is enqueued on the stream given to lbdps_create (a hipStream_t passed
 *    as void*).  lbdps_step returns without waiting.  The calls documented
 *    as synchronising (lbdps_get_*, lbdps_conservation, lbdps_counters,
 *    lbdps_diag_last, lbdps_count_histogram, lbdps_outlet_crossings, ...)
 *    enqueue their copies on the same stream and wait for it; device-side
 *    errors latched since the last such call (a particle outside the domain,
 *    a contact row over its capacity, a stalled sweep, a non-finite value
 *    found by the periodic check) are returned by them.
 *  - A context is not thread-safe; separate contexts are independent.
 */
#ifndef LBDPS_H
#define LBDPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBDPS_OK = 0,
  LBDPS_E_INVALID = -1,     /* a parameter or input value is out of range      */
  LBDPS_E_SHAPE = -2,       /* a size does not match the context or workspace   */
  LBDPS_E_DEVICE = -3,      /* a HIP runtime call failed                        */
  LBDPS_E_UNSUPPORTED = -4, /* valid for the method, not supported by this library */
  LBDPS_E_NONFINITE = -5,   /* a NaN or infinity appeared in the state           */
  LBDPS_E_CAPACITY = -6,    /* a particle has more contacts than LBDPS_MAX_CONTACTS */
  LBDPS_E_STALL = -7        /* collision resolution exceeded its bounded wait    */
} lbdps_status;

/* Storage and arithmetic precision of a context. */
typedef enum {
  LBDPS_FP64 = 0,            /* FP64 storage and arithmetic                      */
  LBDPS_FP32 = 1,            /* populations stored as FP32 deviations f_i - w_i, FP32 arithmetic */
  LBDPS_FP32_STORE_FP16 = 2, /* populations stored as FP16 deviations f_i - w_i, FP32 arithmetic */
  LBDPS_FP32_STORE_BF16 = 3  /* populations stored as BF16 deviations f_i - w_i, FP32 arithmetic */
} lbdps_precision;

/* Boundary type of a lattice face.  x faces take PERIODIC or WALL; y faces take
 * any.  PERIODIC must be set on both faces of an axis.  Particles see a wall on
 * every non-periodic face (unless lbdps_params.particles_periodic_y). */
typedef enum {
  LBDPS_BC_PERIODIC = 0,
  LBDPS_BC_WALL = 1,  /* halfway bounce-back for the gas; particle walls           */
  LBDPS_BC_INLET = 2, /* incoming populations set to f^eq(1, (0, u_in(x)))         */
  LBDPS_BC_OUTLET = 3 /* incoming populations copied from the boundary row         */
} lbdps_bc;

/* Largest number of particle sub-steps per lattice step (lbdps_params.n_sub). */
#define LBDPS_MAX_SUBSTEPS 64

/* Contacts recorded per particle; a particle with more is an LBDPS_E_CAPACITY error. */
#define LBDPS_MAX_CONTACTS 32

typedef struct {
  int32_t nx, ny;            /* lattice size, nx, ny >= 3, nx * ny < 2^29            */
  int32_t bc[4];             /* lbdps_bc of faces x-, x+, y-, y+                       */
  double tau;                /* relaxation time, tau = 3 nu + 1/2 (Eq. 3), > 0.5      */
  double rho_g;              /* gas density in the drag laws (Eqs. 19, 22), > 0       */
  double rho_s;              /* solid density, > 0; particle mass rho_s pi d^3/6      */
  double d_p;                /* particle diameter in cells, 0 < d_p < 1               */
  double e_pp;               /* particle-particle restitution e of Eqs. 17-18, [0, 1]  */
  double e_pw;               /* particle-wall restitution, [0, 1]                      */
  double g[2];               /* gravity on particles; the (1 - rho_g/rho_s) factor of
                                Sec. 3 is applied by the library                       */
  double body_force[2];      /* force per cell on the gas (drives periodic beds)      */
  int32_t drag_ratio_mode;   /* Eq. 28: 0 signed ratio F_pg/F_pre (default), 1 ratio of
                                absolute values as printed, 2 signed ratio with F_pg
                                split equally among the cell's particles where their
                                pre-drags cancel (sum |F_pre| > 100 |sum F_pre|; not in
                                the paper: keeps dense beds stable over long runs)     */
  int32_t u_gas_porosity;    /* superficial -> actual gas velocity (after Eq. 24):
                                0 divide by eps_2d (default), 1 by the 3-D voidage, 2 none */
  int32_t omega_mode;        /* 0 EMMS correction of Eq. 20 (default), 1 omega = 1 (Eq. 6) */
  int32_t pressure_force_sign; /* sign s of the s V_p grad p term of Eq. 16: -1 (default), 0, +1 */
  double omega_dense;        /* omega used where eps_g <= 0.74 (Eq. 20 undefined), default 1 */
  double cs_smag;            /* Smagorinsky constant C_s of Eqs. 12-15 (>= 0); 0 = plain BGK     */
  int32_t precision;         /* lbdps_precision                                        */
  int32_t diagnostics;       /* 1: each step also records per-cell n, v_s and per-particle
                                drag for lbdps_get_fields / lbdps_get_particles          */
  int32_t n_sub;             /* particle sub-steps per lattice step, 0..LBDPS_MAX_SUBSTEPS
                                (0 and 1: one).  The drag, pressure and gravity
                                accelerations of Eq. 16 are taken once per lattice step
                                and held; each sub-step of length 1/n_sub integrates
                                Eq. 16 and runs the collision stage (Sec. 2.2, time-driven
                                hard spheres at the finer interval).  lbdps_counters and
                                lbdps_get_pairs then describe the last sub-step.  Batched
                                beds (lbdps_batch_*) take one: LBDPS_E_UNSUPPORTED else */
  int32_t particles_periodic_y; /* 1: particles leaving through a non-periodic y face re-enter
                                   at the opposite one, with no particle wall there (the
                                   circulating loop of the riser, Sec. 3.2); the gas keeps its
                                   faces.  0 (default): particles follow the gas faces */
  int32_t diag_every;        /* > 0: after every diag_every-th step lbdps_step also enqueues
                                the FP64 conservation sums (as lbdps_conservation) and
                                latches a non-finite value in populations or velocities,
                                reported as LBDPS_E_NONFINITE by the next synchronising
                                call; lbdps_diag_last returns the latest sums.  0 (default):
                                off.  Batched beds: LBDPS_E_UNSUPPORTED if > 0 */
} lbdps_params;

typedef struct lbdps_ctx lbdps_ctx;

/* Check parameters without touching any device.  0 <= max_particles < 2^29 (arrays
 * are addressed by 32-bit byte offsets); LBDPS_E_SHAPE otherwise. */
lbdps_status lbdps_validate_params(const lbdps_params *p, int64_t max_particles);

/* Workspace size for a context holding up to max_particles particles.  Device-free. */
lbdps_status lbdps_workspace_bytes(const lbdps_params *p, int64_t max_particles, size_t *bytes);

/*
 * Create a context on the current HIP device.  d_workspace: device buffer of at
 * least lbdps_workspace_bytes() bytes, 256-byte aligned.  h_inlet_uy: host array
 * of nx inlet velocities (y component) used by INLET faces, or NULL for zero.
 * stream: hipStream_t for all work of this context (NULL = default stream).
 * The state starts as f = f^eq(1, 0) and no particles.
 */
lbdps_status lbdps_create(const lbdps_params *p, int64_t max_particles, void *d_workspace, size_t bytes,
                          const double *h_inlet_uy, void *stream, lbdps_ctx **out);

/*
 * Replace the state.  d_f: device [9][ny][nx] FP64 pre-collision populations,
 * or NULL for f^eq(1, 0) everywhere.  d_pos, d_vel: device [n][2] FP64 particle
 * centres in [0, nx) x [0, ny) and velocities, particle index order (the index
 * orders the collisions, Eqs. 17-18).  n <= max_particles.  Positions outside
 * the domain are reported as LBDPS_E_INVALID by the next synchronising call.
 * In reduced precisions values are rounded to the internal representation.
 */
lbdps_status lbdps_set_state(lbdps_ctx *ctx, const double *d_f, const double *d_pos, const double *d_vel,
                             int64_t n);

/* Enqueue nsteps coupled time steps (Sec. 2.4, steps 2-6 each).  Asynchronous. */
lbdps_status lbdps_step(lbdps_ctx *ctx, int32_t nsteps);

/*
 * Enqueue the hard-sphere stage alone on the current state: contact detection
 * at the present positions and binary plus wall collisions (Eqs. 17-18).  This is
 * the last stage of every step; exposed for stage-by-stage checks.  Asynchronous.
 */
lbdps_status lbdps_collide_particles(lbdps_ctx *ctx);

/*
 * Node fields of the most recent step, device FP64 [ny][nx] (vectors [ny][nx][2]):
 * density rho (Eq. 5), actual gas velocity (Eq. 24 and the note after it),
 * force on the gas F_p->g (Eq. 25), drag coefficient beta (Eq. 19).  With
 * diagnostics on, also the particle count n_tot (int32) and mean solid
 * velocity v_s (Eq. 8) per cell used by that step.  Any pointer may be NULL.
 * Synchronises the stream.
 */
lbdps_status lbdps_get_fields(lbdps_ctx *ctx, double *d_rho, double *d_ugas, double *d_fpg, double *d_beta,
                              int32_t *d_ncell, double *d_vs);

/*
 * Particle state in index order, device FP64 [n][2]: positions, velocities, and
 * (diagnostics on) the corrected drag of the most recent step (Eq. 28); d_cell
 * receives the int32 [n][2] cell of each particle.  Any pointer may be NULL.
 * Synchronises the stream.
 */
lbdps_status lbdps_get_particles(lbdps_ctx *ctx, double *d_pos, double *d_vel, double *d_fd, int32_t *d_cell);

/*
 * Acceleration of Eq. 16 taken by each particle in the most recent step,
 * device FP64 [n][2] in particle-index order:
 *   a = g_eff + (F_d + s V_p grad p_k) / m,
 * computed in the context's arithmetic; the integration then takes
 * v <- v + a h (h = 1 / n_sub) before the hard-sphere stage, so with one
 * sub-step the velocity entering that stage is the previous velocity plus a.
 * Held with diagnostics on (or n_sub > 1); LBDPS_E_INVALID otherwise.
 * Synchronises the stream.
 */
lbdps_status lbdps_get_accel(lbdps_ctx *ctx, double *d_acc);

/*
 * Contact pairs (i, j), i < j by particle index, at the current positions
 * (after a step: those of its last hard-sphere stage, since positions do not
 * change after it), in lexicographic order, device int32 [cap][2] (Sec. 2.2:
 * centres at most d_p apart).  *n_out receives the number of pairs (also when
 * it exceeds cap; then only cap are written).  Synchronises the stream.
 */
lbdps_status lbdps_get_pairs(lbdps_ctx *ctx, int32_t *d_pairs, int64_t cap, int64_t *n_out);

/* Checkpoint: FP64 populations [9][ny][nx], positions and velocities [n][2]
 * (index order) and the step counter.  Any pointer may be NULL.  Synchronises. */
lbdps_status lbdps_get_state(lbdps_ctx *ctx, double *d_f, double *d_pos, double *d_vel, int64_t *h_step);

/*
 * FP64 conservation sums over the current state, fixed-order reductions:
 * h_out[0] = sum of f (mass), h_out[1..2] = sum c_i f_i (gas momentum),
 * h_out[3..4] = sum m v (particle momentum), h_out[5] = 1 if any value is not
 * finite, else 0.  Returns LBDPS_E_NONFINITE in that case.  Synchronises.
 */
lbdps_status lbdps_conservation(lbdps_ctx *ctx, double h_out[6]);

/*
 * lbdps_conservation without any scratch of the context's: for callers that
 * cannot allocate device memory or must not touch more of it (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation).  The
 * same kernels and the same fixed-order sums, so h_out equals lbdps_conservation's
 * bit for bit; the reduction's partial sums, outputs and flag live in one
 * library-static device array per GPU (about 21 KB, held until the process
 * ends).  Its size does not depend on the bed (the reduction always runs on
 * the same fixed grid), so every context fits.  Allocates nothing.  Calls
 * that overlap on one GPU (contexts on different streams, or threads) share
 * that array and race: serialise them.  Returns LBDPS_E_NONFINITE as
 * lbdps_conservation does.  Synchronises the stream.
 */
lbdps_status lbdps_conservation_noalloc(lbdps_ctx *ctx, double h_out[6]);

/*
 * The sums of the latest periodic check (lbdps_params.diag_every > 0), in
 * lbdps_conservation's layout, and the step after which it ran (*h_step; -1
 * and zeros if none ran since the context was created or its state was last
 * set).  Synchronises the stream.
 */
lbdps_status lbdps_diag_last(lbdps_ctx *ctx, double h_out[6], int64_t *h_step);

/*
 * Event counts of the most recent hard-sphere stage: h_out[0] contact pairs,
 * h_out[1] pairs that collided, h_out[2] particle-wall collisions, h_out[3]
 * (diagnostics on) cell components with a zero Eq. 28 denominator in the most
 * recent drag.  Synchronises.
 */
lbdps_status lbdps_counters(lbdps_ctx *ctx, int64_t h_out[4]);

/*
 * Outlet solids flux (Sec. 3.2, the solids flux at the riser's outlet): the
 * net number of particles that crossed the outlet plane y = ny upward since
 * the previous call (or since lbdps_set_state), and the number of steps taken
 * meanwhile.  A crossing is counted in the move of Eq. 16 (every sub-step)
 * where a particle periodic in y (lbdps_params.particles_periodic_y, the
 * circulating loop, or a y-periodic bed) ends at or beyond y = ny (+1, it
 * re-enters at the bottom) or below y = 0 (-1); with particle walls in y
 * nothing crosses.  The solids mass flux through the outlet is then
 *   G_s = m h_net / (nx h_steps),  m = rho_s pi d^3 / 6,
 * mass per unit width (unit depth) per unit time in lattice units.
 * Synchronises the stream.
 */
lbdps_status lbdps_outlet_crossings(lbdps_ctx *ctx, int64_t *h_net, int64_t *h_steps);

/*
 * Replace the inlet profile used by INLET faces (Sec. 3.1: the gas pulse of the
 * bubble experiment is switched off this way).  h_inlet_uy: host array of nx
 * finite y velocities, read before return.  Waits for the context's queued work
 * first, so steps already enqueued keep the old profile.  LBDPS_E_INVALID for a
 * NULL array or a non-finite value.
 */
lbdps_status lbdps_set_inlet(lbdps_ctx *ctx, const double *h_inlet_uy);

/*
 * Voidage statistics of the current particle positions (Sec. 3: the equivalent
 * bubble diameter of Sec. 3.1 and the time-averaged voidage profiles of
 * Sec. 3.2).  The gas voidage of a cell is the 3-D voidage of Eq. 11 for the
 * cell's particle count, eps_g = 1 - eps_s,3d, as the drag laws see it.
 *   d_row_sum: device [ny] FP64, or NULL.  Row j gets += sum over x of eps_g.
 *   d_col_sum: device [nx] FP64, or NULL.  Column i gets += sum of eps_g over
 *              rows y0 .. y1-1.  Both accumulate, for time averages.
 *   d_count:   device int64, or NULL.  Set (=) to the number of cells in rows
 *              y0 .. y1-1 whose eps_g exceeds threshold; the equivalent bubble
 *              diameter is sqrt(4 count / pi) cells.
 * Sums run in a fixed order.  0 <= y0 <= y1 <= ny and a finite threshold, else
 * LBDPS_E_INVALID.  Asynchronous (stream order).
 */
lbdps_status lbdps_voidage(lbdps_ctx *ctx, int32_t y0, int32_t y1, double threshold, double *d_row_sum,
                           double *d_col_sum, int64_t *d_count);

/*
 * Histogram of particles per cell at the current positions (metrics of the
 * deposition: the count at which the solid fraction of Eq. 10 reaches its
 * clamp, and the one from which eps_g <= 0.74 selects the dense branch of
 * Eq. 19, follow from d_p).  h_hist[b], b < nbins - 1: cells holding exactly
 * b particles; h_hist[nbins - 1]: cells holding nbins - 1 or more.
 * nbins in [2, 256], else LBDPS_E_INVALID.  Synchronises.
 */
lbdps_status lbdps_count_histogram(lbdps_ctx *ctx, int64_t *h_hist, int32_t nbins);

/*
 * The 3-D gas lattice, first piece of the 3-D extension (the paper names 3-D
 * as future work): one BGK collide-stream step (the 3-D form of Eqs. 2-3, no
 * particles) of the D3Q19 lattice on a periodic nx x ny x nz box.  D3Q19: the
 * rest velocity (weight 1/3), the 6 face neighbours (1/18) and the 12 edge
 * neighbours (1/36) in the order rest, +x, -x, +y, -y, +z, -z, (+x+y),
 * (-x-y), (+x-y), (-x+y), (+x+z), (-x-z), (+x-z), (-x+z), (+y+z), (-y-z),
 * (+y-z), (-y+z); f^eq of Eq. 4 with c_s^2 = 1/3.
 *   d_fin, d_fout: distinct device buffers [19][nz][ny][nx] in the storage of
 *   precision (lbdps_precision): FP64 values, or the deviations f_i - w_i as
 *   FP32, FP16 or BF16 with FP32 arithmetic.  The caller owns both.
 *   tau > 0.5.  stream: hipStream_t (NULL = default).  Asynchronous.
 * LBDPS_E_INVALID for NULL or equal buffers, a bad tau or precision;
 * LBDPS_E_SHAPE for a dimension below 1.
 */
lbdps_status lbdps3_bgk_step(const void *d_fin, void *d_fout, int32_t nx, int32_t ny, int32_t nz, double tau,
                             int32_t precision, void *stream);

/*
 * The 3-D lattice with solids in its cells, second piece of the 3-D
 * extension: one collide-stream step of the D3Q19 lattice above on a
 * periodic box with the partially saturated collision of Eqs. 6-7, its
 * weighting gamma of Eq. 9 and the solids' force of Eq. 25, with the solids
 * given per cell (the deposition of Eq. 8 done by the caller):
 *   eps_s = min(n pi d^3 / 6, pi / (3 sqrt 2))   (h = 1; the densest sphere
 *           packing bounds it as the densest disc packing bounds Eq. 10)
 *   Om_i  = f_opp(i) - f_i + f^eq_i(rho, v_s) - f^eq_opp(i)(rho, u)
 *   f*_i  = f_i - (1 - gamma) / tau (f_i - f^eq_i(rho, u)) + gamma Om_i
 *   F     = gamma sum_i c_i Om_i, then push streaming with periodic wrap.
 *   d_fin, d_fout: as for lbdps3_bgk_step.
 *   d_n:     device [nz][ny][nx] int32, spheres per cell (>= 0).
 *   d_vs:    device [3][nz][ny][nx], their mean velocity (x plane, y plane,
 *            z plane), FP64 for LBDPS_FP64, else FP32.
 *   d_force: device [3][nz][ny][nx], same type, receives F (=).
 *   tau > 0.5, d > 0 (sphere diameter in lattice units).  The caller owns
 *   every buffer.  Asynchronous (stream order).
 * LBDPS_E_INVALID for NULL or equal buffers, a bad tau, d or precision;
 * LBDPS_E_SHAPE for a dimension below 1.
 */
lbdps_status lbdps3_psm_step(const void *d_fin, void *d_fout, const int32_t *d_n, const void *d_vs, void *d_force,
                             int32_t nx, int32_t ny, int32_t nz, double tau, double d, int32_t precision,
                             void *stream);

/* ------------------------------------------------------------- the 3-D coupled step
 * The procedure of Sec. 2.4 on a fully periodic D3Q19 box with spheres (the
 * fully 3-D simulation the paper names as the natural extension): per cell
 * the count n and the mean velocity v_s of its spheres (Eq. 8, summed in
 * ascending particle index), the solid fraction n pi d^3 / 6 held at the
 * densest sphere packing pi / (3 sqrt 2), the voidage eps_g = 1 - eps_s,
 * gamma of Eq. 9, omega of Eq. 20 at eps_g (omega_dense where eps_g <= 0.74);
 * the collision of Eq. 23 with the solid term of Eq. 7 and the body-force
 * source 3 w_i c_i.G, F_pg of Eq. 25, the superficial velocity of Eq. 24, the
 * gas velocity u_sup / eps_g, beta of Eqs. 19, 21, 22 at eps_g; trilinear
 * interpolation (nodes at the cell centres) of u_gas, eps_s, beta and grad p
 * for Eqs. 26-28; Eq. 16 with periodic wrap; contacts |P_i - P_j| <= d and
 * the binary collisions of Eqs. 17-18 in lexicographic order.  D3Q19
 * directions and weights as for lbdps3_bgk_step.  Same conventions as the
 * 2-D context: the caller's workspace, canonical FP64 in and out, errors
 * latched on the device and returned by the next synchronising call.
 */
typedef struct {
  int32_t nx, ny, nz;         /* periodic box, each >= 3, nx ny nz < 2^28            */
  double tau;                 /* relaxation time (Eq. 3), > 0.5                      */
  double rho_g, rho_s;        /* gas density in the drag laws, solid density, > 0    */
  double d_p;                 /* sphere diameter in cells, [0.1, 1)                  */
  double e_pp;                /* restitution of Eqs. 17-18, [0, 1]                    */
  double g[3];                /* gravity on particles (the library applies 1 - rho_g/rho_s) */
  double body_force[3];       /* force per cell on the gas                           */
  double omega_dense;         /* omega where eps_g <= 0.74                           */
  int32_t pressure_force_sign; /* s of the s V_p grad p term of Eq. 16: -1, 0, +1     */
  int32_t precision;          /* lbdps_precision                                      */
  int32_t diagnostics;        /* 1: record per-cell counts, drags and accelerations   */
} lbdps3_params;

typedef struct lbdps3_ctx lbdps3_ctx;

/* Device-free checks; LBDPS_E_SHAPE for sizes out of range, LBDPS_E_INVALID else. */
lbdps_status lbdps3_validate_params(const lbdps3_params *p, int64_t max_particles);
/* Workspace size of a 3-D context for up to max_particles spheres.  Device-free. */
lbdps_status lbdps3_workspace_bytes(const lbdps3_params *p, int64_t max_particles, size_t *bytes);
/* Create on the current device with the caller's workspace (256-byte aligned)
 * and stream; the state starts as f = f^eq(1, 0), no spheres. */
lbdps_status lbdps3_create(const lbdps3_params *p, int64_t max_particles, void *d_workspace, size_t bytes,
                           void *stream, lbdps3_ctx **out);
/* Replace the state: d_f device [19][nz][ny][nx] FP64 or NULL for f^eq(1, 0);
 * d_pos, d_vel device [n][3] FP64 in particle-index order, positions in the
 * box (a position outside is reported as LBDPS_E_INVALID by the next
 * synchronising call).  Reduced precisions round to the internal storage. */
lbdps_status lbdps3_set_state(lbdps3_ctx *ctx, const double *d_f, const double *d_pos, const double *d_vel,
                              int64_t n);
/* Enqueue nsteps coupled steps.  Asynchronous. */
lbdps_status lbdps3_step(lbdps3_ctx *ctx, int32_t nsteps);
/* Canonical FP64 state: populations [19][nz][ny][nx], positions and
 * velocities [n][3] in index order.  Any pointer may be NULL.  Synchronises. */
lbdps_status lbdps3_get_state(lbdps3_ctx *ctx, double *d_f, double *d_pos, double *d_vel);
/* Node fields of the most recent step, device FP64 [nz][ny][nx] (vectors
 * [nz][ny][nx][3]): rho, u_gas, F_pg, beta, and with diagnostics the count
 * n_tot (int32).  Any pointer may be NULL.  Synchronises. */
lbdps_status lbdps3_get_fields(lbdps3_ctx *ctx, double *d_rho, double *d_ugas, double *d_fpg, double *d_beta,
                               int32_t *d_ncell);
/* With diagnostics: the corrected drag of Eq. 28 and the acceleration of
 * Eq. 16 of the most recent step, device FP64 [n][3] by particle index.
 * Synchronises. */
lbdps_status lbdps3_get_drag(lbdps3_ctx *ctx, double *d_fd, double *d_acc);
/* Contact pairs (i, j), i < j, of the most recent step in lexicographic order,
 * as lbdps_get_pairs.  Synchronises. */
lbdps_status lbdps3_get_pairs(lbdps3_ctx *ctx, int32_t *d_pairs, int64_t cap, int64_t *n_out);
/* h_out[0] contact pairs, h_out[1] pairs that collided in the most recent
 * step.  Synchronises. */
lbdps_status lbdps3_counters(lbdps3_ctx *ctx, int64_t h_out[2]);
/* Release the host context (the workspace stays the caller's). */
/* FP64 conservation sums over the current state, fixed-order reductions (the
 * invariants of the collision and coupling, Eqs. 7, 17-18, 25, 28-29):
 * h_out[0] = sum of f (mass), h_out[1..3] = sum c_i f_i (gas momentum),
 * h_out[4..6] = sum m v (particle momentum, m = rho_s pi d_p^3 / 6), h_out[7]
 * = 1 if any value is not finite, else 0; returns LBDPS_E_NONFINITE then.
 * Synchronises. */
lbdps_status lbdps3_conservation(lbdps3_ctx *ctx, double h_out[8]);
lbdps_status lbdps3_destroy(lbdps3_ctx *ctx);

/* Kernels of one step, for per-kernel timing. */
typedef enum {
  LBDPS_K_COLLIDE = 0,    /* deposition + collision + streaming                     */
  LBDPS_K_DRAG = 1,       /* drag, integration, and the per-cell count of new cells  */
  LBDPS_K_SCAN = 2,       /* prefix sum of the cell counts                           */
  LBDPS_K_SCATTER = 3,    /* particle records -> their cell's slots                  */
  LBDPS_K_CONTACTS = 4,   /* contact detection, wall collisions of contact-free particles */
  LBDPS_K_RESOLVE = 5,    /* binary collisions, then the remaining wall collisions   */
  LBDPS_K_COUNT = 6
} lbdps_kernel;

/*
 * How the most recent collision stage (Sec. 2.2, Eqs. 17-18) was split:
 * h_out[0] = particles whose contacts and collisions the tile kernel resolved
 * in LDS (sphere_tile > 0), h_out[1] = particles it left to the neighbour rows
 * (all of them with sphere_tile 0 or after a batched step).  Synchronises.
 */
lbdps_status lbdps_tile_stats(lbdps_ctx *ctx, int64_t h_out[2]);

/*
 * Time every later launch of the kernels in `mask` (bit k = lbdps_kernel k):
 * the launch carries a pair of hipEvents that its dispatch stamps at the
 * kernel's start and end (hipExtLaunchKernel), so the time is the kernel's own.
 * mask 0 stops.  For measurement only; the events belong to the context.
 */
lbdps_status lbdps_time_kernels(lbdps_ctx *ctx, uint32_t mask);

/*
 * Wait for the stream, then return per kernel the summed time in milliseconds
 * (h_ms[LBDPS_K_COUNT]) and the number of timed steps (h_launches[LBDPS_K_COUNT];
 * LBDPS_K_RESOLVE sums its two launches per step) since the previous call, and
 * reset both.
 */
lbdps_status lbdps_kernel_times(lbdps_ctx *ctx, double *h_ms, int64_t *h_launches);

/*
 * Launch shapes that do not change results (every setting gives the same
 * numbers bit for bit), only speed:
 *   cluster_lists      candidate lists of the contact kernel taken by one
 *                      workgroup of the cluster resolution, [1, 256] (default 1);
 *   cluster_groups_max most workgroups of the cluster resolution (default: no
 *                      limit);
 *   drag_tile          cells of the drag kernel's workgroup tile (its node fields
 *                      staged in LDS): 0 = 32 x 8 (default), 1 = 64 x 4,
 *                      2 = 128 x 2.  The beds of a batch share one.
 *   sphere_tile        cells of the collision stage's workgroup tile, whose
 *                      particles and the ring of cells around it are held in LDS
 *                      (contacts, clusters inside the tile resolved there, the
 *                      rest through neighbour rows): 0 = none, every particle
 *                      through the rows (default), 1 = 32 x 8, 2 = 16 x 16,
 *                      3 = 64 x 4.  A batched step takes the rows.
 * A context starts with the defaults.
 */
typedef struct {
  int32_t cluster_lists;
  int32_t cluster_groups_max;
  int32_t drag_tile;
  int32_t sphere_tile;
} lbdps_tuning;
lbdps_status lbdps_set_tuning(lbdps_ctx *ctx, const lbdps_tuning *t);
lbdps_status lbdps_get_tuning(lbdps_ctx *ctx, lbdps_tuning *t);

/* Autotuner: run `steps` steps under each candidate launch shape, twice over
 * the candidates in turn, time them with hipEvents on the context's stream and
 * keep the candidate with the fastest of its two times (written to *chosen if
 * not NULL): first the collision stage's tile shapes (4, none among them),
 * then the cluster-resolution shapes (9) and then the drag tile shapes (3),
 * each under the choices before it.  The bed advances by 2 x steps x 16.
 * Synchronises. */
lbdps_status lbdps_autotune(lbdps_ctx *ctx, int32_t steps, lbdps_tuning *chosen);

/* Release the host context (the workspace stays the caller's).  A bed of a
 * batch is released by lbdps_batch_destroy instead (LBDPS_E_INVALID here). */
lbdps_status lbdps_destroy(lbdps_ctx *ctx);

/* ---------------------------------------------------------------- batches
 * Many independent beds (uneven lattices and particle counts; each with its own
 * parameters, boundary faces and inlet profile, one precision for all) advance
 * together: each phase of the step of Sec. 2.4 is one launch for every bed.
 * Every bed is an ordinary context (lbdps_batch_bed) for set_state and the
 * get_* / conservation / counters calls; lbdps_step on it steps that bed alone.
 * Beds do not record diagnostics.  A batch is not thread-safe.
 */
typedef struct lbdps_batch lbdps_batch;

/* Workspace for a batch: two small launch tables, then each bed's workspace. */
lbdps_status lbdps_batch_workspace_bytes(const lbdps_params *beds, int32_t nbeds, const int64_t *max_particles,
                                         size_t *bytes);

/*
 * beds[nbeds], max_particles[nbeds]: as for lbdps_create, per bed.
 * h_inlet_uy: NULL, or nbeds host pointers (each NULL or [nx] of that bed).
 * d_workspace: caller-owned device memory of lbdps_batch_workspace_bytes,
 * 256-byte aligned.  stream: hipStream_t for every launch of the batch; graph
 * capture needs a stream other than the null stream.  Each bed starts as
 * lbdps_create leaves a context (gas at rest, no particles).  Synchronises.
 */
lbdps_status lbdps_batch_create(const lbdps_params *beds, int32_t nbeds, const int64_t *max_particles,
                                const double *const *h_inlet_uy, void *d_workspace, size_t bytes, void *stream,
                                lbdps_batch **out);

/* The context of bed `bed` (owned by the batch). */
lbdps_status lbdps_batch_bed(lbdps_batch *batch, int32_t bed, lbdps_ctx **out);

/* Enqueue nsteps steps of every bed: 7 launches per step for the whole batch.
 * Results equal nsteps calls of lbdps_step on each bed, bit for bit. */
lbdps_status lbdps_batch_step(lbdps_batch *batch, int32_t nsteps);

/*
 * Capture nsteps batched steps (even, >= 2) into a hipGraph on the batch's
 * stream.  The graph holds the beds' particle counts and buffer parities of
 * this moment: lbdps_batch_launch refuses to replay it once a bed has been
 * changed otherwise (set_state, lbdps_step, lbdps_batch_step with an odd count).
 */
lbdps_status lbdps_batch_capture(lbdps_batch *batch, int32_t nsteps);

/* Replay the captured graph: nsteps more steps of every bed. */
lbdps_status lbdps_batch_launch(lbdps_batch *batch);

/* Wait for the stream; report the first bed's latched device error. */
lbdps_status lbdps_batch_sync(lbdps_batch *batch);

/* As lbdps_time_kernels / lbdps_kernel_times, for the batched launches of
 * lbdps_batch_step (each timed launch covers every bed; graph replays are not
 * timed).  LBDPS_K_RESOLVE sums both resolution launches of a step and counts
 * them as one. */
lbdps_status lbdps_batch_time_kernels(lbdps_batch *batch, uint32_t mask);
lbdps_status lbdps_batch_kernel_times(lbdps_batch *batch, double *h_ms, int64_t *h_launches);

/*
 * Autotuner of a batch: beds are grouped into size classes by particle count
 * (up to 2048, 4096, 8192, ...).  Class by class, every candidate
 * cluster-resolution shape is applied to the class's beds and `steps` batched
 * steps are timed, twice over the candidates in turn; the candidate with the
 * fastest of its two times is kept.  Then the drag tile shapes are timed the
 * same way on the whole batch (one drag launch covers every bed, so the beds
 * share the fastest).  Every bed advances by the steps taken.  cache_path (or
 * NULL): a text file of chosen shapes per class and precision; when every
 * class is found there nothing is timed, and the file is rewritten with all
 * classes.  Synchronises.
 */
lbdps_status lbdps_batch_autotune(lbdps_batch *batch, int32_t steps, const char *cache_path);

/* Release the batch and its beds' contexts (the workspace stays the caller's). */
lbdps_status lbdps_batch_destroy(lbdps_batch *batch);

const char *lbdps_status_str(lbdps_status s);
const char *lbdps_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LBDPS_H */
