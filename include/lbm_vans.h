/*
 * lbm_vans.h -- C-ABI of the MI355X (gfx950) volume-averaged lattice
 * Boltzmann solver.
 *
 * The method is the D2Q9 lattice Boltzmann model of Zhang, Wang & Ouyang,
 * "Lattice Boltzmann Model for the Volume-Averaged Navier-Stokes Equations"
 * (arXiv:1406.6438): BGK relaxation toward the porosity-weighted equilibrium
 * of eq. (d2q9eq), the pressure-correction term P_i of eq. (pi), the Guo
 * force term F_i of eq. (Fi) carrying a body force plus the Darcy-Forchheimer
 * drag with the Ergun closure (Section "Examples and discussions"), the
 * density and velocity of eqs. (0moment) and (1moment), periodic or
 * half-way bounce-back boundaries.  One time step is the final lattice
 * Boltzmann equation of the Chapman-Enskog section:
 *     f_i(x + e_i, t + 1) = f_i - (f_i - f_i^eq)/tau + P_i + F_i.
 *
 * Lattice units throughout (delta_t = delta_x = 1), D2Q9 with c_s^2 = 1/3 and
 * the velocity ordering
 *     e_0 = (0,0), e_1 = (1,0), e_2 = (0,1), e_3 = (-1,0), e_4 = (0,-1),
 *     e_5 = (1,1), e_6 = (-1,1), e_7 = (-1,-1), e_8 = (1,-1).
 * Every plain field is row-major [Ly][Lx] (x fastest); a population field is
 * [9][Ly][Lx].
 *
 * Memory.  The library allocates no device memory.  The caller passes one
 * device work buffer of lbm_vans_work_bytes() bytes (256-byte aligned) and
 * keeps it alive until lbm_vans_destroy(); the library never frees it.
 * Every other pointer is borrowed for the duration of the call only.  The
 * handle itself is a small host struct owned by the library.
 *
 * Streams.  Every call enqueues its work on the HIP stream given to
 * lbm_vans_init() (NULL = the null stream) and returns without waiting,
 * except where a call says it synchronises.
 *
 * Errors.  Every int-returning call returns LBM_VANS_OK (0) or a negative
 * code and sets a thread-local message readable with lbm_vans_last_error();
 * the calls that report diagnostics may instead return the positive warning
 * LBM_VANS_WMACH (with a message) after completing normally.
 * No C++ exception crosses this interface.
 *
 * Threads.  A handle may be used by one host thread at a time.  Calls on
 * different handles are independent.
 */
#ifndef LBM_VANS_H
#define LBM_VANS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_VANS_ABI_VERSION 9

/* Return codes. */
#define LBM_VANS_OK 0
#define LBM_VANS_EINVAL (-1)     /* invalid argument (message says which)            */
#define LBM_VANS_EHIP (-2)       /* a HIP runtime call failed (message has its text)  */
#define LBM_VANS_ENONFINITE (-3) /* diagnostics found a NaN or Inf in the state       */
#define LBM_VANS_ENOTIMPL (-4)   /* the requested feature is not built                */
/* Warning (positive): the flow left the low-Mach range of the lattice BGK model,
 * max |u| / c_s > LBM_VANS_MACH_WARN (c_s = 1/sqrt(3)); the call itself succeeded. */
#define LBM_VANS_WMACH 1
#define LBM_VANS_MACH_WARN 0.3

/* Boundary kind of one axis (applies to both ends of that axis). */
#define LBM_BC_PERIODIC 0   /* wrap-around streaming (Section "Examples and discussions") */
#define LBM_BC_BOUNCEBACK 1 /* half-way bounce-back wall beyond node -1/2 and L-1/2; the
                               y-walls may slide along x (lbm_vans_params.u_wall)         */
#define LBM_BC_OPEN 2       /* x only: inflow reservoir beyond x = 0, outflow reservoir
                               beyond x = Lx-1.  From state n = 1 on, a population that
                               enters across an open end is the equilibrium (eq. (d2q9eq))
                               of a reservoir with the boundary node's porosity, density
                               rho_in / rho_out and velocity (u_in, 0) / (u_out, 0); one
                               that leaves is absorbed.  Behind a y-wall bounce-back wins. */
#define LBM_BC_INOUT 3      /* x only: velocity inlet beyond x = 0, pressure outlet beyond
                               x = Lx-1 (the through-flow channel; the paper gives no rule
                               for one, so both are equilibria of eq. (d2q9eq), each with
                               the boundary node's porosity and one free quantity taken
                               from the node itself, zero-gradient):
                                 entering at x = 0 at step n+1: f_i^eq(eps rho of node
                                   (0, y) at step n, (u_in, 0));
                                 entering at x = Lx-1 at step n+1: f_i^eq(eps rho_out,
                                   velocity of node (Lx-1, y) at step n);
                               a population that leaves is absorbed; behind a y-wall
                               bounce-back wins.  Applies from the first step on; the
                               state f(., n) alone determines the next (get_state /
                               set_state hold everything).  rho_in and u_out unused.   */

/* Population storage.  The collision arithmetic is FP64 for LBM_F64 and FP32
 * otherwise.  The shifted forms store the deviation of each population from
 * the local rest state w_i eps rho0, which keeps the significant digits of
 * the flow in the stored bits. */
#define LBM_F64 0
#define LBM_F32_SHIFTED 1
#define LBM_F16_SHIFTED 2

/* Drag law of the force F (Section "Examples and discussions"):
 *     F = G - (eps^2 nu / K) u - (eps^3 F_eps / sqrt(K)) |u| u.
 * LBM_DRAG_ERGUN: K = eps^3 d_p^2 / (150 (1-eps)^2), F_eps = 1.75/sqrt(150 eps^3)
 *                 (Ergun closure); d_p = INFINITY gives no drag.
 * LBM_DRAG_CONST: K and F_eps given directly (uniform); K = INFINITY gives no drag. */
#define LBM_DRAG_ERGUN 0
#define LBM_DRAG_CONST 1

/* Number of doubles in one diagnostics record (see lbm_vans_moments). */
#define LBM_VANS_NDIAG 8
/* Records kept by the in-sweep diagnostics ring (see lbm_vans_diag_read). */
#define LBM_VANS_DIAG_RING 4096

typedef struct lbm_vans_params {
    int32_t Lx, Ly;        /* lattice nodes, 1 <= Lx, Ly (Lx >= 2 with open x ends);
                              padded nodes (Lx rounded up to 256) x Ly < 2^31          */
    int32_t bc_x, bc_y;    /* LBM_BC_PERIODIC or LBM_BC_BOUNCEBACK; bc_x may be LBM_BC_OPEN
                              or LBM_BC_INOUT                                          */
    int32_t storage;       /* LBM_F64, LBM_F32_SHIFTED or LBM_F16_SHIFTED             */
    int32_t drag;          /* LBM_DRAG_ERGUN or LBM_DRAG_CONST                        */
    double tau;            /* BGK relaxation time, > 1/2; nu = (tau - 1/2)/3         */
    double d_p;            /* Ergun particle diameter (> 0, may be INFINITY)          */
    double K, F_eps;       /* LBM_DRAG_CONST: permeability (> 0, may be INFINITY), F_eps >= 0 */
    double G[2];           /* external body-force density in the (eps rho u) equation */
    double rho0;           /* initial density (> 0); also the storage shift reference */
    double u0[2];          /* initial velocity                                        */
    int32_t fp16_scale_log2; /* LBM_F16_SHIFTED: stored value = deviation * 2^s, 0..24 */
    int32_t diag_every;    /* > 0: record diagnostics of every state n with n % diag_every == 0
                              during lbm_vans_step; 0: none                           */
    double rho_in, u_in;   /* LBM_BC_OPEN: inflow reservoir density (> 0), x-velocity;
                              LBM_BC_INOUT: u_in is the inlet velocity               */
    double rho_out, u_out; /* LBM_BC_OPEN: outflow reservoir density (> 0), x-velocity;
                              LBM_BC_INOUT: rho_out (> 0) is the outlet density      */
    double u_wall[2];      /* LBM_BC_BOUNCEBACK in y: x-velocity of the wall below y = 0
                              and of the wall above y = Ly-1 (sliding plates, as the
                              Couette experiment of Section "Examples and discussions");
                              0 otherwise.  A population returned by a sliding wall gains
                              6 w_i eps(x) rho0 (e_i . u_w), the momentum the moving wall
                              imparts under half-way bounce-back.                     */
    int32_t sweep_vec;     /* nodes per lane of the one-step sweep: 0 = automatic (the
                              widest: 4, or 2 in LBM_F64, unless its tiles (64 lanes
                              of that many nodes, by 4 rows; FP16: 8 rows) would be
                              fewer than the GPU's compute units, then 1); 1; or the
                              widest.  Results do not depend on it beyond rounding.   */
    int32_t steps_per_pass;/* most time steps one pass over the lattice takes: 1, 2, 3
                              or 4 (4: LBM_F32_SHIFTED storage, 24-row chunks of
                              58-column strips); 0 = automatic: 4 with FP32 storage and
                              pass_rows = 0 when the four-step pass has at least as many
                              waves as the GPU holds of its kernel at once (three times
                              as many with open x ends), else 3
                              when the three-step pass has enough
                              waves (60 columns x pass_rows rows each) for the GPU:
                              0.9 times as many as it holds of the kernel at once in
                              24-row chunks, half in 12-row chunks, a fifth in 6-row
                              chunks (FP32; with open x ends 4 times, 1.5 times and a
                              fifth), 0.7
                              times (FP16, or an explicit pass_rows); else 2 when the
                              two-step pass has >= 2048 waves (62 x 8, 16 in FP16),
                              else 1.  Several steps per pass need
                              LBM_F32_SHIFTED or LBM_F16_SHIFTED storage and
                              diag_every = 0 (else one step per pass), and with
                              periodic y a lattice of at least pass_rows + 6 rows for
                              three steps (32 for four, chunk rows + 4 for two; else
                              fewer steps);
                              the intermediate states stay in registers (so FP16
                              storage rounds once per pass) and each pass recomputes
                              its chunk's halo.                                       */
    int32_t pass_rows;     /* output rows per chunk (wave) of the three-step pass:
                              0 = automatic; LBM_F32_SHIFTED: 6, 12, 24 or 28
                              (automatic: 28 when that still gives four times as many
                              waves as the GPU holds of the kernel at once, else 24
                              when that gives 0.9 times as many, else 12 when that
                              gives half as many, else 6; with open x ends 24 from 4
                              times, 12 from 1.5 times: taller chunks recompute
                              fewer halo rows but give fewer waves);
                              LBM_F16_SHIFTED: 24.  Batches take 24 or 28.  Results
                              do not depend on it beyond rounding.                    */
} lbm_vans_params;

typedef struct lbm_vans_handle lbm_vans_handle;

/* Bytes of device work memory the solver needs for these parameters, or 0 if
 * the parameters are invalid (lbm_vans_last_error() says why). */
size_t lbm_vans_work_bytes(const lbm_vans_params *p);

/* Create a solver and set the state to the initial condition of Section
 * "Examples and discussions" (density rho0 and velocity u0 everywhere):
 *     f_i(x, 0) = f_i^eq(eps(x) rho0, u0)            (eq. (d2q9eq)).
 * eps:   device pointer to the porosity field [Ly][Lx], double for LBM_F64,
 *        float otherwise; every value in (0, 1].  It is copied into the work
 *        buffer, so the caller may free it after this call returns.
 * work:  device buffer of at least lbm_vans_work_bytes(p) bytes, 256-byte
 *        aligned, owned by the caller, not touched by anyone else while the
 *        handle lives.
 * stream: hipStream_t to run on (NULL = null stream).
 * On success *out receives the handle.  The porosity check synchronises the
 * stream once.  Returns LBM_VANS_EINVAL for invalid parameters, a short or
 * misaligned work buffer, or a porosity outside (0, 1]. */
int lbm_vans_init(const lbm_vans_params *p, const void *eps, void *work, size_t work_bytes,
                  void *stream, lbm_vans_handle **out);

/* Advance nsteps (>= 0) time steps of the final lattice Boltzmann equation:
 * for every node, the moments of eqs. (0moment)/(1moment) (velocity implicit
 * through the drag, solved exactly), collision toward eq. (d2q9eq) with the
 * sources of eqs. (pi) and (Fi), and streaming with the boundary rule, fused
 * in one pass per step, or per two, three or four steps where
 * params.steps_per_pass allows it (the intermediate states then never leave the
 * GPU's registers).
 * Asynchronous. */
int lbm_vans_step(lbm_vans_handle *h, int64_t nsteps);

/* Number of steps taken since init (the current state is f(., n)). */
int64_t lbm_vans_step_count(const lbm_vans_handle *h);

/* Launch plan of lbm_vans_step: the most steps one pass takes (params.
 * steps_per_pass, or the automatic choice made at init from the lattice and the
 * GPU) and the rows per chunk of the three-step pass (params.pass_rows, or the
 * automatic choice; 0 when the handle has no multi-step pass: LBM_F64 storage or
 * a lattice too large for it).  Either pointer may be NULL.  Host only. */
int lbm_vans_pass_plan(const lbm_vans_handle *h, int32_t *steps_per_pass, int32_t *pass_rows);

/* Macroscopic fields of the current state f(., n) (eqs. (0moment), (1moment)):
 * eps_rho, rho, ux, uy are device arrays [Ly][Lx] of the compute type (double
 * for LBM_F64, float otherwise); any may be NULL.
 * diag: host array of LBM_VANS_NDIAG doubles or NULL.  When given, the call
 * reduces in FP64 on the device and synchronises the stream, then fills
 *   diag[0] = sum_x eps rho            diag[1], diag[2] = sum_x m (m = sum_i e_i f_i)
 *   diag[3], diag[4] = sum_x eps rho u diag[5] = max_x |u|
 *   diag[6] = number of nodes whose moments are not finite
 *   diag[7] = n (step index).
 * Returns LBM_VANS_ENONFINITE (after filling diag) if diag[6] > 0, else
 * LBM_VANS_WMACH if diag[5] / c_s exceeds LBM_VANS_MACH_WARN. */
int lbm_vans_moments(lbm_vans_handle *h, void *eps_rho, void *rho, void *ux, void *uy,
                     double *diag);

/* Copy the current state f(., n) out as plain populations: f is a device
 * array of 9*Ly*Lx doubles in the layout [9][Ly][Lx]. */
int lbm_vans_get_state(lbm_vans_handle *h, void *f);

/* Replace the current state with the plain populations f (device, 9*Ly*Lx
 * doubles, [9][Ly][Lx]); the step counter is kept.  Storage rounding applies. */
int lbm_vans_set_state(lbm_vans_handle *h, const void *f);

/* Copy the in-sweep diagnostics records (params.diag_every > 0) to the host,
 * oldest first: at most max_records records of LBM_VANS_NDIAG doubles with the
 * meaning of lbm_vans_moments' diag, for the states n = 0, k, 2k, ... swept so
 * far (the last LBM_VANS_DIAG_RING of them).  *n_records receives the count.
 * Synchronises the stream.  Returns LBM_VANS_ENONFINITE if any copied record
 * counts non-finite nodes, else LBM_VANS_WMACH if any record's max |u| / c_s
 * exceeds LBM_VANS_MACH_WARN. */
int lbm_vans_diag_read(lbm_vans_handle *h, double *records, int32_t max_records,
                       int32_t *n_records);

/* Objective of lbm_vans_grad: the outlet mass flux, J = sum over the last
 * column x = Lx-1 of eps rho u_x of the state f(., nsteps) (eqs. (0moment),
 * (1moment)): the superficial mass flux through that section per unit depth. */
#define LBM_OBJ_OUTLET_FLUX 0

/* Value of the objective (LBM_OBJ_OUTLET_FLUX) for the current state f(., n),
 * computed on the device in FP64 (the value lbm_vans_grad returns as J after
 * the same steps), without a reverse sweep.  J: host double.  Synchronises the
 * stream.  Returns LBM_VANS_ENONFINITE if J is not finite. */
int lbm_vans_objective(lbm_vans_handle *h, int32_t objective, double *J);

/* Bytes of device memory lbm_vans_grad needs as grad_work for these
 * arguments (0 if invalid): one population buffer per checkpoint
 * (ceil(nsteps / ckpt_every)), ckpt_every buffers for a recomputed segment --
 * two sets of them when there are two or more segments, so that one segment is
 * recomputed while the reverse steps of the next run --, two adjoint buffers
 * of 9 values per node (FP64 with LBM_F64 storage, FP32 otherwise) and three
 * FP64 accumulators of the porosity grid (with LBM_F32 / LBM_F16_SHIFTED
 * storage also an FP64 copy of the porosity). */
size_t lbm_vans_grad_work_bytes(const lbm_vans_params *p, int32_t objective, int64_t nsteps,
                                int32_t ckpt_every);

/* Value and porosity gradient of the objective after nsteps steps from the
 * initial state (the state is reset to f(., 0), then advanced): J and
 * dJdeps(x) = dJ/deps(x), the exact derivative of the discrete map (up to
 * rounding), computed by the reverse (adjoint) sweep: a forward pass keeping
 * a checkpoint every ckpt_every steps (up to three steps per pass in between, as
 * in lbm_vans_step, when params.steps_per_pass allows it), then, segment by segment
 * from the last, the states recomputed one step at a time from the
 * checkpoint (on a second stream of the handle, one segment ahead) and the
 * adjoint stepped back through them.  Porosity enters
 * through eps itself (density, drag), through grad(eps), through the
 * open-boundary reservoirs (and the boundary density / velocity a velocity
 * inlet / pressure outlet carries) and the initial state.  The reverse steps
 * compute in FP64 for every storage: with LBM_F32 / LBM_F16_SHIFTED storage
 * they decode the recomputed FP32 / FP16 states into FP64, hand the adjoints
 * from one step to the next in FP32 (one rounding per value and step) and add
 * every step's sensitivities to FP64 accumulators; the gradient's error is then
 * that of the stored forward states (the FP32 adjoints add about 1e-7 of the
 * gradient's largest value).
 * grad_work: device buffer of lbm_vans_grad_work_bytes() bytes, 256-byte
 * aligned, caller-owned.  dJdeps: device array [Ly][Lx] of doubles.
 * J: host double or NULL.  Synchronises the stream.  Afterwards the state is
 * f(., nsteps) and the step count is nsteps.  Returns LBM_VANS_ENONFINITE if
 * J is not finite. */
int lbm_vans_grad(lbm_vans_handle *h, int32_t objective, int64_t nsteps, int32_t ckpt_every,
                  void *grad_work, size_t grad_work_bytes, double *dJdeps, double *J);

/* Bytes of the library-held gradient workspace of lbm_vans_grad_static (64 MiB). */
#define LBM_VANS_GRAD_STATIC_BYTES ((size_t)64 << 20)

/* lbm_vans_grad without a caller buffer, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same computation and results, with the workspace in a
 * fixed array of LBM_VANS_GRAD_STATIC_BYTES that the library holds on every GPU
 * it runs on until the process ends.  The call allocates nothing.  Returns
 * LBM_VANS_EINVAL (message gives the bytes needed) when
 * lbm_vans_grad_work_bytes(p, objective, nsteps, ckpt_every) exceeds that size.
 * Every call on one GPU shares that GPU's array and leaves it holding its last
 * contents (each call initialises what it reads); calls that overlap in time on
 * the same GPU (two host threads, or two streams) race and must be serialised by
 * the caller.  Synchronises the stream, as lbm_vans_grad. */
int lbm_vans_grad_static(lbm_vans_handle *h, int32_t objective, int64_t nsteps,
                         int32_t ckpt_every, double *dJdeps, double *J);

/* Release the handle (host memory only; the work buffer stays the caller's).
 * Waits for the handle's queued work first.  NULL is ignored. */
void lbm_vans_destroy(lbm_vans_handle *h);

/* ---- Ensembles --------------------------------------------------------
 * A batch advances many independent problems (members) with one kernel
 * launch per time step: the tiles of all members form one work list, and
 * every member takes exactly the step lbm_vans_step would take (same node
 * update, per member tau, drag, forcing, reservoirs and size).  Members are
 * existing handles; they must share storage, bc_x and bc_y, have
 * diag_every = 0 and be at the same step.  A member stays a normal handle:
 * lbm_vans_moments / get_state / set_state / step work on it between batch
 * calls (a member stepped on its own puts the batch out of step, and batch
 * calls then fail with LBM_VANS_EINVAL until the others catch up).  The batch
 * borrows the members: destroy it before them.  Batched work runs on the
 * batch's stream; ordering it against a member's own stream is the caller's
 * (one stream for all is simplest). */
typedef struct lbm_vans_batch lbm_vans_batch;

/* Launch shape of the batched sweep. */
typedef struct lbm_vans_batch_config {
    int32_t vec;          /* nodes per lane, a power of two up to 4 (2 for LBM_F64): tiles
                             are 64*vec nodes wide; a member whose Lx is not a multiple
                             uses the largest power of two below that divides its Lx   */
    int32_t grid;         /* 0: one workgroup per tile; else a persistent grid of that
                             many workgroups (a multiple of 8) walking the tile list   */
    int32_t graph_steps;  /* steps per replay of the captured step graph (even); 0: plain
                             launches.  lbm_vans_batch_step replays the graph for whole
                             chunks from state n >= 1 and launches the rest one by one */
    int32_t steps_per_pass;/* most steps one launch takes, as lbm_vans_params.
                             steps_per_pass (1, 2, 3, or 4 with LBM_F32_SHIFTED
                             storage and members that take the four-step pass; 0 =
                             automatic: 4 with FP32 storage, pass_rows = 0 and at
                             least as many waves of the batched four-step pass as
                             the GPU holds of it, else 3): with LBM_F32 /
                             LBM_F16_SHIFTED storage the multi-step pass over every
                             member; vec and grid apply to single steps           */
    int32_t pass_rows;    /* rows per chunk of the batched three-step pass, 24 or 28
                             with FP32 storage (0 = automatic: 28 when the whole
                             batch has four times as many waves of 28 rows as the
                             GPU holds of the batched kernel, else 24; the batched
                             four-step pass takes 24); the members' own pass_rows
                             are not used                                          */
    double us_per_step;   /* lbm_vans_batch_tune: measured microseconds per step       */
} lbm_vans_batch_config;

/* Bytes of the device table a batch of these members needs (0 if invalid). */
size_t lbm_vans_batch_work_bytes(lbm_vans_handle *const *members, int32_t nmembers);

/* Create a batch of nmembers handles (the array is copied).  work: device
 * buffer of lbm_vans_batch_work_bytes() bytes, 256-byte aligned, caller-owned,
 * kept alive until lbm_vans_batch_destroy().  stream: hipStream_t of the
 * batched work (NULL = null stream); graphs are captured on a private stream
 * and replayed on it.  Default configuration: widest vec, one workgroup per
 * tile, 24-step graphs, automatic steps per launch.
 * Synchronises the stream (table upload). */
int lbm_vans_batch_create(lbm_vans_handle *const *members, int32_t nmembers, void *work,
                          size_t work_bytes, void *stream, lbm_vans_batch **out);

/* Set the launch shape (validated as documented in lbm_vans_batch_config).
 * Results do not depend on it.  Synchronises the stream. */
int lbm_vans_batch_configure(lbm_vans_batch *b, const lbm_vans_batch_config *cfg);
int lbm_vans_batch_get_config(const lbm_vans_batch *b, lbm_vans_batch_config *cfg);

/* Autotune the launch shape on the current members: every vec (widest
 * first) with one workgroup per tile and with persistent grids of 1, 2, 4 and
 * 8 workgroups per compute unit, each timed with HIP events over reps sweeps
 * of the current state (read only: the state does not change), and, with
 * LBM_F32 / LBM_F16_SHIFTED storage, the two- and three-step passes and, with
 * FP32 storage, the four-step pass (their time per launch divided by 2, 3 and
 * 4; steps_per_pass 2, 3 and 4 in those trials, 1 in the others).  The fastest becomes the configuration (graph_steps kept; the
 * best single-step vec and grid kept when a multi-step pass wins) and is
 * written to *best (may be NULL); trials
 * (may be NULL if max_trials is 0) receive up to max_trials of the timed
 * shapes and *n_trials (may be NULL) their number.  Synchronises. */
int lbm_vans_batch_tune(lbm_vans_batch *b, int32_t reps, lbm_vans_batch_config *best,
                        lbm_vans_batch_config *trials, int32_t max_trials, int32_t *n_trials);

/* Advance every member nsteps (>= 0) time steps (as lbm_vans_step; with
 * LBM_F32 / LBM_F16_SHIFTED storage up to steps_per_pass steps per launch, the
 * steps left over in a shorter launch).  Asynchronous. */
int lbm_vans_batch_step(lbm_vans_batch *b, int64_t nsteps);

/* Launch plan of lbm_vans_batch_step under the current configuration: the most
 * steps one launch takes and the rows per chunk of its multi-step pass (0
 * without one), as lbm_vans_pass_plan.  Host only. */
int lbm_vans_batch_pass_plan(const lbm_vans_batch *b, int32_t *steps_per_pass,
                             int32_t *pass_rows);

/* Bytes of grad_work for lbm_vans_batch_grad: the members' lbm_vans_grad
 * workspaces, each rounded up to 256 bytes, back to back (0 if invalid). */
size_t lbm_vans_batch_grad_work_bytes(const lbm_vans_batch *b, int32_t objective,
                                      int64_t nsteps, int32_t ckpt_every);

/* lbm_vans_grad for every member at once, each forward and reverse step one
 * batched launch: dJdeps is a host array of nmembers device pointers (each
 * [Ly][Lx] doubles of its member), J a host array of nmembers doubles or NULL.
 * Afterwards every member is at state f(., nsteps).  Synchronises.  Returns
 * LBM_VANS_ENONFINITE if a member's J is not finite. */
int lbm_vans_batch_grad(lbm_vans_batch *b, int32_t objective, int64_t nsteps,
                        int32_t ckpt_every, void *grad_work, size_t grad_work_bytes,
                        double *const *dJdeps, double *J);

/* Release the batch (waits for its stream; the members are untouched).
 * NULL is ignored. */
void lbm_vans_batch_destroy(lbm_vans_batch *b);

/* Message of the last failed call on this thread ("" if none). */
const char *lbm_vans_last_error(void);

/* LBM_VANS_ABI_VERSION of the built library. */
int lbm_vans_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_VANS_H */
