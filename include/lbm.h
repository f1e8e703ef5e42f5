/*
 * lbm.h -- C ABI of the MI355X (gfx950) implementation of the Galilean-
 * invariant preconditioned cascaded central-moment D2Q9 lattice Boltzmann
 * method (Hajabdollahi & Premnath, arXiv:1806.10251).
 *
 * One time step is one fused pass over the lattice: pull-streaming with the
 * boundary links (eq. 2b; Sec. 6 boundary rules), macroscopic fields, the
 * same-time-level density gradient, the local strain-rate estimate
 * (eqs. 51-55), the extended-equilibrium GI corrections (eqs. 45-47) and the
 * cascaded collision of Sec. 5 (eq. 2a), written to the second lattice.
 *
 * Conventions shared by every call:
 *   - Every call returns an int status (LBM_OK or a negative LBM_E* code); on
 *     failure lbm_last_error() returns a thread-local message.  Nothing throws
 *     across the ABI.
 *   - Host input arrays are copied during the call; the caller keeps them.
 *     Output buffers are allocated by the caller.
 *   - A context owns all device memory it uses; lbm_destroy frees it
 *     (NULL is a no-op).
 *   - Arrays of nodes are row-major [ny][nx]; node (i, j) sits at
 *     x = i + 1/2, y = j + 1/2; the walls are half-way, at x in {0, nx} and
 *     y in {0, ny}.  Population arrays are [9][ny][nx] in the velocity order
 *     e = (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1).
 *   - "Device" pointers are HIP device addresses on the context's device.
 *   - Work is queued on the context's stream (its own, or the one given to
 *     lbm_set_stream); calls that return host data synchronise that stream.
 */
#ifndef LBM_H
#define LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;     /* one lattice; opaque */
typedef struct lbm_batch lbm_batch; /* many independent lattices; opaque */

enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,    /* invalid argument or configuration                 */
  LBM_ENOMEM = -2,    /* device or host allocation failed                  */
  LBM_EDEVICE = -3,   /* a HIP call failed                                 */
  LBM_EUNSTABLE = -4, /* the fields became non-finite (divergence)         */
  LBM_ESTATE = -5     /* call not valid in the current state               */
};

/* Side kinds (Sec. 6).  side[] is ordered W, E, S, N. */
enum {
  LBM_SIDE_PERIODIC = 0, /* both sides of an axis must be periodic          */
  LBM_SIDE_WALL = 1,     /* stationary half-way bounce-back                 */
  LBM_SIDE_LID = 2,      /* momentum-augmented half-way bounce-back, moving
                            tangentially (+x on S/N, +y on W/E) at u_lid     */
  LBM_SIDE_INLET = 3,    /* W only: moving-wall bounce-back with the
                            parabolic profile 4 U y (H - y) / H^2            */
  LBM_SIDE_OUTLET = 4    /* E only: convective condition on the velocity,
                            density held at rho0 (see the design notes)      */
};

/* Population storage (all compute is FP32, except F64 which computes in FP64).
 * Populations are stored as deviations f - w*rho0; BF16/FP16 store them
 * multiplied by a power-of-two scale and rounded stochastically (seeds from
 * the node and the step index: runs are reproducible, checkpoints resume the
 * sequence), which leaves a rounding-noise floor on the one-step residual
 * (about 4e-4 for FP16 and 3e-3 for BF16 in a channel at gamma 0.2). */
enum { LBM_STORE_F64 = 0, LBM_STORE_F32 = 1, LBM_STORE_BF16 = 2, LBM_STORE_F16 = 3 };

typedef struct {
  int32_t nx, ny;  /* nodes per row / per column, >= 2 each               */
  int32_t side[4]; /* LBM_SIDE_* for W, E, S, N                            */
} lbm_grid;

typedef struct {
  double nu;      /* kinematic viscosity; w4 = w5 = 1/(3 nu/gamma + 1/2),
                     from nu = gamma/3 (1/w - 1/2) (Sec. 2, eq. 49)        */
  double omega3;  /* bulk relaxation rate (eq. 49); 0 -> 1.0               */
  double omega6, omega7, omega8; /* third/fourth-order rates; 0 -> 1.0    */
  double gamma;   /* preconditioning parameter, 0 < gamma <= 1             */
  double u_lid;   /* speed of LID sides                                    */
  double u_in_max;/* peak of the INLET profile; also the OUTLET's U_max    */
  double rho0;    /* reference density; 0 -> 1.0                          */
  double fx, fy;  /* uniform body force (source moments of Sec. 3)         */
  double storage_scale; /* BF16/FP16 scale (power of two); 0 -> default    */
  int32_t storage;      /* LBM_STORE_*                                      */
  int32_t gi_correct;   /* 1: Sec. 5 kernel; 0: eq. 4 kernel (uncorrected) */
  int32_t drho_stencil; /* 0: isotropic FD (default); 1: central FD        */
  int32_t check_every;  /* K >= 1: residual/mass reduction cadence (steps) */
  int32_t strain_fd;    /* 0: strain rates of the GI corrections from the
                           non-equilibrium moments (eqs. 51-55, default);
                           1: from finite differences of the velocity at the
                           same time level (the alternative of Sec. 5), with
                           the drho_stencil stencil; lattices only, a batch
                           rejects it */
  int32_t mrt;          /* 0: cascaded central-moment collision (default);
                           1: non-orthogonal raw-moment MRT form (eq. 7 with
                           the raw equilibria of Sec. 3 and, with gi_correct,
                           the same extended second-order equilibria); rates
                           (w3, w4, w5, w6, w7, w8) as for the cascaded kernel;
                           lattices only, a batch rejects it */
} lbm_params;

/* Create a lattice at rest (f = w*rho0) on the current HIP device: the
 * problem statement of the paper's test cases (Sec. 6: geometry with solid
 * nodes, walls, a moving lid, a parabolic inlet and a convective outlet;
 * viscosity nu and the preconditioning parameter gamma of Sec. 2, eq. 49).
 * solid_mask: ny*nx bytes, nonzero = solid node, NULL = all fluid; copied.
 * Errors: LBM_EINVAL for sizes < 2, a periodic side facing a non-periodic
 * one, INLET off W or OUTLET off E, gamma <= 0, nu <= 0, an unknown storage,
 * check_every < 1, solid nodes in the two columns next to an OUTLET, or a
 * lattice whose nine framed population planes would reach 2^32 bytes at the
 * chosen storage (it is addressed with 32-bit byte offsets: up to about 10800^2
 * nodes in FP32, 7600^2 in FP64, 15300^2 in 16-bit storage);
 * LBM_ENOMEM / LBM_EDEVICE from HIP. */
int lbm_create(const lbm_grid* grid, const uint8_t* solid_mask, const lbm_params* params,
               lbm_ctx** out);

/* Re-initialise every fluid node to the equilibrium (Sec. 3 raw equilibria;
 * central fourth order rho/9) at the given host fields (ny*nx doubles each;
 * NULL -> rho0 / zero velocity).  Resets the step counter. */
int lbm_init_fields(lbm_ctx* ctx, const double* rho, const double* ux, const double* uy);

/* Same, from device arrays of ny*nx floats (e.g. a warm-start prediction
 * already on the GPU).  NULL -> rho0 / zero velocity.  The arrays must be
 * complete with respect to the context's stream (synchronise the stream that
 * wrote them, or share it via lbm_set_stream); the call synchronises the
 * context's stream before it returns, so the caller may free them then. */
int lbm_init_fields_device(lbm_ctx* ctx, const float* rho, const float* ux, const float* uy);

/* Queue all further work on hip_stream (a hipStream_t; NULL = the context's
 * own stream).  The stream must outlive the context or a later call here. */
int lbm_set_stream(lbm_ctx* ctx, void* hip_stream);

/* Advance n >= 0 time steps (asynchronous on the stream).  One step is
 * eq. 2a (collision with the Sec. 5 kernel: strain estimate of eqs. 51-55,
 * corrections of eqs. 45-47; or eq. 4 when gi_correct = 0) followed by eq. 2b
 * (streaming, with the Sec. 6 boundary links).  Every step whose 1-based
 * index is a multiple of check_every also reduces, in FP64, the steady-state
 * residual and the mass.  Errors: LBM_EINVAL for n < 0 or a null context;
 * LBM_EDEVICE when a launch fails. */
int lbm_step(lbm_ctx* ctx, int64_t n);

/* Replace the current state by the mean of the two lattices: after
 * lbm_step(n >= 1) they hold the states of the last two steps (after an
 * initialisation, the initial state twice).  Every undamped period-2
 * component of the state (eigenvalue -1 of the step map, such as the
 * staggered momenta that bounce-back lattices keep) cancels, a
 * steady state is left unchanged, and the fixed point of the iteration is
 * the same.  Meant for warm starts from predicted fields, which excite such
 * components while the state at rest does not.  Asynchronous. */
int lbm_average_last_two(lbm_ctx* ctx);

/* Residual of the last check step, sqrt(sum |u^{n+1}-u^n|^2 / sum |u^n|^2)
 * over fluid nodes, summed in FP64.  The paper shows convergence histories
 * to steady state (Sec. 6, lid-driven cavity and square cylinder) without
 * defining the norm; this relative one-step change is the definition the
 * library adopts (the stopping rule of its steady drivers).  Synchronises.
 * LBM_ESTATE before the first check step; LBM_EUNSTABLE (and *r set) when it
 * is not finite. */
int lbm_residual(lbm_ctx* ctx, double* r);

/* FP64 sum of rho over fluid nodes at the last check step.  Synchronises. */
int lbm_mass(lbm_ctx* ctx, double* m);

/* Number of fluid nodes whose 2x2 strain system was replaced by its gamma-
 * free form (singular-system guard) at the last check step. */
int lbm_guard_count(lbm_ctx* ctx, int64_t* n);

/* Steps taken since the last initialisation. */
int lbm_steps(lbm_ctx* ctx, int64_t* n);

/* Macroscopic fields of the current state into caller-owned host arrays of
 * ny*nx doubles (any may be NULL): rho = sum f and rho u = sum e f - F/(2
 * gamma) of the post-collision populations (the moments of Sec. 2 with the
 * forcing shift of Sec. 3).  Solid nodes report 0.  Synchronises.  Errors:
 * LBM_EINVAL for a null context; LBM_EDEVICE when a HIP call fails. */
int lbm_fields(lbm_ctx* ctx, double* rho, double* ux, double* uy);

/* Same into device arrays of ny*nx floats.  Synchronises. */
int lbm_fields_device(lbm_ctx* ctx, float* rho, float* ux, float* uy);

/* lbm_fields for callers that cannot allocate device memory (code running
 * under graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same values into the same caller-owned host arrays, staged through a
 * fixed 3 MiB device array of the library (one per GPU, 131072 nodes per
 * chunk of whole rows) instead of a per-call allocation; no hipMalloc or
 * hipFree.  The staging array is shared by every call on a GPU and keeps
 * the last call's contents: calls that overlap on one GPU (several threads,
 * or contexts on different streams) race for it and must be serialised by
 * the caller.  Synchronises the context's stream.  Errors: LBM_EINVAL for a
 * null context or rows longer than 131072 nodes; LBM_EDEVICE when a HIP
 * call fails. */
int lbm_fields_noalloc(lbm_ctx* ctx, double* rho, double* ux, double* uy);

/* Current post-collision populations f (not deviations), decoded to FP64,
 * into a caller-owned host array of 9*ny*nx doubles.  Synchronises. */
int lbm_populations(lbm_ctx* ctx, double* f);

/* Checkpoint: raw storage lattice, outlet history and step counter. */
int lbm_save(lbm_ctx* ctx, const char* path);
int lbm_load(lbm_ctx* ctx, const char* path);

/* Convert the current state to another storage type in place (used to
 * finish a run in FP64 once FP32 storage has reached its rounding floor).
 * storage_scale as in lbm_params.  Rebuilds cached graphs. */
int lbm_set_storage(lbm_ctx* ctx, int32_t storage, double storage_scale);

/* Per-node body force (Sec. 2 forcing with a spatially varying F, as the
 * Hartmann and four-rolls mill flows of Sec. 6 need): fx, fy are host arrays
 * of ny*nx doubles, copied (converted to the compute type: FP64 for F64
 * storage, FP32 otherwise) and used at every node in place of the uniform
 * lbm_params.fx, fy, including the F/(2 gamma) momentum shift of the
 * exported fields.  Both NULL: back to the uniform force.  One NULL or a
 * non-finite value: LBM_EINVAL.  Synchronises the stream and rebuilds cached
 * graphs; kept across lbm_set_storage and initialisation, not written to
 * checkpoints.  Reads 2 more compute values per node and step. */
int lbm_set_force_field(lbm_ctx* ctx, const double* fx, const double* fy);

/* Launch shape of the fused step: block of 64 x by threads, each thread
 * holding `rows` lattice rows (the autotuner's knobs).  Supported pairs are
 * listed by lbm_launch_shapes.  Rebuilds cached graphs. */
int lbm_set_launch(lbm_ctx* ctx, int32_t by, int32_t rows);
int lbm_get_launch(lbm_ctx* ctx, int32_t* by, int32_t* rows);
/* Writes up to cap (by, rows) pairs into shapes[2*i], shapes[2*i+1]; returns
 * the number of supported pairs. */
int lbm_launch_shapes(int32_t* shapes, int32_t cap);

/* Average device time of the fused step kernel over the last lbm_step call
 * that was timed (set timing=1 first), in milliseconds. */
int lbm_set_timing(lbm_ctx* ctx, int32_t timing);
int lbm_last_step_ms(lbm_ctx* ctx, double* ms);

void lbm_destroy(lbm_ctx* ctx);

/* Thread-local description of the last failure on this thread. */
const char* lbm_last_error(void);

/* ---------------------------------------------------------------------- */
/* Batch: n independent steady cases advanced together, each time step    */
/* one launch over the tiles of every active case (a case retires when    */
/* its residual falls below tol at a check step, or stops improving).     */
/* Storage is FP32 or FP64 deviations for all cases.                      */
/* ---------------------------------------------------------------------- */

/* grids[c], masks[c] (ny*nx bytes or NULL), params[c] for c < n.  All
 * params must use the same storage (LBM_STORE_F32 or LBM_STORE_F64) and the
 * same check_every.  Inputs copied. */
int lbm_batch_create(int32_t n, const lbm_grid* grids, const uint8_t* const* masks,
                     const lbm_params* params, lbm_batch** out);

/* Equilibrium initialisation of case c from host fields (NULL -> rest). */
int lbm_batch_init_fields(lbm_batch* b, int32_t c, const double* rho, const double* ux,
                          const double* uy);
/* Same from device float arrays (complete with respect to the batch's
 * stream; synchronises that stream before it returns). */
int lbm_batch_init_fields_device(lbm_batch* b, int32_t c, const float* rho, const float* ux,
                                 const float* uy);

int lbm_batch_set_stream(lbm_batch* b, void* hip_stream);

/* Run until every case has residual < tol at a check step, or max_steps
 * steps.  steps_per_case (n entries, may be NULL) receives the step at which
 * each case retired (or max_steps).  Returns LBM_EUNSTABLE if some case
 * diverged (that case retires with its step count negated). */
int lbm_batch_run(lbm_batch* b, double tol, int64_t max_steps, int64_t* steps_per_case);

/* Plateau retirement: a case also retires (status 2) once its residual has
 * not dropped below factor * (its best residual) for `checks` consecutive
 * check steps (checks = 0 disables; default).  This is how an FP32 run
 * detects its rounding floor. */
int lbm_batch_set_plateau(lbm_batch* b, int32_t checks, double factor);

/* Per-case outcome of the last lbm_batch_run (n entries): 0 still running at
 * max_steps, 1 converged (residual < tol), 2 plateau, 3 diverged. */
int lbm_batch_status(lbm_batch* b, int32_t* status);

/* Which cases the next runs advance (n entries, nonzero = advance; NULL =
 * all).  Disabled cases keep their state. */
int lbm_batch_set_enabled(lbm_batch* b, const int32_t* enabled);

/* Convert every case's state to LBM_STORE_F32 or LBM_STORE_F64 in place. */
int lbm_batch_set_storage(lbm_batch* b, int32_t storage);

/* For every enabled case, as lbm_average_last_two. */
int lbm_batch_average_last_two(lbm_batch* b);

/* Residual of case c at its last check step. */
int lbm_batch_residual(lbm_batch* b, int32_t c, double* r);

int lbm_batch_fields(lbm_batch* b, int32_t c, double* rho, double* ux, double* uy);

/* Launch knobs of the batch (the autotuner's).  rows_per_item: block height
 * in wavefronts of one lattice row each, 4, 8 or 16 (0 = 4).  schedule:
 * 0 = one step kernel per time step over all active tiles, case after case,
 * a window of check_every steps captured into a HIP graph and replayed;
 * 1 = the same with tiles interleaved across cases; 2 = one persistent
 * kernel per window in which each tile waits only for its own case's
 * previous step (per-case counters).  LBM_EINVAL for other values. */
int lbm_batch_set_launch(lbm_batch* b, int32_t rows_per_item, int32_t schedule);

void lbm_batch_destroy(lbm_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
