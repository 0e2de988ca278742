/*
 * ddcc.h - C ABI of the MI355X DD-CCLB library (libddcc.so).
 *
 * The library advances the diffuse-domain consistent and conservative
 * lattice Boltzmann scheme of Liu, Zhan, Chen, Chai and Shi (arXiv
 * 2311.10314), Section 3: N phase-field distribution sets f^i (eq. 3.1) and
 * one flow set g (eq. 3.2), Hermite-moment collision Lambda = H^-1 S H
 * (eqs. 3.3-3.4), diffuse-domain and wetting sources from the smooth
 * characteristic function psi (eq. 2.14, eqs. 3.5-3.13), pull streaming, and
 * recovery of C_i, u and P (moment recovery of Section 3, eq. 19).
 *
 * Units are lattice units: dx = dt = c = 1, c_s^2 = d0 (Section 3).
 * Grids are periodic boxes; walls are embedded through psi (Section 2.3).
 *
 * Array layout of every field crossing this ABI: C order, x fastest:
 *   scalar field  [nz][ny][nx]            (nz = 1 in 2D)
 *   per-phase     [nphase][nz][ny][nx]
 *   vector        [dim][nz][ny][nx]       (component 0 = x, 1 = y, 2 = z)
 * Host arrays are float64. The *_dev variants take device pointers to
 * float64 arrays of the same layout (e.g. torch tensors on the GPU) and work
 * on the context's stream without a host copy.
 *
 * Ownership: the caller owns every array it passes. The library copies
 * inputs in during the call (host variants) or enqueues the copy on its stream
 * (device variants: keep the memory alive until ddcc_sync returns). The
 * context owns all of its device memory and releases it in ddcc_destroy.
 *
 * Errors: every call returns DDCC_OK (0) or one of the DDCC_E_* codes; no C++
 * exception crosses the ABI. ddcc_last_error() gives a message for the last
 * failed call on that context. A context stays valid for ddcc_destroy after
 * any error.
 */
#ifndef DDCC_H
#define DDCC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DDCC_OK 0
#define DDCC_E_INVAL 1       /* bad shape, parameter or non-finite input      */
#define DDCC_E_STATE 2       /* call out of order (step before both inits)     */
#define DDCC_E_NOMEM 3       /* device allocation failed                       */
#define DDCC_E_HIP 4         /* HIP runtime error; text in ddcc_last_error     */
#define DDCC_E_NONFINITE 5   /* a diagnostic found NaN/Inf in the populations */
#define DDCC_E_UNSUPPORTED 6 /* valid input the library has no kernel for    */

/* Velocity sets (Section 3 tables; D3Q19 weights from the same moment
 * constraints). */
#define DDCC_D2Q9 0
#define DDCC_D3Q7 1
#define DDCC_D3Q15 2
#define DDCC_D3Q19 3

/* Storage / arithmetic precision of the populations and history. In every
 * precision the rest populations of the phase sets are float64 and take back
 * the storage rounding of the node's moving populations, so the mass of each
 * phase is conserved to the rounding of the arithmetic; the flow set's rest
 * population is stored as the deviation g_0 - rho0. */
#define DDCC_FP64 0  /* float64 storage, float64 arithmetic              */
#define DDCC_FP32 1  /* float32 storage, float32 arithmetic              */
#define DDCC_FP16 2  /* moving populations in IEEE half, history, T and
                        geometry in float32, float32 arithmetic          */
#define DDCC_BF16 3  /* moving populations in bfloat16, otherwise as
                        DDCC_FP16                                        */

#define DDCC_MAX_PHASES 4
#define DDCC_MAX_WALLS 8

/* Rate slots of s_f[] and s_g[]: the diagonal of S (Section 3 lattice
 * tables): s0, s1, s21, s22, s3, s4. For the flow set s_g[2] and s_g[3] are
 * ignored: s21 and s22 follow the local viscosity through eq. (16). */
#define DDCC_S0 0
#define DDCC_S1 1
#define DDCC_S21 2
#define DDCC_S22 3
#define DDCC_S3 4
#define DDCC_S4 5

typedef struct ddcc_params {
  int dim;          /* 2 or 3                                               */
  int nx, ny, nz;   /* grid size; nz = 1 when dim = 2; all >= 1             */
  int nphase;       /* N, 2 <= N <= DDCC_MAX_PHASES                          */
  int lattice_f;    /* velocity set of the phase sets: DDCC_D2Q9 in 2D,
                       DDCC_D3Q15 or DDCC_D3Q7 (needs d0 < 1/3) in 3D     */
  int lattice_g;    /* velocity set of the flow set   (DDCC_D2Q9 / D3Q19)    */
  int precision;    /* DDCC_FP64, DDCC_FP32, DDCC_FP16 or DDCC_BF16          */
  double d0;        /* c_s^2 / c^2, inside the lattices' positive-weight range */
  double eps;       /* fluid-fluid interface width (cells), Section 2.1       */
  double m0;        /* mobility of eq. (2.5)                                  */
  double rho0;      /* constant of g^eq_0, eq. (3.8)                          */
  double psi_min;   /* floor of psi in the divisions phi X / phi (> 0)        */
  double lam;       /* penalty coefficient of (1 - psi) u, eq. (2.13c) (>= 0) */
  double sigma[DDCC_MAX_PHASES][DDCC_MAX_PHASES]; /* symmetric, zero diagonal,
                                                     > 0 off the diagonal     */
  double rho[DDCC_MAX_PHASES];  /* phase densities (> 0)                      */
  double nu[DDCC_MAX_PHASES];   /* phase kinematic viscosities (> 0)          */
  double eta[DDCC_MAX_PHASES];  /* eta_i of eq. (3.5); <= 0 means derive it
                                   from m0 and s_f[1] by eq. (17)            */
  double s_f[6];    /* rates of the phase sets, each in (0, 2)               */
  double s_g[6];    /* rates of the flow set (slots 2, 3 unused)             */
  double accel[3];  /* body acceleration a; adds psi rho a to the force      */
  double force[3];  /* body force density G; adds psi G to the force        */
} ddcc_params;

typedef struct ddcc_ctx ddcc_ctx;

/* Fills *p with defaults: the lattice and rate choices of Section 4
 * (s_f = {1, 10/19, 1.2, 1.2, 1.2, 1.2}, s_g = {1, 1.2, -, -, 1.2, 1.2}),
 * d0 = 0.4, eps = 5, m0 = 0.05, rho0 = 1, psi_min = 1e-30, sigma_ij = 0.001
 * (i != j), rho_i = 1 and nu_i = 0.1 for every phase, eta derived by eq.
 * (17), no body force, for a 2D D2Q9 N = 2 FP64 box of 64 x 64. Always
 * returns DDCC_OK for p != NULL. */
int ddcc_default_params(ddcc_params* p);

/* Validates *p and allocates the device state on the current HIP device.
 * `stream` is a hipStream_t to run on (e.g. a torch stream), or NULL for a
 * stream the context creates and owns. On success *out holds a new context;
 * on failure *out is NULL and the return code says why. */
int ddcc_create(const ddcc_params* p, void* stream, ddcc_ctx** out);

/* Static geometry (eq. 2.14 and Section 2.3): psi [nz][ny][nx] in [0, 1]
 * and cos_theta [N-1][nz][ny][nx]: cos of the contact angle theta_iN of
 * phase i against phase N, measured inside phase i (eqs. 2.7-2.9), each in
 * [-1, 1]; NULL means 90 degrees everywhere. Must precede ddcc_init_fields. */
int ddcc_init_geometry(ddcc_ctx* ctx, const double* psi,
                       const double* cos_theta);

/* Static geometry of several walls (Section 4.5): psi [nwalls][nz][ny][nx],
 * the smooth characteristic function psi_k of each wall, and cos_theta
 * [nwalls][N-1][nz][ny][nx], each wall's own contact angles theta^k_iN (NULL:
 * 90 degrees). The box's characteristic function is psi = prod_k psi_k and
 * the wetting term of eq. (2.14) sums cos theta^k_jq |grad psi_k| over the
 * walls; each psi_k must be smooth on the periodic box by itself (fluid on
 * both sides of a band). ddcc_init_geometry is the case nwalls = 1.
 * 1 <= nwalls <= DDCC_MAX_WALLS. Synchronises. */
int ddcc_init_geometry_walls(ddcc_ctx* ctx, int nwalls, const double* psi,
                             const double* cos_theta);
int ddcc_init_geometry_dev(ddcc_ctx* ctx, const double* psi_dev,
                           const double* cos_theta_dev);

/* Initial state: C [N][nz][ny][nx] (volume fractions), u [dim][..] or NULL
 * for rest, P [..] or NULL for zero. Populations start at their equilibria
 * (eqs. 3.5, 3.8) and every time derivative starts at zero. Resets time. */
int ddcc_init_fields(ddcc_ctx* ctx, const double* C, const double* u,
                     const double* P);
int ddcc_init_fields_dev(ddcc_ctx* ctx, const double* C_dev,
                         const double* u_dev, const double* P_dev);

/* Advances nsteps >= 0 time steps (eqs. 3.1, 3.2), asynchronously on the
 * context stream: in 2D one fused kernel per step; in 3D three, one forming
 * C_i from the pulled phase populations, one z-marching kernel for the
 * chemical potential mu_i, and one z-marching kernel for the node update.
 * Contexts whose step moves more than the 256 MB memory-side cache run the
 * same kernels with nontemporal stores, and in 2D with the loads of a tile
 * issued earlier (same results bit for bit). */
int ddcc_step(ddcc_ctx* ctx, int64_t nsteps);

/* C_i, u and P of the current time level (moment recovery of Section 3 and
 * eq. 19); any pointer may be NULL to skip that field. Host variant
 * synchronises the stream; device variant only enqueues. */
int ddcc_read_moments(ddcc_ctx* ctx, double* C, double* u, double* P);
int ddcc_read_moments_dev(ddcc_ctx* ctx, double* C_dev, double* u_dev,
                          double* P_dev);

/* Per-phase mass sum_x sum_p f^i_p in float64 (conserved exactly by the
 * scheme: sum_p F^i_p = 0 and sum_p f^i,eq_p = phi C_i). Synchronises.
 * Returns DDCC_E_NONFINITE if any population is NaN or Inf. */
int ddcc_mass(ddcc_ctx* ctx, double* mass /* [nphase] */);

/* ddcc_mass for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * calls no hipMalloc, hipFree or other allocating routine. The per-block
 * partial sums live in a static device workspace of the library, one copy
 * per GPU of 36 KiB (1024 blocks x 4 phases float64 plus 1024 flags), held
 * until the process ends; every call on one GPU shares it, so calls that
 * overlap on one GPU (contexts on different streams) race and must be
 * ordered by the caller. Contexts never need more than that workspace;
 * DDCC_E_INVAL with a message if one did.
 * mass_dev      device float64 [nphase] out: the masses of ddcc_mass, bit for
 *               bit (same partials, summed in the same block order)
 * nonfinite_dev device int out (may be NULL): 1 if a population was NaN or
 *               Inf, else 0
 * Enqueues on the context stream and returns without synchronising; the
 * outputs are valid once the stream has run (ddcc_sync). Errors:
 * DDCC_E_INVAL (NULL ctx or mass_dev), DDCC_E_STATE (before init_fields),
 * DDCC_E_HIP. */
int ddcc_mass_noalloc(ddcc_ctx* ctx, double* mass_dev, int* nonfinite_dev);

/* Number of completed steps since ddcc_init_fields. */
int64_t ddcc_time(const ddcc_ctx* ctx);

/* Exact checkpoint of populations and history. With buf == NULL, *bytes
 * receives the size needed; otherwise *bytes must be at least that size and
 * the state is copied to host memory `buf`. Synchronises. */
int ddcc_save(ddcc_ctx* ctx, void* buf, size_t* bytes);
/* Restores a checkpoint written by ddcc_save for identical ddcc_params. */
int ddcc_load(ddcc_ctx* ctx, const void* buf, size_t bytes);

/* Waits for all work queued on the context stream. With periodic
 * diagnostics on (ddcc_set_diagnostics), returns DDCC_E_NONFINITE once a
 * check has seen a NaN or Inf population (the step is in the message). */
int ddcc_sync(ddcc_ctx* ctx);

/* Periodic conservation diagnostics inside the step stream: every `every`
 * time levels (t % every == 0, counted by ddcc_step) the per-phase masses
 * sum_x sum_p f^i_p of ddcc_mass are summed on the device, in float64, and
 * a sticky flag records the first level at which a population was not
 * finite, without a host synchronisation. The paper's scheme conserves
 * each phase's mass exactly (sum_p F^i_p = 0, sum_p f^i,eq_p = phi C_i;
 * Section 3), so the masses are a check of the run. every = 0 turns the
 * checks off (the default); every < 0 returns DDCC_E_INVAL. Setting it,
 * ddcc_init_fields and ddcc_load clear the record. Allocates two small
 * device buffers on first use. Synchronises. */
int ddcc_set_diagnostics(ddcc_ctx* ctx, int every);

/* The record of the periodic checks: the masses of the last check (NaN if
 * none has run yet) into mass[nphase] (may be NULL), its time level into
 * *t_checked (-1 if none), and the first level whose check saw a
 * non-finite population into *t_nonfinite (-1 if none). DDCC_E_STATE if
 * the checks are off. Synchronises. */
int ddcc_diagnostics(ddcc_ctx* ctx, double* mass, int64_t* t_checked,
                     int64_t* t_nonfinite);

/* ---- Adjoint (reverse-time) sweep ------------------------------------------
 * Gradient of a phase-weighted objective of the state after nsteps steps,
 *   J = sum_x w(x) phi C_k(x) / sum_x phi C_k(x),   phi C_k = sum_p f^k_p,
 * (w(x) = x, the node index along x, gives the centroid x of phase k; an
 * indicator of a region gives the fraction of phase k inside it) with
 * respect to the per-node wetting angles cos theta_iN (eq. 2.9) and the
 * smooth characteristic function psi (Section 2), the state at the call
 * (populations and history) held fixed. The derivative is that of the
 * library's discrete step, transposed by hand stage by stage: collision
 * (eqs. 3.1-3.4), equilibria and sources (3.5-3.12), force and velocity
 * (3.13), pressure (eq. 19), chemical potential (2.14), mobility (2.5),
 * the finite-difference stencils, pull streaming. |grad psi| is taken to
 * have derivative 0 where grad psi = 0.
 *
 * Runs the nsteps forward steps (checkpointing the state every `interval`
 * steps on the device), evaluates J, then sweeps back one segment of
 * `interval` steps at a time, recomputing the segment's states from its
 * checkpoint; the next segment is recomputed on a second stream of
 * default priority while the current one is swept. Device memory: about
 * (nsteps / interval + 2 interval + 1) states plus a few adjoint states,
 * released on return. On success the
 * context is left at the final level (time advanced by nsteps).
 *
 * weight     host [ny][nx] float64, finite (the w above)
 * phase      k in [0, nphase)
 * J          host scalar out (may be NULL)
 * grad_cos   host [nphase - 1][ny][nx] out: dJ/dcos theta_iN (may be NULL)
 * grad_psi   host [ny][nx] out: dJ/dpsi (may be NULL)
 * Needs a 2D FP64 or FP32 context whose geometry came from one wall
 * (ddcc_init_geometry). Errors: DDCC_E_INVAL (bad argument), DDCC_E_STATE
 * (before init_fields), DDCC_E_UNSUPPORTED (3D, 16-bit storage, several
 * walls), DDCC_E_NONFINITE (zero or non-finite phase mass at the end),
 * DDCC_E_NOMEM, DDCC_E_HIP. Synchronises. */
int ddcc_adjoint(ddcc_ctx* ctx, int64_t nsteps, int interval, int phase,
                 const double* weight, double* J, double* grad_cos,
                 double* grad_psi);

/* The objective J of ddcc_adjoint on the current state, without stepping:
 * sum_x w(x) phi C_k(x) / sum_x phi C_k(x) in float64. weight: host
 * [ny][nx]. 2D FP64 or FP32 contexts. Errors as ddcc_adjoint. Synchronises. */
int ddcc_objective(ddcc_ctx* ctx, int phase, const double* weight, double* J);

/* Kernel launch shape of the step kernel: tile (tx, ty) of nodes per
 * workgroup; 0 keeps the default. tx is 64 (one wavefront per row); ty is
 * 2, 4, 8 or 16 in 2D (default 4 for DDCC_FP64, 8 otherwise) and 2 or 4
 * in 3D (default 4). Any other value returns DDCC_E_INVAL. Takes effect on
 * the next ddcc_step; results do not depend on the tile. */
int ddcc_set_tile(ddcc_ctx* ctx, int tx, int ty);

/* Times `steps` steps (after two untimed ones) with each tile height (2, 4,
 * 8, 16 in 2D; 2, 4 in 3D) on the current state and keeps the fastest for
 * later steps; the state and time level are restored afterwards, bit for
 * bit. The chosen height is written to *ty_out if not NULL. Needs
 * init_fields; allocates a temporary device copy of the state (populations,
 * history, T) and returns DDCC_E_NOMEM, with the state and tile untouched,
 * if that copy does not fit. Synchronises. */
int ddcc_autotune(ddcc_ctx* ctx, int steps, int* ty_out);

/* Message of the last failed call on ctx (never NULL; "" if none). */
const char* ddcc_last_error(const ddcc_ctx* ctx);

/* Releases the context and its device memory; NULL is a no-op. */
void ddcc_destroy(ddcc_ctx* ctx);

/* Library version string. */
const char* ddcc_version(void);

/* ---- Batches of independent boxes -----------------------------------------
 * Many independent 2D D2Q9 instances of the same method and parameters, on
 * grids of different sizes, advanced together: one persistent kernel launch
 * per time step drains a queue of (instance, tile) work items, and
 * ddcc_batch_set_graph captures groups of steps in a HIP graph. Each
 * instance's state, inputs and outputs are exactly those of a single context
 * of its size (same layouts as the single-context calls, per instance).
 * Every plane of every device field holds all instances one after another,
 * so the batch owns one allocation per field. */
typedef struct ddcc_batch ddcc_batch;

/* Creates a batch of count instances with grids nx[i] x ny[i] (host
 * arrays, copied) and the method parameters of *params (dim must be 2; its
 * nx, ny, nz are ignored). hip_stream as for ddcc_create; NULL creates a
 * stream of the library's own (the legacy default stream cannot be
 * captured). Total nodes at most 2^29. Errors: DDCC_E_INVAL,
 * DDCC_E_UNSUPPORTED (dim != 2), DDCC_E_NOMEM, DDCC_E_HIP. */
int ddcc_batch_create(const ddcc_params* params, int count, const int* nx,
                      const int* ny, void* hip_stream, ddcc_batch** out);

/* Method parameters of instance i alone (parameter samples: densities,
 * viscosities, surface tensions, mobility, rates, forces ...), replacing the
 * batch's for that instance; dim, nphase, the lattices and the precision
 * must be the batch's (DDCC_E_INVAL otherwise), and the parameters are
 * validated as in ddcc_create. Call it before the instance's
 * ddcc_batch_init_fields (the initial equilibrium uses them); it may also be
 * called later, and then takes effect on the next step. Synchronises. */
int ddcc_batch_set_params(ddcc_batch* b, int i, const ddcc_params* params);

/* Geometry of instance i: psi [ny_i][nx_i] in [0, 1] and the N-1 wetting
 * cosines cos theta_iN [N-1][ny_i][nx_i] in [-1, 1] (NULL: 90 degrees).
 * Resets the instance's fields (init_fields again before stepping). */
int ddcc_batch_init_geometry(ddcc_batch* b, int i, const double* psi,
                             const double* cos_theta_iN);

/* Initial C [N][ny_i][nx_i], u [2][ny_i][nx_i] (NULL: 0), P (NULL: 0) of
 * instance i, populations at equilibrium (as ddcc_init_fields).
 * DDCC_E_STATE before its geometry. Synchronises the batch stream. */
int ddcc_batch_init_fields(ddcc_batch* b, int i, const double* C,
                           const double* u, const double* P);

/* Advances every instance by nsteps time steps (asynchronous on the batch
 * stream). DDCC_E_STATE unless every instance has its fields. */
int ddcc_batch_step(ddcc_batch* b, int64_t nsteps);

/* C, u, P of instance i at the current step (layouts as init_fields; NULL
 * skips). Synchronises. */
int ddcc_batch_read_moments(ddcc_batch* b, int i, double* C, double* u,
                            double* P);

/* Per-phase totals of instance i, float64 (as ddcc_mass). Synchronises. */
int ddcc_batch_mass(ddcc_batch* b, int i, double* mass);

/* Tile height of the step kernel: 4, 8 (default) or 16 rows of 64 nodes. */
int ddcc_batch_set_tile(ddcc_batch* b, int ty);

/* Times `steps` steps with each tile height and keeps the fastest; the
 * state is restored afterwards (the trial steps are not counted). The
 * chosen height is written to *ty_out if not NULL. Needs every instance's
 * fields; allocates a temporary copy of the state. */
int ddcc_batch_autotune(ddcc_batch* b, int steps, int* ty_out);

/* Steps per captured HIP graph: 0 (default) launches every step directly;
 * an even number in [2, 1024] replays graphs of that many steps (the rest
 * of a ddcc_batch_step call is launched directly). */
int ddcc_batch_set_graph(ddcc_batch* b, int steps_per_graph);

/* Waits for the batch stream. */
int ddcc_batch_sync(ddcc_batch* b);

/* Steps taken since the batch was created (-1 for NULL). */
int64_t ddcc_batch_time(const ddcc_batch* b);

/* Message of the last failed call on b (never NULL). */
const char* ddcc_batch_last_error(const ddcc_batch* b);

/* Releases the batch and its device memory; NULL is a no-op. */
void ddcc_batch_destroy(ddcc_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* DDCC_H */
