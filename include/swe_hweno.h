/*
 * swe_hweno.h — C ABI of the MI355X (gfx950) solver for the well-balanced fifth-order
 * finite-difference Hermite WENO scheme for the shallow water equations in pre-balanced form
 * (Zhao & Zhang, arXiv 2208.01260).
 *
 * What the library computes (in FP64; the _f32 entry points run the same scheme in FP32):
 *   - the semi-discrete right-hand side of Sec. 2.1 (1D, eq. (2.8)) and Sec. 3 (2D, eq. (3.8)):
 *     Lax-Friedrichs split (eq. (2.4)), characteristic-wise nonlinear HWENO reconstruction of the
 *     original-equation fluxes (eqs. (2.5), (2.7)), linear Hermite derivative fluxes (eq. (2.6)),
 *     the source split that reuses the flux weights (Step 2), and in 2D the four-point mixed
 *     terms (eq. (3.7));
 *   - the HWENO derivative limiter of Sec. 2.2 (eqs. (2.12), (2.13)), dimension by dimension;
 *   - SSP-RK3 with modified derivatives (eq. (2.11)) at CFL-limited time steps.
 *
 * Conventions:
 *   - All array arguments are DEVICE pointers to contiguous FP64 data unless stated otherwise.
 *   - Node (i, j) sits at the cell centre (x0 + (i + 1/2) dx, y0 + (j + 1/2) dy).
 *   - A state is a stack of planes [field][ny][nx], x fastest:
 *       dim = 1: eta = h + b, m = hu, H = eta_x, M = m_x                            (4 planes, ny = 1)
 *       dim = 2: eta, m = hu, w = hv, H1 = eta_x, M1 = m_x, W1 = w_x,
 *                H2 = eta_y, M2 = m_y, W2 = w_y                                      (9 planes)
 *   - The bottom b and its derivatives bx = b_x, by = b_y are single planes.
 *   - Readings where the paper is silent: alpha of the Lax-Friedrichs split is global per
 *     direction and per right-hand-side evaluation (max |u| + sqrt(g h), max |v| + sqrt(g h));
 *     interface eigenvectors use the arithmetic mean of the two adjacent nodes; the limiter uses
 *     the node's own state; the right-hand side of each stage takes the unmodified stage
 *     derivatives; dt = cfl / (alpha_x/dx + alpha_y/dy) from the state at the start of a step.
 *
 * Errors: every entry point returns an int status (SWE_OK or a negative code); nothing is
 * thrown across the ABI. Argument errors are detected on the host before any HIP call.
 * Device-detected dry (h <= 0) or non-finite states set a sticky flag in the context that
 * swe_hweno_run and swe_hweno_sync report.
 *
 * Streams: every call enqueues on the stream given to swe_hweno_init. swe_hweno_rhs,
 * swe_hweno_limit and swe_hweno_step (with dt_used == NULL) do not synchronise; the caller's
 * arrays must stay valid until the stream reaches the enqueued work. Calls on one context
 * must not overlap from several host threads.
 */
#ifndef SWE_HWENO_H
#define SWE_HWENO_H

#ifdef __cplusplus
extern "C" {
#endif

#define SWE_HWENO_ABI_VERSION 1

enum {
  SWE_OK = 0,
  SWE_EINVAL = -1,     /* invalid argument (null pointer, size, parameter out of range) */
  SWE_ENOMEM = -2,     /* device allocation failed */
  SWE_EHIP = -3,       /* a HIP runtime call failed */
  SWE_EDRY = -4,       /* a node with h = eta - b <= 0 was met */
  SWE_ENONFINITE = -5  /* a non-finite value was met */
};

enum { SWE_BC_PERIODIC = 0, SWE_BC_REFLECTIVE = 1 };

/* flags */
enum {
  SWE_FIXED_DT = 1,     /* every step uses params.fixed_dt instead of the CFL step */
  SWE_FIXED_ALPHA = 2,  /* every right-hand side uses params.alpha_x / alpha_y */
  SWE_NO_LIMITER = 4,   /* skip the derivative limiter (D^mod = D) */
  SWE_CHECK_DRY = 8     /* swe_hweno_rhs and swe_hweno_step synchronise and report device-detected
                           dry or non-finite nodes (as swe_hweno_sync) instead of leaving them to a
                           later swe_hweno_sync or swe_hweno_run */
};

typedef struct swe_hweno_ctx swe_hweno_ctx; /* opaque, owned by the library */

typedef struct {
  int dim;                  /* 1 or 2 */
  int nx, ny;               /* nodes per direction; nx >= 4; ny >= 4 (dim 2) or ny == 1 (dim 1) */
  double x0, x1, y0, y1;    /* domain; x1 > x0 (and y1 > y0 in 2D) */
  double g;                 /* gravitational constant, > 0 (the paper uses 9.812, Sec. 4) */
  double cfl;               /* CFL number, > 0 (the paper uses 0.6, Sec. 4) */
  double eps;               /* epsilon of the nonlinear weights, >= 1e-20 (1e-6, eq. (2.7)) */
  int bc_x, bc_y;           /* SWE_BC_PERIODIC or SWE_BC_REFLECTIVE (mirror about the wall face) */
  int flags;                /* SWE_FIXED_DT | SWE_FIXED_ALPHA | SWE_NO_LIMITER | SWE_CHECK_DRY */
  double fixed_dt;          /* > 0 when SWE_FIXED_DT is set */
  double alpha_x, alpha_y;  /* > 0 when SWE_FIXED_ALPHA is set (alpha_y ignored in 1D) */
} swe_hweno_params;

/* Create a context for the semi-discrete scheme of Sec. 2.1 (1D) or Sec. 3 (2D) on the grid and
 * parameters of params (g, the CFL number and epsilon as in Sec. 4 and eq. (2.7)): validates
 * params, allocates the stage buffers (about 2.7 states of device memory in 2D), copies the
 * bottom planes b, bx (and by when dim = 2; pass NULL in 1D) from the caller's device memory.
 * stream is a hipStream_t (NULL = the null stream). On error *out is left NULL and nothing is
 * allocated. */
int swe_hweno_init(const swe_hweno_params* params, const double* b, const double* bx, const double* by,
                   void* stream, swe_hweno_ctx** out);

/* Right-hand side R(state) of the semi-discrete scheme (eq. (2.8) / (3.8)): rhs has the layout
 * of state. alpha_x < 0 computes alpha from the state on the device (then alpha_y is ignored);
 * otherwise the given alpha_x (and alpha_y in 2D) are used and must be finite and positive
 * (NaN is SWE_EINVAL). state and rhs must not overlap. A node with h <= 0, or a non-finite
 * result, sets the context's error flag (reported by swe_hweno_sync, or by this call with
 * SWE_CHECK_DRY); its right-hand side values are then meaningless. */
int swe_hweno_rhs(swe_hweno_ctx* ctx, const double* state, double* rhs, double alpha_x, double alpha_y);

/* Limited derivatives Lim(state) (Sec. 2.2, eq. (2.13)): dmod receives 2 planes (H, M) in 1D or
 * 6 planes (H1, M1, W1, H2, M2, W2) in 2D. */
int swe_hweno_limit(swe_hweno_ctx* ctx, const double* state, double* dmod);

/* Lax-Friedrichs speeds of a state: alpha_host[0] = max |u| + c, alpha_host[1] = max |v| + c
 * (HOST array of 2). Synchronises the stream. Returns SWE_EDRY / SWE_ENONFINITE if met. */
int swe_hweno_alpha(swe_hweno_ctx* ctx, const double* state, double* alpha_host);

/* One SSP-RK3 step (eq. (2.11)) of state in place. dt <= 0 takes the CFL step (or fixed_dt with
 * SWE_FIXED_DT). If dt_used (HOST pointer) is not NULL the call synchronises and stores the dt. */
int swe_hweno_step(swe_hweno_ctx* ctx, double* state, double dt, double* dt_used);

/* nsteps SSP-RK3 steps (eq. (2.11) of Sec. 2.2, each as swe_hweno_step) of state in place,
 * replaying a captured per-step HIP graph. With t_end > 0 it stops at t_end (the last step
 * clipped to it; nsteps <= 0 means "until t_end"); t_out and steps_out (HOST, nullable) receive
 * the time reached and the steps taken. Synchronises and returns device-detected errors. */
int swe_hweno_run(swe_hweno_ctx* ctx, double* state, int nsteps, double t_end, double* t_out, int* steps_out);

/* Synchronise the context's stream and report (and clear) a device-detected error. */
int swe_hweno_sync(swe_hweno_ctx* ctx);

/* Free the context (synchronises its stream first). NULL is a no-op. */
void swe_hweno_destroy(swe_hweno_ctx* ctx);

/* Static message for a status code. */
const char* swe_hweno_strerror(int code);

/* SWE_HWENO_ABI_VERSION of the built library. */
int swe_hweno_abi_version(void);

/* Kernel timing with HIP events on the context's stream. swe_hweno_set_timing(ctx, 1) turns it on
 * (and resets the totals): swe_hweno_run then launches each step's kernels directly instead of
 * replaying its graph, with an event pair around every fused stage kernel, and swe_hweno_rhs
 * brackets its kernel too. swe_hweno_get_timing synchronises and returns, in HOST arrays of 4,
 * the summed milliseconds and launch counts of [bare right-hand side, stage 1, stage 2, stage 3]. */
int swe_hweno_set_timing(swe_hweno_ctx* ctx, int on);
int swe_hweno_get_timing(swe_hweno_ctx* ctx, double* ms, long long* launches);

/* One SSP-RK3 step (as swe_hweno_step) with no context and no device allocation. For callers
 * that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). The stage buffers and device scalars live in one static
 * device array of swe_hweno_noalloc_capacity() bytes (32 MiB), one copy per GPU, held by the
 * library until the process ends. A grid needs 256 bytes plus 24 planes (2D) or 10 planes (1D)
 * of nx*ny doubles; a larger grid is rejected with SWE_EINVAL (2D: at most 174,761 nodes, e.g.
 * 418 x 418). params, state, dt and dt_used as for swe_hweno_init and swe_hweno_step (FP64);
 * b, bx and by (NULL in 1D) are read in place, not copied, and must stay valid until the stream
 * (a hipStream_t, NULL = the null stream) reaches the step. The call allocates nothing (no
 * hipMalloc, hipFree or allocating library routine) and, with dt_used == NULL, does not
 * synchronise. Every call on one GPU uses that GPU's single array and overwrites what the
 * previous call left: calls that overlap on one GPU (several streams or host threads) race
 * and must be serialised by the caller. Device-detected errors are reported only through a
 * non-NULL dt_used (the call then synchronises). */
int swe_hweno_step_noalloc(const swe_hweno_params* params, double* state, const double* b, const double* bx,
                           const double* by, double dt, void* stream, double* dt_used);
/* Bytes of the static device array behind swe_hweno_step_noalloc. Host-only, no HIP call. */
unsigned long swe_hweno_noalloc_capacity(void);

/* ------------------------------------------------------------------------------------------
 * Single precision. The same scheme, kernels and launch shapes with every array and all device
 * arithmetic in FP32 (the paper's lake-at-rest tables report single, double and quadruple
 * precision runs, Sec. 4, Tables 1-3). A context made by swe_hweno_init_f32 takes float planes
 * (same layouts as above) and only the _f32 calls below plus the type-free ones (sync,
 * destroy, timing, tile); an FP64 call on it, or an _f32 call on an FP64 context, returns
 * SWE_EINVAL. Parameters, alpha and dt stay double on the host; the speeds are reduced in
 * FP32 and dt is formed in FP64 from them. swe_hweno_init_f32 also rejects eps < 1e-9: the
 * unnormalised nonlinear weights are of order eps^4 where the data are flat and must stay
 * normal floats (they overflow for smoothness indicators above about 1e9).
 * ------------------------------------------------------------------------------------------ */
int swe_hweno_init_f32(const swe_hweno_params* params, const float* b, const float* bx, const float* by,
                       void* stream, swe_hweno_ctx** out);
int swe_hweno_rhs_f32(swe_hweno_ctx* ctx, const float* state, float* rhs, double alpha_x, double alpha_y);
int swe_hweno_limit_f32(swe_hweno_ctx* ctx, const float* state, float* dmod);
int swe_hweno_alpha_f32(swe_hweno_ctx* ctx, const float* state, double* alpha_host);
int swe_hweno_step_f32(swe_hweno_ctx* ctx, float* state, double dt, double* dt_used);
int swe_hweno_run_f32(swe_hweno_ctx* ctx, float* state, int nsteps, double t_end, double* t_out, int* steps_out);

/* Dimensions of the fused stage kernel's tiles (columns of output per wavefront and the default
 * rows per wavefront march); for tests and benchmarks. Host-only, no HIP call. */
int swe_hweno_tile(int* cols_per_wave, int* rows_per_wave);

/* The tile a context uses: rows per march are chosen at init from the grid and the device's
 * compute-unit count (environment variable SWE_HWENO_ROWS overrides). Host-only. */
int swe_hweno_ctx_tile(const swe_hweno_ctx* ctx, int* cols_per_wave, int* rows_per_wave);

/* The library's own arithmetic building blocks, applied elementwise on the device for
 * verification against IEEE division and square root. Each is correctly rounded on its domain:
 * which = 0: y = 1/x (hardware reciprocal estimate and two Newton steps; 2^-1021 <= |x| <= 2^1021),
 * 1: y = sqrt(x) (reciprocal square root estimate, one Goldschmidt step and two corrections;
 * 2^-1000 <= x), 2: y = x/3 (product with the rounded 1/3 and one FMA correction of the exact
 * remainder; x = 0, returned as +0, or 2^-1000 <= |x|). Outside those domains (where the residuals
 * are subnormal) the last bit may differ. x and y are DEVICE arrays of n doubles, stream a
 * hipStream_t; the call synchronises. */
int swe_hweno_math_check(int which, const double* x, double* y, unsigned long n, void* stream);

/* sha256 (first 16 hex digits) of the sources the library was built from (its HIP sources,
 * this header and the compiler flags). The Python binding refuses a library whose stamp does
 * not match the sources beside it. Host-only. */
const char* swe_hweno_source_hash(void);

/* ------------------------------------------------------------------------------------------
 * Batched solver: many independent 2D instances of uneven sizes, each with its own bottom,
 * state, Lax-Friedrichs speeds and CFL time step, advanced together. Every stage of every
 * instance is one launch of the fused stage kernel over all instances' tiles (a per-wavefront
 * table maps each wavefront to its instance and tile), and the steps of a run are replayed
 * from captured HIP graphs of at most 16 steps. Each step is the one swe_hweno_step takes (the
 * scheme of Sec. 2 and 3 of the paper: SSP-RK3 stages, each a full right-hand side, limiter and
 * update). Each instance's result is bitwise the result of the plain solver on the same
 * instance with the same rows per march: the batch tiling changes no arithmetic. FP64 only.
 * ------------------------------------------------------------------------------------------ */
typedef struct swe_hweno_batch swe_hweno_batch; /* opaque, owned by the library */

typedef struct {
  int nx, ny;               /* nodes, >= 4 each */
  double x0, x1, y0, y1;    /* domain */
  int bc_x, bc_y;           /* SWE_BC_PERIODIC or SWE_BC_REFLECTIVE */
  const double* b;          /* DEVICE planes of nx*ny: bottom and its x-, y-derivatives (copied at init) */
  const double* bx;
  const double* by;
  double* state;            /* DEVICE, 9 planes of nx*ny, caller-owned; advanced in place by batch_run */
} swe_hweno_instance;

/* Create a batch of `count` (1..65535) instances. From `common` only g, cfl, eps, flags,
 * fixed_dt, alpha_x, alpha_y are used (dim must be 2; nx, ny, domain and bc are per instance).
 * The instance array is read during the call only; the state pointers are kept and must stay
 * valid while the batch exists. */
int swe_hweno_batch_init(const swe_hweno_params* common, const swe_hweno_instance* inst, int count, void* stream,
                         swe_hweno_batch** out);

/* nsteps SSP-RK3 steps of every instance (each at its own CFL step; no end time), replayed from
 * captured graphs. Every run starts each instance's clock at 0 and its speeds from its current
 * state; t_out (HOST array of count, nullable) receives the time each instance advanced.
 * Synchronises. An instance whose time step turns non-finite, or whose state is found dry or
 * non-finite (by the speeds of its initial state or of a stage's result), stops at the start of
 * the next step while the others go on: its state stays that of the step in which the error was
 * met (unchanged if its initial state was bad), and the call returns SWE_ENONFINITE (SWE_EDRY).
 * The error is then cleared: a later run steps the instance again. nsteps < 1 is SWE_EINVAL. */
int swe_hweno_batch_run(swe_hweno_batch* bt, int nsteps, double* t_out);

/* Rows per wavefront march of the batch kernels (>= 1); swe_hweno_batch_autotune times the
 * first two fused stage kernels of a step (limiter as configured) on the batch's own data for a
 * set of candidates (8 to 64 rows; they write only the batch's stage buffers, the states are not
 * touched), keeps the fastest and returns it. Rows per march are the tile's one free dimension:
 * its width is the 60 output columns of a 64-lane wavefront. The choice is cached for the life
 * of the process per size class: the device's architecture and compute-unit count and
 * power-of-two buckets of the instance count, the total nodes and the largest instance width
 * and height. A batch of a class already tuned takes the cached rows without timing. The cache
 * is shared by all threads (guarded by a mutex); tune_cache_size counts its entries and
 * tune_cache_clear empties it (host-only, no HIP call). */
int swe_hweno_batch_set_rows(swe_hweno_batch* bt, int rows);
int swe_hweno_batch_autotune(swe_hweno_batch* bt, int* rows_out);
int swe_hweno_batch_tune_cache_size(void);
void swe_hweno_batch_tune_cache_clear(void);

/* Synchronise and report (and clear) device-detected errors of any instance. */
int swe_hweno_batch_sync(swe_hweno_batch* bt);

/* Free the batch (synchronises first). NULL is a no-op. */
void swe_hweno_batch_destroy(swe_hweno_batch* bt);

/* ------------------------------------------------------------------------------------------
 * Adjoint (reverse mode), 2D FP64 contexts. Vector-Jacobian products of the scheme with the
 * Lax-Friedrichs speeds frozen: of the right-hand side (eq. (3.8), with the split of eq. (2.4),
 * the weights of eqs. (2.5)-(2.7), the source split of Step 2 and the mixed terms of eq. (3.7)),
 * of the limiter (Sec. 2.2, eq. (2.13)) and of a run of SSP-RK3 steps (eq. (2.11)) at a fixed dt.
 * The bottom b and its slopes bx, by enter as independent inputs; swe_hweno_bottom_slopes and
 * its transpose tie them together when the gradient with respect to b alone is wanted. Work
 * buffers are allocated on first use and kept with the context until swe_hweno_destroy: about
 * 170 planes of nx*ny doubles, plus 27 per step of the checkpoint interval (the recomputed stage
 * states of one segment) and 9 per checkpoint. All arrays are DEVICE arrays; outputs are
 * overwritten. FP64 contexts only (an FP32 context returns SWE_EINVAL).
 * ------------------------------------------------------------------------------------------ */

/* rbar (state layout) is the adjoint of R(state) with alpha = (alpha_x, alpha_y) > 0 fixed.
 * sbar (state layout) receives rbar^T dR/dstate; bbar, bxbar, bybar (planes) receive
 * rbar^T dR/db, dR/dbx, dR/dby. */
int swe_hweno_rhs_vjp(swe_hweno_ctx* ctx, const double* state, double alpha_x, double alpha_y, const double* rbar,
                      double* sbar, double* bbar, double* bxbar, double* bybar);

/* dmbar (6 planes: H1, M1, W1, H2, M2, W2) is the adjoint of Lim(state); sbar (state layout)
 * and bbar receive its products with dLim/dstate and dLim/db. */
int swe_hweno_limit_vjp(swe_hweno_ctx* ctx, const double* state, const double* dmbar, double* sbar, double* bbar);

/* Reverse of nsteps steps of swe_hweno_run from state0 (not modified). The context must have
 * SWE_FIXED_DT and SWE_FIXED_ALPHA set (the map is then smooth). sbar_T (state layout) is the
 * adjoint of the final state; sbar_0 receives the adjoint of state0 and bbar, bxbar, bybar
 * those of the bottom planes. The stage states are recomputed from checkpoints stored every
 * checkpoint_every steps (>= 1). Synchronises; returns SWE_EDRY / SWE_ENONFINITE if the
 * recomputed forward run met them. */
int swe_hweno_run_vjp(swe_hweno_ctx* ctx, const double* state0, int nsteps, int checkpoint_every,
                      const double* sbar_T, double* sbar_0, double* bbar, double* bxbar, double* bybar);

/* The same reverse in two halves, for callers that run the forward themselves (an autograd
 * forward): swe_hweno_run_checkpointed advances state in place by nsteps steps (as
 * swe_hweno_run; same flags required) and keeps the states at the start of every
 * checkpoint_every steps in the context; swe_hweno_run_vjp_checkpointed then runs the reverse
 * of that run from those checkpoints (nsteps and checkpoint_every must match, else SWE_EINVAL;
 * a swe_hweno_run_vjp call on the context in between discards them). Outputs as for
 * swe_hweno_run_vjp. */
int swe_hweno_run_checkpointed(swe_hweno_ctx* ctx, double* state, int nsteps, int checkpoint_every);
int swe_hweno_run_vjp_checkpointed(swe_hweno_ctx* ctx, int nsteps, int checkpoint_every, const double* sbar_T,
                                   double* sbar_0, double* bbar, double* bxbar, double* bybar);

/* Bottom slopes by the fourth-order centred difference
 *   bx_i = (b_{i-2} - 8 b_{i-1} + 8 b_{i+1} - b_{i+2}) / (12 dx)   (by likewise along y),
 * with b extended through the boundary (periodic wrap, or even about a reflective wall), for
 * the grid of params (dim 2), on a hipStream_t. The _vjp form adds the transpose of that map
 * applied to (bxbar, bybar) into bbar. */
int swe_hweno_bottom_slopes(const swe_hweno_params* params, const double* b, double* bx, double* by, void* stream);
int swe_hweno_bottom_slopes_vjp(const swe_hweno_params* params, const double* bxbar, const double* bybar,
                                double* bbar, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SWE_HWENO_H */
