/*
 * fde.h -- C ABI of libfde, an MI355X (gfx950) solver for the per-time-step linear systems of the
 * Crank-Nicolson weighted-and-shifted-Grunwald (CN-WSGD) discretisation of the 2-D two-sided
 * space-fractional diffusion equation, preconditioned by multigrid (Moghaderi, Dehghan, Donatelli,
 * Mazza, "Spectral analysis and multigrid preconditioners for two-dimensional space-fractional
 * diffusion equations").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - A "field" is an array of n1*n2 values for the interior grid points, row-major [n2][n1]: row j is
 *    y_{j+1}, column i is x_{i+1}, x varies fastest.  This is the lexicographic ordering of the vectors
 *    u, d+-, e+-, v in Sec. 2 of the paper.
 *  - Every array argument is a DEVICE pointer (HIP device memory of the current device), FP64, owned
 *    by the caller.  The library never frees or retains caller memory after a call returns.
 *  - The grid: x_i = a1 + i*hx, hx = (b1-a1)/(n1+1), i = 1..n1 (likewise y); tau is the time step
 *    (Sec. 2, grid definition).
 *  - The operator.  With T_g = [w_{i-j+1}] the lower-Hessenberg Toeplitz matrix of the WSGD weights
 *    (eq. (AN): the paper's A^g is -T_g; weights of eq. (w) from the Grunwald coefficients of eq. (gk)),
 *        L u = D+ (I kron T_a) u/hx^a + D- (I kron T_a^T) u/hx^a + E+ (T_b kron I) u/hy^b
 *              + E- (T_b^T kron I) u/hy^b                                  (eq. (AxAy)),
 *    and each CN step solves (I - tau/2 L^(m)) u^(m) = (I + tau/2 L^(m-1)) u^(m-1) + tau v^(m-1/2)
 *    (eq. (CNWSGD), matrix form eq. (system)).  The paper's scaled matrix of eq. (M) is this system
 *    matrix times 1/r, r = tau/(2 hx^a): the same solution and the same relative residuals.
 *  - Work is ordered on the handle's HIP stream.  Calls that return statistics synchronise that
 *    stream; all others are asynchronous.  One handle must not be used by two host threads at once.
 *  - Return value: 0 on success, a negative FDE_E* code on a usage or device error, FDE_ENOCONV (> 0)
 *    when the iteration limit was reached (outputs then hold the last iterate).  The text of the last
 *    error of a handle is available from fde_last_error; errors raised before a handle exists are
 *    available from fde_last_error(NULL).  No C++ exception crosses this interface.
 */
#ifndef FDE_H
#define FDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------------------------------- */
#define FDE_OK 0
#define FDE_EINVAL (-1)      /* invalid argument (range, null pointer, unsupported size)            */
#define FDE_ENEGCOEF (-2)    /* a diffusion coefficient is negative (Sec. 2 requires d, e >= 0)    */
#define FDE_ENOMEM (-3)      /* device allocation failed or the request exceeds a memory budget    */
#define FDE_ENONFINITE (-4)  /* NaN or Inf in an input or in the iterate                           */
#define FDE_EDEVICE (-5)     /* a HIP runtime error                                                */
#define FDE_EAGAIN (-6)      /* batch: the request does not fit now; retry after others finish     */
#define FDE_ENOCONV 1        /* iteration limit reached before the tolerance                       */

/* ---- options ---------------------------------------------------------------------------------- */
#define FDE_FP64 0             /* every kernel in FP64                                              */
#define FDE_MIXED_FP32 1       /* multigrid preconditioner in FP32 inside FP64 flexible GMRES        */
#define FDE_MIXED_BF16GEMM 2   /* as FDE_MIXED_FP32; the rediscretised levels too large for the dense
                                  kernel (n > 255) apply their Toeplitz factors as BF16 MFMA products
                                  with FP32 accumulation instead of FP32 FFTs                        */
#define FDE_MIXED_FP32_CYCLE 3 /* as FDE_MIXED_FP32, and each restart cycle in FP32 too: the Krylov
                                  basis is stored in FP32 and A z_j is the preconditioner's FP32
                                  fine-level operator (dot products, norms and the least-squares
                                  problem stay FP64).  Every cycle starts from the FP64 true residual
                                  b - A x and adds its correction to the FP64 iterate, so a restarted
                                  solve is iterative refinement with FP32 inner solves and the
                                  tolerance still holds for the FP64 residual.  Needs a rediscretised
                                  fine level: not with FDE_MG_BAND                                 */
#define FDE_MIXED_CYCLE_BF16 4 /* as FDE_MIXED_FP32_CYCLE with the Krylov basis stored in BF16: each
                                  new direction is orthogonalised in FP32 and stored rounded to BF16
                                  (a basis orthonormal to about 3 digits, enough for the modest
                                  reduction each restart cycle delivers on solves that take many
                                  cycles; a solve that would end inside its first cycle takes a
                                  second one); half the Gram-Schmidt traffic again.  Not with
                                  FDE_MG_BAND                                                       */

#define FDE_MG_GEOMETRIC 0     /* rediscretised coarse operators, Sec. 4.2 (the paper's P_MGM)      */
#define FDE_MG_GALERKIN 1      /* Galerkin coarse operators R A P, Sec. 4 TGM step 3 (tilde P_MGM)   */
#define FDE_MG_BAND 2          /* the band preconditioner P_2 = (1/r) I - (P_x + (s/r) P_y) of
                                  Sec. 4.3: the system matrix with the Laplacian matrix
                                  tridiag(1, -2, 1) in place of both fractional factors and the
                                  same scalings r = tau/(2 hx^alpha), s = tau/(2 hy^beta), applied
                                  (as r P_2) through one Galerkin V-cycle; the outer operator stays
                                  fractional                                                       */

typedef struct fde_handle fde_handle;

/* Problem and solver description (Sec. 2 problem statement; Sec. 4.2 and Sec. 5 solver settings). */
typedef struct fde_problem {
  double alpha, beta;   /* fractional orders, each in (1,2) (Sec. 2)                               */
  int32_t n1, n2;       /* interior points in x and y, 2^l - 1 or 2^l with l >= 3, at most 2048; on
                           an odd side coarse point J sits at fine 2J + 1, on an even side at fine
                           2J (0-based; the down-sampling K of Sec. 4.1).  Even sides: geometric
                           hierarchy only, not with FDE_MIXED_BF16GEMM                           */
  double a1, b1, a2, b2;/* domain (a1,b1) x (a2,b2), a < b                                         */
  double tau;           /* time step, > 0                                                          */
  int32_t precision;    /* FDE_FP64 | FDE_MIXED_FP32 | FDE_MIXED_BF16GEMM | FDE_MIXED_FP32_CYCLE |
                           FDE_MIXED_CYCLE_BF16                                                     */
  int32_t mg_variant;   /* FDE_MG_GEOMETRIC | FDE_MG_GALERKIN | FDE_MG_BAND                        */
  double omega;         /* Jacobi damping (Lemma lemsmo), 0 < omega <= 1; 0 selects 0.7             */
  int32_t nu_pre;       /* pre-smoothing steps per level, >= 0 (< 0 selects 1)                      */
  int32_t nu_post;      /* post-smoothing steps per level, >= 0 (< 0 selects 1)                     */
  int32_t coarsest_n;   /* coarsen while min(n1,n2) > coarsest_n; 0 selects the paper's 8 x 8
                           coarsest grid (Sec. 4.2): 8 when both sides are 2^l (8 x 8 points),
                           else 7 (7 x 7 points, 8 x 8 cells)                                     */
  int32_t restart;      /* GMRES restart length, 1..32; 0 selects 20 (Sec. 5)                      */
  int32_t maxit;        /* total iteration limit per solve; 0 selects 5000 (enough for the
                           strongly anisotropic 2047^2 instances, which take ~530)              */
  double rtol;          /* stop when ||b - A x||_2 <= rtol ||b||_2; 0 selects 1e-10                */
} fde_problem;

/* Per-solve statistics. */
typedef struct fde_stats {
  int32_t iters;        /* GMRES iterations (preconditioner applications) in this solve           */
  int32_t restarts;     /* completed restart cycles beyond the first                               */
  int32_t converged;    /* 1 if the true relative residual met rtol                                */
  int32_t reorth_steps;  /* Arnoldi steps that took a second Gram-Schmidt pass: with an FP64
                           basis when the first pass left less than 1e-6 of ||w||^2, with FP32
                           restart cycles (FP32 or BF16 basis) less than 1/10.  The environment
                           variable FDE_REORTH_KEEP (a fraction in [0, 1], read by fde_setup)
                           overrides the threshold for measurements                             */
  double relres_true;   /* ||b - A x|| / ||b|| computed in FP64 from the returned x               */
  double relres_est;    /* the Arnoldi (Givens) estimate at exit                                   */
} fde_stats;

/* Fills *p with the defaults above for the given sizes, orders and time step (unit square). */
void fde_problem_default(fde_problem* p, double alpha, double beta, int32_t n1, int32_t n2,
                         double tau);

/* Creates a solver handle.  dp, dm, ep, em: the coefficient fields d+, d-, e+, e- at the time level
 * of the left-hand side (Sec. 2, D+- and E+- of eq. (AxAy)); they are copied, the caller keeps them.
 * The same fields are used for the explicit half of the next fde_step until fde_update_coeffs is
 * called.  Builds the multigrid hierarchy on the device (geometric: coefficients injected at the
 * coarse points, Sec. 4.2; Galerkin: R A P with R = P^T/4, Sec. 4), the Toeplitz symbols, and the
 * FP64 inverse of the coarsest-level matrix (Gauss-Jordan with partial pivoting).  stream: a hipStream_t (NULL = the default stream).
 * Errors: FDE_EINVAL, FDE_ENEGCOEF, FDE_ENONFINITE, FDE_ENOMEM, FDE_EDEVICE; *out is NULL then. */
int fde_setup(const fde_problem* p, const double* dp, const double* dm, const double* ep,
              const double* em, void* stream, fde_handle** out);

/* Time-dependent coefficients (Sec. 2: D^(m) at t^(m), D^(m-1) at t^(m-1)).  The current left-hand
 * side fields become the explicit (right-hand side) fields and the given fields become the new
 * left-hand side; the hierarchy is rebuilt on the device.  Errors as for fde_setup. */
int fde_update_coeffs(fde_handle* h, const double* dp, const double* dm, const double* ep,
                      const double* em);

/* One CN step (eq. (system)): b = (I + tau/2 L^(m-1)) u_prev + tau v_half, then solve
 * (I - tau/2 L^(m)) u_next = b with GMRES(restart) right-preconditioned by one V-cycle, zero initial
 * guess (Sec. 5).  v_half: the source at t^(m-1/2), may be NULL (no source).  u_next may not alias
 * u_prev.  stats may be NULL.  Returns 0, FDE_ENOCONV, or an error. */
int fde_step(fde_handle* h, const double* u_prev, const double* v_half, double* u_next,
             fde_stats* stats);

/* As fde_step with a separable source v_half = sum_k phi[k] * S[k], k < nsrc <= 4; phi is a HOST
 * array of scalars, S a HOST array of device pointers to fields. */
int fde_step_sources(fde_handle* h, const double* u_prev, int32_t nsrc, const double* phi,
                     const double* const* S, double* u_next, fde_stats* stats);

/* Solves (I - tau/2 L) x = b for the left-hand side operator (Sec. 2, eq. (system)) with the
 * configured preconditioned GMRES.  x may not alias b.  stats may be NULL. */
int fde_solve(fde_handle* h, const double* b, double* x, fde_stats* stats);

/* Multigrid as a stand-alone solver (the V-cycle iteration of Sec. 4 without a Krylov method):
 * x_{k+1} = x_k + MG(b - A x_k) from x_0 = 0, one V(nu_pre, nu_post) cycle in the handle's
 * preconditioner precision per iteration and the FP64 true residual after each, until
 * ||b - A x||_2 <= rtol ||b||_2 or max_cycles (>= 1) cycles.  stats->iters = cycles.  The error
 * contracts by the spectral radius of the V-cycle iteration matrix per cycle.  x may not alias b.
 * Returns 0, FDE_ENOCONV (x = last iterate) or an error. */
int fde_solve_mg(fde_handle* h, const double* b, double* x, int32_t max_cycles, fde_stats* stats);

/* Releases every device buffer of the handle.  NULL is ignored. */
void fde_destroy(fde_handle* h);

/* Message of the last error on h (or of the last failed fde_setup / batch call when h is NULL). */
const char* fde_last_error(const fde_handle* h);

/* ---- inspection and test hooks (the same kernels as the solver) ------------------------------ */

/* Number of multigrid levels (level 0 = the fine grid). */
int fde_num_levels(const fde_handle* h);
/* Interior sizes of a level: n1 = (n1_{l-1} - 1)/2 (coarse J <-> fine 2J, Sec. 4.1). */
int fde_level_size(const fde_handle* h, int level, int32_t* n1, int32_t* n2);

/* y = A_level x with A_level the level-`level` matrix of the preconditioner hierarchy (level 0 =
 * I - tau/2 L).  prec names the hierarchy: FDE_FP64 (FP64 handles) or FDE_MIXED_FP32 (the FP32
 * hierarchy of FDE_MIXED_FP32 and FDE_MIXED_BF16GEMM handles; inputs rounded to FP32, result widened
 * to FP64; BF16 levels use their MFMA products).  For level 0 and prec = FDE_FP64 this is the outer
 * FP64 operator of the solver, available on every handle. */
int fde_apply(fde_handle* h, int level, int prec, const double* x, double* y);

/* r = b - A_level x (the residual epilogue of the operator passes, as the V-cycle forms it before
 * restricting, Sec. 4 V-cycle), same levels, precisions and layout as fde_apply.  r may alias
 * neither x nor b. */
int fde_residual(fde_handle* h, int level, int prec, const double* b, const double* x, double* r);

/* One damped-Jacobi step on a level (Lemma lemsmo): x <- x + omega D^-1 (b - A x), D = diag(A).
 * With zero_guess != 0 the incoming x is ignored and treated as 0. */
int fde_smooth(fde_handle* h, int level, int prec, const double* b, double* x, int zero_guess);

/* Full-weighting restriction rc = P^T r / 4 from `level` to level+1 (Sec. 4.1, Sec. 4.2). */
int fde_restrict(fde_handle* h, int level, int prec, const double* r, double* rc);

/* Bilinear prolongation and correction x += P e from level+1 to `level` (Sec. 4.1, Lemma lemapp). */
int fde_prolong(fde_handle* h, int level, int prec, const double* e, double* x);

/* Exact solve on the coarsest level with the FP64 inverse of its matrix. */
int fde_coarse_solve(fde_handle* h, const double* b, double* x);

/* One V(nu_pre, nu_post) cycle with zero initial guess (Sec. 4 V-cycle, Sec. 4.2 settings) in the
 * handle's preconditioner precision: x = MG(b). */
int fde_vcycle(fde_handle* h, const double* b, double* x);

/* The pointwise diagonal of A_level (used by the Jacobi smoother), as FP64. */
int fde_level_diag(fde_handle* h, int level, double* diag);

/* ---- kernel timing -----------------------------------------------------------------------------
 * For performance reports: launches of the selected kernel families are bracketed by HIP events on
 * the handle's stream.  Launches issued for Arnoldi steps that the device skipped (after
 * convergence) are not counted.  bytes: the algorithmic bytes of the counted launches (every input
 * and output field once). */
#define FDE_KFAM_OUTER_Y 0   /* FP64 system operator, column (y) pass: Arnoldi products of FP64  */
                             /* cycles, true residuals, right-hand sides                        */
#define FDE_KFAM_OUTER_X 1   /* FP64 system operator, row (x) pass with epilogue                 */
#define FDE_KFAM_MG0_Y 2     /* fine-level FP32/FP64 preconditioner operator, FFT column pass    */
                             /* (with FP32 cycles also the Arnoldi products)                     */
#define FDE_KFAM_MG0_X 3     /* fine level: FFT row pass (residual / Jacobi; Arnoldi product with */
                             /* FP32 cycles), dense or MFMA passes                               */
#define FDE_KFAM_MGC_Y 4     /* coarser levels, FFT column pass                                  */
#define FDE_KFAM_MGC_X 5     /* coarser levels: FFT row pass, dense, Galerkin or MFMA kernels    */
#define FDE_KFAM_CGS 6       /* Gram-Schmidt passes, norms (the streaming kernels)               */
#define FDE_KFAM_TRANSFER 7  /* pre-smoothing from zero, restriction, prolongation               */
#define FDE_KFAM_COARSE 8    /* one-workgroup V-cycle of the small levels                        */
#define FDE_KFAM_UPDATE 9    /* x += Z y                                                         */
#define FDE_KFAM_CGS_FINALIZE 10 /* one-workgroup combination of the Gram-Schmidt partials, Givens  */
                                 /* (problems of up to 32 * 2048 unknowns combine them inside the  */
                                 /* pass, in its last workgroup, and never launch this family)     */
#define FDE_KFAM_COUNT 11
int fde_profile_enable(fde_handle* h, uint32_t family_mask);
/* Time only every `every`-th launch of each selected family (every >= 1; 1 after setup): each event
 * pair costs the stream a few microseconds, so a sparse sample keeps a timed run close to an
 * untimed one.  Pick a stride coprime to 3 and to the restart length so that the sample rotates
 * over the pass kinds and basis sizes.  Resets the launch counters. */
int fde_profile_stride(fde_handle* h, int every);
int fde_profile_read(fde_handle* h, int family, int64_t* launches, double* total_ms, double* bytes);
int fde_profile_reset(fde_handle* h);

/* Synchronises the handle's stream; returns FDE_EDEVICE if an asynchronous error occurred. */
int fde_sync(fde_handle* h);

/* ---- batching and serving ---------------------------------------------------------------------
 * A batch owns independent CN time-stepping requests (the recursion of eq. (CNWSGD)/(system), each
 * request with its own sizes, orders, coefficients and source), resident on the device and advanced
 * together: every request has its own stream, its restart cycles are replayed from a captured HIP
 * graph, and the host never blocks on one request while others can run.  Requests are admitted
 * against a device-memory budget (bytes); one that does not fit returns FDE_EAGAIN and can be
 * retried after others leave.  A request runs exactly the kernels it would run alone, in the same
 * order, so its result does not depend on the mix.  A batch is used from one host thread.
 */
typedef struct fde_batch fde_batch;

/* Device bytes a solver handle for problem *p needs while resident (hierarchy, Krylov storage,
 * fields); 0 if *p is invalid.  A batch request needs (2 + nsrc) * n1 * n2 * 8 bytes more. */
size_t fde_footprint(const fde_problem* p);

/* Creates an empty batch with a device-memory budget; `stream` is unused (every request gets a
 * stream of its own).  FDE_EINVAL if out is NULL. */
int fde_batch_create(size_t budget_bytes, void* stream, fde_batch** out);
void fde_batch_destroy(fde_batch* b);

/* Grouped mode: requests with equal shape (n1, n2, precision, multigrid settings, restart; the
 * geometric hierarchy, any precision but FDE_MIXED_BF16GEMM) and max(n1, n2) <= max_n share a
 * group of `slots` equal slots of one device region and one stream.  A group's restart cycle is one
 * captured HIP graph whose every kernel covers all slots (one launch per kernel for the whole
 * group instead of one per request), issued while any member solves; empty slots and members whose
 * solve has stopped are skipped by every kernel, so each member computes exactly what it computes
 * alone.  A group is created when the first request of its shape is admitted and charges
 * slots * (fde_footprint rounded up to 4 KiB) to the budget until the batch is destroyed; its members
 * are charged (2 + nsrc) * n1 * n2 * 8 bytes each.  max_n = 0 turns grouping off (the default).
 * Only on an empty batch; FDE_EINVAL for slots outside 1..1024 (with max_n > 0) or a batch that
 * holds requests. */
int fde_batch_set_grouping(fde_batch* b, int32_t max_n, int32_t slots);

/* Streams.  lanes = 0 (the default): every ungrouped request and every group gets a stream of its own.
 * lanes >= 2: the batch creates that many streams at once (consecutive streams go to different
 * hardware queues of the device); the ungrouped requests are dealt in turn to the first lanes / 2 of
 * them, with at most one piece in flight per lane, and the groups to the others.  The larger
 * (ungrouped) requests then keep to their own hardware queues instead of queueing in front of the
 * small requests' kernels.  Only on an empty batch (no requests or groups); FDE_EINVAL for lanes 1 or
 * above 16. */
int fde_batch_set_lanes(fde_batch* b, int32_t lanes);

/* Scheduling.  piece_steps > 0 issues every restart cycle (Sec. 5: GMRES restarted every 20 steps) in
 * pieces of piece_steps Arnoldi steps and a tail (x update, true residual), with a read of the solver
 * state after each piece: once a cycle has converged its remaining steps are not issued at all, and
 * the scheduler can switch requests between pieces; 0 (the default) issues whole cycles, which keeps
 * the device busiest when cycles run full.  Only on an empty batch when piece_steps changes.
 * max_running > 0: at most that many ungrouped requests have a piece in flight at once; the others
 * wait at a piece boundary, and each free place goes to the waiting request with the least work left
 * (n1 * n2 * remaining steps), so small requests pass large ones instead of sharing the device with
 * them (preemption at piece boundaries), at the price of some concurrency; 0 (the default) issues
 * every due piece at once.  busy_running >= 0: while any group (grouping, above) has a member with a
 * step to do, at most busy_running ungrouped requests have a piece in flight (0: none — the small
 * grouped requests then have the device to themselves for their short solves); -1: no extra limit.
 * Results do not depend on any setting.  FDE_EINVAL for values out of range or a piece change on a
 * batch that holds requests. */
int fde_batch_set_policy(fde_batch* b, int32_t max_running, int32_t piece_steps, int32_t busy_running);

/* Admits a request: problem *p (as for fde_setup), coefficient fields (copied), initial field u0
 * (device, copied), nsteps CN steps from t0, and a separable source sum_k phi_k(t) S_k with
 * phi_k(t) = coef[k] * exp(rate[k] * t) evaluated at the half steps (nsrc <= 4; coef, rate host
 * arrays; S host array of device fields, copied).  Blocks until the request is resident.  Returns
 * a request id >= 0, FDE_EAGAIN if it does not fit the budget, or an error code. */
int fde_batch_admit(fde_batch* b, const fde_problem* p, const double* dp, const double* dm,
                    const double* ep, const double* em, const double* u0, int32_t nsteps,
                    double t0, int32_t nsrc, const double* coef, const double* rate,
                    const double* const* S);

/* Makes progress on every active request (starting steps, issuing restart cycles) and returns once
 * at least one CN step has completed somewhere, or when no request is active.  Returns the number
 * of requests still stepping (>= 0) or an error.  Requests may be admitted between calls. */
int fde_batch_step(fde_batch* b);

/* Status of request id: 1 finished, 2 finished but some steps stopped at the iteration limit (their
 * last iterates were kept), 0 still stepping, < 0 an error (unknown id: FDE_EINVAL; a failed
 * request returns its error code once and is released).  With u_out (device, n1*n2 FP64) a finished
 * request's final field is copied out and the request is released.  iters_out (host, may be NULL)
 * receives the GMRES iterations so far. */
int fde_batch_poll(fde_batch* b, int id, double* u_out, int64_t* iters_out);

/* Cancels a request (waiting for its in-flight work) and releases its memory. */
int fde_batch_cancel(fde_batch* b, int id);

/* Number of requests still stepping and the budgeted bytes in use. */
int fde_batch_info(const fde_batch* b, int32_t* active, size_t* bytes_in_use);

/* ---- an entry point that allocates nothing ----------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  y = (I - tau/2 L) x, the FP64 system operator of
 * fde_apply (level 0, FDE_FP64) for the problem *p (alpha, beta, n1, n2, domain and tau are read;
 * the solver settings are ignored), without a handle.  dp, dm, ep, em, x, y: device FP64 fields
 * [n2][n1] owned by the caller (coefficients are not scanned for sign or finiteness); y may not alias
 * x.  All work is issued on `stream` (NULL: the default stream) and the call returns without
 * waiting.  The weights, symbols, twiddles, coefficient pairs and the intermediate field are kept in
 * a fixed library-owned device array of about 42 MB (5 * 1023^2 doubles plus tables), one per GPU
 * the library runs on, held until the process ends: n1 and n2 are limited to FDE_NOALLOC_MAX_N
 * (FDE_EINVAL beyond).  The call performs no device allocation and no host-device copy.  Every call
 * on one GPU uses the same array, so calls that overlap on one GPU (different streams or host
 * threads) race; order them on one stream.  Returns 0 or FDE_EINVAL / FDE_EDEVICE (message in
 * fde_last_error(NULL)). */
#define FDE_NOALLOC_MAX_N 1023
int fde_apply_noalloc(const fde_problem* p, const double* dp, const double* dm, const double* ep,
                      const double* em, const double* x, double* y, void* stream);


#ifdef __cplusplus
}
#endif
#endif /* FDE_H */
