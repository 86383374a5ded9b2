/*
 * sylv.h -- C ABI of the MI355X (gfx950) solver for the posterior mean of the CMB
 * source-separation model: matrix-free preconditioned conjugate gradients on
 *
 *     G(X) = sum_j Q_j X E_jj + sum_f D_f X a_f a_f^T  =  B_rhs,
 *     Q_j  = tau_j (kappa_j^2 I - Lap)^T (kappa_j^2 I - Lap),   D_f = diag(W[f, :]),
 *     B_rhs[j, p] = sum_f W[f, p] Y[f, p] A[f, j],
 *
 * i.e. the system (Q + B^T C B) mu = B^T C Y of Section 3, eq. (Axb), with the paper's prior
 * phi_l D^2 generalised to the SPDE prior (kappa_j^2 - Lap)^2 (kappa_j = 0, tau_j = phi_l is the
 * paper's case; Section 3 and App. C), its separable noise precision T (x) N generalised to
 * per-map, per-pixel weights W[f, p], and Lap the 5-point Laplacian of a periodic grid (the
 * paper's D on a grid whose pixels each have four edge neighbours).  The solver is Alg. 2
 * (conjugate gradients) with a block-Jacobi preconditioner, run in float64 or with float32
 * operator applies inside float64 iterative refinement.
 *
 * Conventions shared by every entry point:
 *  - Every array argument is a DEVICE pointer (hipMalloc / torch CUDA memory) on the current
 *    device, including the small parameter arrays kappa, tau and A.  Structs are host memory.
 *  - Maps are component-major: X[j * n_pix + p], with pixel p = iy * nx + ix (row-major grid).
 *    W and Y are stacked by map: W[f * n_pix + p] (Section 2.1).  A is row-major f x k:
 *    A[f * k + j], row f is a_f.
 *  - The caller owns all memory.  The library allocates nothing on the device: scratch space
 *    comes from the caller's workspace `ws` of `ws_bytes` bytes (256-byte aligned), sized by
 *    sylv_workspace_bytes().  The workspace must not be shared by calls that overlap in time.
 *    (sylv_pcg_solve_noalloc uses a static per-device array of the library instead.)
 *  - Host-side state: solves with the adaptive schedule (and the Lanczos-Sylvester solver) read
 *    their convergence reports from one small pinned host block with four events per calling
 *    host thread, allocated on the thread's first such call (hipHostMalloc, hipEventCreate) and
 *    kept until the thread ends.  sylv_lanczos_solve and sylv_kohler_solve copy tau, A and t to
 *    the host (the k x k decompositions run there) and sylv_lanczos_stats is a host struct; every
 *    other result is written to device memory.  The enqueue-only calls and fixed-schedule solves
 *    touch no host state but the thread-local last-error string.
 *  - `stream` is a hipStream_t (NULL = the null stream).  sylv_apply, sylv_precond,
 *    sylv_prepare, sylv_rhs and sylv_po_perturb only enqueue work, with no host
 *    synchronisation, so they may be captured into a HIP graph.  sylv_pcg_solve and
 *    sylv_pcg_backward with the adaptive schedule (the default) enqueue work and synchronise
 *    `stream` a few times to test convergence, returning when the solve has finished; with
 *    schedule = SYLV_SCHED_FIXED they only enqueue work and may be captured as well.
 *    sylv_lanczos_solve synchronises at every convergence check (its small projected problems
 *    are solved on the host) and refuses a capturing stream; sylv_autotune times whole solves
 *    and synchronises as well.
 *  - Return value: 0 on success, a negative SYLV_E_* code when the arguments are rejected before
 *    any work is enqueued (then sylv_last_error() describes why), or SYLV_E_HIP when a HIP call
 *    failed.  Numerical outcomes of a solve (converged, not converged, breakdown, non-finite
 *    values) are reported per solve in sylv_pcg_stats.status, not as the return value.
 *  - Limits: 1 <= k <= 8, 1 <= f <= 16, ny, nx >= 1, ny * nx < 2^29.
 *  - Lap is the graph Laplacian of the pixel grid (Section 3's D): periodic, or one HEALPix base
 *    face whose border pixels have fewer neighbours (sylv_problem.boundary).
 */
#ifndef SYLV_H
#define SYLV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return and status codes ------------------------------------------------------------- */
#define SYLV_OK              0  /* converged (stats) / success (return value)                  */
#define SYLV_NOT_CONVERGED   1  /* max_iter (or refine_max) reached; X holds the last iterate   */
#define SYLV_BREAKDOWN       2  /* <p, G p> <= 0 or <r, z> <= 0: operator or preconditioner not
                                   positive definite (e.g. negative tau, or kappa = 0 with no
                                   data weight at all)                                          */
#define SYLV_NONFINITE       3  /* a NaN or Inf appeared in a residual or inner product         */
#define SYLV_STAGNATED       4  /* mixed precision: an outer refinement step did not reduce the
                                   float64 residual                                             */
#define SYLV_BAD_INPUT       5  /* Lanczos-Sylvester: some n_p is not a positive finite number  */
#define SYLV_E_INVALID     (-1) /* bad argument (null pointer, size out of range, bad option)   */
#define SYLV_E_WORKSPACE   (-2) /* ws_bytes smaller than sylv_workspace_bytes()                  */
#define SYLV_E_HIP         (-3) /* a HIP runtime call failed                                     */

/* ---- element types, precisions, preconditioners ------------------------------------------ */
#define SYLV_F64 0
#define SYLV_F32 1

#define SYLV_PREC_F64   0       /* every vector and every apply in float64                       */
#define SYLV_PREC_MIXED 1       /* float32 vectors and applies inside float64 refinement         */

#define SYLV_BC_PERIODIC 0      /* periodic grid: every pixel has 4 neighbours (torus)            */
#define SYLV_BC_FACE     1      /* one HEALPix base face: 4-neighbour links only inside the grid,
                                   so border pixels have 2 or 3 (App. A; D of Section 3 with minus
                                   the row sum on the diagonal)                                  */

#define SYLV_STOP_R0 0          /* stopping test relative to the initial residual (Alg. 2)        */
#define SYLV_STOP_B  1          /* stopping test relative to ||b||                                 */

#define SYLV_SCHED_ADAPTIVE 0   /* host checks convergence between batches of queued iterations  */
#define SYLV_SCHED_FIXED    1   /* every iteration up to the caps is queued at once, no host
                                   synchronisation (graph capture)                               */

#define SYLV_PC_NONE   0        /* z = r (plain Alg. 2)                                           */
#define SYLV_PC_JACOBI 1        /* z = r / diag(G)                                                */
#define SYLV_PC_BLOCK  2        /* z_p = (G_pp)^-1 r_p, G_pp the k x k block of pixel p           */
#define SYLV_PC_FOURIER 3       /* z = (Q + I (x) Mbar)^-1 r through 2-D transforms that
                                   diagonalise the prior (the DFT on periodic grids, the cosine
                                   transform DCT-II on face grids): the operator with the
                                   weights replaced by their pixel means (Mbar = sum_f
                                   mean_p(W[f, p]) a_f a_f^T), exact for pixel-independent
                                   weights.  Grid sides powers of two in [4, 4096], k * ny complex
                                   values within the column pass's LDS (float32: k * ny <= 8192,
                                   float64: k * ny <= 8192 with the stage twiddles read from
                                   global memory beyond 4096 minus padding); independent CG only
                                   (else SYLV_E_INVALID)                                         */
#define SYLV_PC_FOURIER_DIAG 4  /* z = S^-1 (Q + I (x) Mbar)^-1 S^-1 r, S = diag(s) per pixel and
                                   component with s^2 = diag(G) / diag(Q + I (x) Mbar): the
                                   SYLV_PC_FOURIER operator scaled so that its diagonal is G's
                                   (the heteroscedastic weights enter through the scale; s = 1
                                   for pixel-independent weights).  Same grids and limits as
                                   SYLV_PC_FOURIER                                               */
#define SYLV_PC_FOURIER_BLOCK 5 /* z = T^T (Q + I (x) Mbar)^-1 T r, T block diagonal over the
                                   pixels with T_p = L0_p Lp^-1 (Lp, L0_p the Cholesky factors of
                                   the k x k pixel blocks of G and of Q + I (x) Mbar): the
                                   operator it inverts has G's pixel blocks.  Same grids as
                                   SYLV_PC_FOURIER, and the row passes hold every component of
                                   two grid rows: k * nx <= 8192 (else SYLV_E_INVALID)          */

/* One posterior-mean system (Section 2, Section 3).  Host struct of device pointers. */
typedef struct sylv_problem {
    int64_t ny, nx;        /* grid, n_pix = ny * nx < 2^29 (else SYLV_E_INVALID)                 */
    int32_t k;             /* components (the paper's m: sources)                                */
    int32_t f;             /* maps (the paper's n: frequencies)                                  */
    const double *kappa;   /* [k]  kappa_j >= 0   (prior range parameter)                        */
    const double *tau;     /* [k]  tau_j > 0      (prior precision scale; the paper's phi_l)     */
    const double *A;       /* [f * k] mixing matrix, row-major                                   */
    const double *W;       /* [f * n_pix] noise precision per map and pixel, >= 0 (0 = masked)   */
    int32_t boundary;      /* SYLV_BC_PERIODIC or SYLV_BC_FACE (all problems of one call alike)  */
    int32_t reserved;      /* 0                                                                   */
} sylv_problem;

typedef struct sylv_pcg_opts {
    double  tol;           /* stop when ||b - G x||_2 <= tol * ||b - G x0||_2 (Alg. 2 test; see
                              stop_ref)                                                           */
    int32_t max_iter;      /* iteration cap of each (inner) conjugate-gradient run               */
    int32_t precision;     /* SYLV_PREC_F64 or SYLV_PREC_MIXED                                   */
    double  inner_tol;     /* mixed: smallest relative reduction asked of one float32 inner run
                              (0 = 1e-5)                                                          */
    int32_t refine_max;    /* mixed: maximum number of float64 refinement steps (0 = 8)          */
    int32_t precond;       /* SYLV_PC_NONE, _JACOBI, _BLOCK, _FOURIER, _FOURIER_DIAG, _FOURIER_BLOCK */
    int32_t check_every;   /* iterations enqueued between host convergence checks (0 = 8, 4 with
                              the Fourier preconditioners)                                        */
    int32_t block;         /* 1: block CG over blocks of s right-hand sides of each problem
                              (s = block_size): s x s Gram matrices in float64, alpha and beta
                              from s x s Cholesky solves, converged columns deflated;
                              0: independent CG per right-hand side                              */
    int32_t stop_ref;      /* reference of the stopping test: SYLV_STOP_R0 (||b - G x0||, Alg. 2's
                              test) or SYLV_STOP_B (||b||, for warm starts over a sweep of
                              hyperparameters); the same when x0 = 0                            */
    int32_t schedule;      /* SYLV_SCHED_ADAPTIVE: batches of check_every iterations are queued
                              ahead of a host convergence check, and a float64 run whose
                              recomputed residual misses the threshold is restarted from its x
                              (at most 3 times).  SYLV_SCHED_FIXED: max_iter + 1 iterations per
                              (inner) run and refine_max refinement steps are queued at once with
                              no host synchronisation and no restart, so the call may be captured
                              into a HIP graph; launches after a run has converged return at once
                              (about 1-2 us each), so max_iter and refine_max should be set near
                              what the solve needs; (max_iter + 1) times the refinement steps
                              (mixed; 1 for float64) may not exceed 65536 (else SYLV_E_INVALID).
                              Both schedules compute the same iterates: the device takes every
                              stopping decision.                                                 */
    int32_t block_size;    /* block = 1: columns per block, 2, 4 or 8, dividing nrhs (0 = nrhs,
                              which must then be 2, 4 or 8); the nrhs / s blocks of a problem
                              iterate independently of each other                               */
    int32_t apply_rows;    /* output rows per lane of the independent-CG operator applies: 2, 4
                              or 8, lowered where a precision and k would overflow registers
                              (0 = default: 4 at k <= 3 in float64 and k <= 4 in float32, else
                              2; face grids always 2).  Changes the tiling, so reductions round
                              differently, never the arithmetic per pixel                       */
} sylv_pcg_opts;

/* Per-solve result, written by the device into caller memory (DEVICE pointer). */
typedef struct sylv_pcg_stats {
    int32_t status;        /* SYLV_OK, SYLV_NOT_CONVERGED, SYLV_BREAKDOWN, SYLV_NONFINITE, ... */
    int32_t iters;         /* total conjugate-gradient iterations (all inner runs)              */
    int32_t outer;         /* refinement steps (mixed) or 1 (float64)                           */
    int32_t reserved;
    double  relres_rec;    /* last recursive residual norm / initial residual norm              */
    double  relres_true;   /* ||b - G x||_2 / ||b||_2 recomputed in float64 at the end          */
} sylv_pcg_stats;

/* Bytes of workspace needed.  probs[nprob] are the problems of a batch, each solved for nrhs
 * right-hand sides.  opts == NULL: enough for sylv_prepare / sylv_apply / sylv_precond with
 * nprob = 1 and up to nrhs right-hand sides.  Returns 0 for invalid arguments. */
size_t sylv_workspace_bytes(const sylv_problem *probs, int32_t nprob, int32_t nrhs,
                            const sylv_pcg_opts *opts);

/* Operator set-up for one problem: stencil coefficients of every Q_j (13-point expansion of
 * tau_j (kappa_j^2 - Lap)^2, Section 3.1), the per-pixel mixing blocks
 * M_p = sum_f W[f,p] a_f a_f^T (the block map of Section 3.1 in per-pixel form) and the
 * preconditioner blocks, in float64 and float32.  Written into ws; later calls with
 * prepared = 1 reuse them. */
int sylv_prepare(const sylv_problem *prob, int32_t precond, void *ws, size_t ws_bytes,
                 void *stream);

/* Y = G(X) for nrhs maps (Section 3.1: the matrix-free product x -> (Q + B^T C B) x).
 * X, Y: [nrhs][k][n_pix] of dtype SYLV_F64 or SYLV_F32 (not overlapping).  prepared = 0 runs
 * sylv_prepare first. */
int sylv_apply(const sylv_problem *prob, int32_t dtype, const void *X, void *Y, int32_t nrhs,
               int32_t prepared, void *ws, size_t ws_bytes, void *stream);

/* Z = Minv R with the chosen preconditioner (Section 3.2 remarks on preconditioning).
 * R, Z: [nrhs][k][n_pix] of dtype.  precond must match the sylv_prepare call when prepared. */
int sylv_precond(const sylv_problem *prob, int32_t dtype, int32_t precond, const void *R,
                 void *Z, int32_t nrhs, int32_t prepared, void *ws, size_t ws_bytes,
                 void *stream);

/* Right-hand side B_rhs = B^T C Y (eq. (mu*)): Bout[j*n_pix+p] = sum_f W[f,p] Y[f,p] A[f,j].
 * Y: [f][n_pix] float64, Bout: [k][n_pix] float64. */
int sylv_rhs(const sylv_problem *prob, const double *Y, double *Bout, void *stream);

/* Perturbation for posterior sampling (perturbation optimisation):
 * eta_j = sqrt(tau_j) L_j^T xi_j + sum_f A[f,j] sqrt(W[f,:]) zeta_f, L_j = kappa_j^2 - Lap,
 * so that Cov(eta) = G and G^-1 (B_rhs + eta) is a draw from the posterior of Section 2.2.
 * xi: [nrhs][k][n_pix], zeta: [nrhs][f][n_pix], eta: [nrhs][k][n_pix], all float64. */
int sylv_po_perturb(const sylv_problem *prob, const double *xi, const double *zeta, double *eta,
                    int32_t nrhs, void *stream);

/* Solve G x = b for nprob problems times nrhs right-hand sides each, by preconditioned CG
 * (Alg. 2 plus preconditioner), in float64 or mixed precision.
 *   b = B^T C Y (if Y != NULL) + Bextra (if Bextra != NULL); at least one must be given.
 *   Y:      concatenation over problems of [f_g][n_pix_g] float64 (shared by the g's rhs)
 *   Bextra: concatenation over problems of [nrhs][k][n_pix_g] float64
 *   X:      concatenation over problems of [nrhs][k][n_pix_g] float64: initial guess on entry
 *           (zeros for the paper's x0 = 0), solution on return
 *   stats:  [nprob * nrhs] device structs, problem-major.
 * All problems of one call must share k. */
int sylv_pcg_solve(const sylv_problem *probs, int32_t nprob, int32_t nrhs, const double *Y,
                   const double *Bextra, double *X, const sylv_pcg_opts *opts,
                   sylv_pcg_stats *stats, void *ws, size_t ws_bytes, void *stream);

/* Solve without allocation, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): sylv_pcg_solve with the
 * same arguments and results, except that the workspace is a static array of
 * SYLV_NOALLOC_SCRATCH_BYTES bytes that the library holds on each device it runs on (from the
 * first call on that device until the process ends; the first call on a device looks up its
 * address with hipGetSymbolAddress).  The call allocates nothing and enqueues only kernels.
 *  - opts->schedule must be SYLV_SCHED_FIXED (else SYLV_E_INVALID): the adaptive schedule
 *    needs pinned host memory for its convergence checks.
 *  - A batch whose workspace (sylv_workspace_bytes(probs, nprob, nrhs, opts)) exceeds
 *    SYLV_NOALLOC_SCRATCH_BYTES is rejected with SYLV_E_WORKSPACE before any work is enqueued.
 *  - Every call on one device shares that device's array: calls that overlap in time on one
 *    device (different streams or threads without ordering between them) race and give wrong
 *    results.  Calls ordered on one stream are safe; nothing in the array has to be cleared
 *    between them (each call initialises every region it reads). */
#define SYLV_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int sylv_pcg_solve_noalloc(const sylv_problem *probs, int32_t nprob, int32_t nrhs,
                           const double *Y, const double *Bextra, double *X,
                           const sylv_pcg_opts *opts, sylv_pcg_stats *stats, void *stream);

/* Adjoint of the solve.  Given x* = G^-1 B_rhs (Xstar, [k][n_pix]) and Gbar = dL/dx*, solves
 * G lambda = Gbar (G is symmetric, so this is a second PCG run; Lambda is the initial guess on
 * entry and lambda on return) and forms the gradient of <Gbar, x*> with respect to the
 * parameters, writing (device pointers, each may be NULL to skip):
 *   dkappa[k]  = -4 kappa_j tau_j <lambda_j, L_j x*_j>
 *   dtau[k]    = -<L_j lambda_j, L_j x*_j>
 *   dA[f*k]    = sum_p W[f,p] (r_f(p) lambda_p - (a_f . lambda_p) x*_p),  r_f = Y_f - a_f . x*
 *   dW[f*n_pix]= (a_f . lambda_p) r_f(p)
 *   dY[f*n_pix]= W[f,p] (a_f . lambda_p)
 * Y: [f][n_pix] float64 (the observed maps used for x*). */
int sylv_pcg_backward(const sylv_problem *prob, const double *Y, const double *Xstar,
                      const double *Gbar, double *Lambda, double *dkappa, double *dtau,
                      double *dA, double *dW, double *dY, const sylv_pcg_opts *opts,
                      sylv_pcg_stats *stats, void *ws, size_t ws_bytes, void *stream);

/* ---- Lanczos-Sylvester solver (Section 3.3, Alg. 4 and Alg. 5) ---------------------------------
 *
 * The case the paper solves in Sylvester form: every component shares one kappa and the noise
 * precision is separable, W[f, p] = t_f n_p (C = T (x) N with T = diag(t), N = diag(n)).  With
 * P = diag(tau) and D2 = (kappa^2 I - Lap)^2 the system G(X) = B_rhs is then the Sylvester
 * equation (eq. (Axb-Sylv))
 *
 *     N^-1 D2 M + M Lhat = Yhat,   Lhat = A^T T A P^-1,   Yhat = Y^T T A P^-1,
 *
 * M the n_pix x k matrix whose column j is map j (X[j * n_pix + p] = M[p, j]).  The solver runs
 * the symmetric block Lanczos process for N^-1 D2 in the N inner product (Alg. 4) from Yhat,
 * projects the equation on the block Krylov space (eq. (Sylv-small)) and stops on Alg. 5's
 * residual estimate sqrt(gamma) <= tol ||B_0||_F; the Galerkin approximation is then assembled
 * either from the Lanczos blocks kept in the workspace (SYLV_LZ_KEEP_BASIS) or by the paper's
 * second Lanczos pass, which regenerates the blocks from the kept coefficients (SYLV_LZ_RERUN,
 * for grids and step counts whose basis would not fit).  All arithmetic is float64.
 */

/* Host struct of device pointers. */
typedef struct sylv_sep_problem {
    int64_t ny, nx;        /* grid, n_pix = ny * nx < 2^29 (else SYLV_E_INVALID)                 */
    int32_t k;             /* components (the paper's m), 1..8                                   */
    int32_t f;             /* maps (the paper's n), 1..16                                        */
    double  kappa;         /* common kappa >= 0 (host value; 0 = the paper's D^2 prior)          */
    const double *tau;     /* [k]  tau_j > 0 (the paper's phi: P = diag(tau))                    */
    const double *A;       /* [f * k] mixing matrix, row-major, full column rank                 */
    const double *t;       /* [f]  t_f > 0 (per-map noise precision, T)                          */
    const double *n;       /* [n_pix] n_p > 0 (per-pixel noise precision, N; no masked pixels)   */
    int32_t boundary;      /* SYLV_BC_PERIODIC or SYLV_BC_FACE                                   */
    int32_t reserved;      /* 0                                                                   */
} sylv_sep_problem;

#define SYLV_LZ_KEEP_BASIS 0  /* keep every Lanczos block; M = sum_i V_i G_i is one streaming
                                 pass over them (workspace ~ max_iter * k * n_pix doubles)      */
#define SYLV_LZ_RERUN      1  /* keep only the last two blocks; M is assembled by running the
                                 Lanczos recurrence a second time from the kept small blocks
                                 H_i, B_i (Alg. 5's second pass; workspace ~ 5 k n_pix doubles,
                                 about twice the time)                                           */

typedef struct sylv_lanczos_opts {
    double  tol;           /* stop when sqrt(gamma) <= tol * ||B_0||_F (Alg. 5)                  */
    int32_t max_iter;      /* Lanczos steps at most                                              */
    int32_t check_every;   /* steps enqueued between host convergence checks (0 = 8)             */
    int32_t assembly;      /* SYLV_LZ_KEEP_BASIS or SYLV_LZ_RERUN                                */
    int32_t reserved;      /* 0                                                                   */
} sylv_lanczos_opts;

/* Result of a Lanczos-Sylvester solve (HOST struct, filled before the call returns). */
typedef struct sylv_lanczos_stats {
    int32_t status;        /* SYLV_OK, SYLV_NOT_CONVERGED, SYLV_BREAKDOWN (N-Gram matrix of a new
                              block not positive definite), SYLV_NONFINITE, SYLV_BAD_INPUT       */
    int32_t iters;         /* Lanczos steps whose blocks make up the solution                     */
    double  relres_est;    /* sqrt(gamma) / ||B_0||_F after the last step (Alg. 5)                */
    double  relres_true;   /* ||b - G x||_2 / ||b||_2 of eq. (Axb), recomputed in float64         */
} sylv_lanczos_stats;

/* Bytes of workspace for sylv_lanczos_solve (0 for invalid arguments). */
size_t sylv_lanczos_workspace_bytes(const sylv_sep_problem *prob, const sylv_lanczos_opts *opts);

/* Solve eq. (Axb-Sylv) by Alg. 5 with Alg. 4 inside.
 *   Y: [f][n_pix] float64 observed maps;  X: [k][n_pix] float64, the solution on return.
 * The call copies tau, A and t to the host (the k x k eigenproblem of Lemma 2 is solved there),
 * synchronises `stream` every check_every steps and at the end, and returns when X and *stats
 * are final.  Rejected (SYLV_E_INVALID) when A^T T A is not positive definite. */
int sylv_lanczos_solve(const sylv_sep_problem *prob, const double *Y, double *X,
                       const sylv_lanczos_opts *opts, sylv_lanczos_stats *stats, void *ws,
                       size_t ws_bytes, void *stream);

/* ---- sparse-dense Sylvester solver (Section 3.3.1, Alg. 3) ------------------------------------
 *
 * The same separable, equal-kappa system as sylv_lanczos_solve, N^-1 D2 M + M Lhat = F
 * (eq. (Axb-Sylv), F = Y^T T A P^-1), solved by the method the paper compares against
 * (Alg. 3, the sparse-dense form eq. (sparse-dense-Sylvester) with H = N^-1 D2, L = Lhat): with
 * Lhat = W R W^-1 and R upper triangular, column i of Xhat = M W solves the shifted sparse
 * system (H + R_ii I) xhat_i = F W e_i - sum_(l<i) xhat_l R_li, here multiplied through by N,
 *
 *     (D2 + R_ii N) xhat_i = N (F W e_i - sum_(l<i) xhat_l R_li),
 *
 * whose matrix is symmetric positive definite (R_ii are the eigenvalues of Lhat, positive by
 * Lemma 2), and M = Xhat W^-1.  Each column system is solved on the GPU by the preconditioned
 * conjugate-gradient solver of sylv_pcg_solve, as a one-component problem (kappa, tau = 1,
 * A = sqrt(R_ii), W = n), with the options `opts` (float64 or mixed precision, tolerance
 * relative to each column's right-hand side).
 *   decouple = 0: W is orthogonal and R triangular, a real Schur form of Lhat (Alg. 3); the
 *                 columns are solved one after another, each right-hand side using the
 *                 previous columns.  (The Schur vectors are obtained from Lemma 2's
 *                 eigenvectors U by a QR factorisation U = W Ru, R = Ru diag(rho) Ru^-1.)
 *   decouple = 1: W = U, Lemma 2's eigenvectors, and R = diag(rho): the k column systems are
 *                 independent and run as one batched solve.
 * n_p may be 0 (masked pixels) as long as D2 + R_ii N stays positive definite (kappa > 0).
 *   Y: [f][n_pix] float64;  X: [k][n_pix] float64, the solution M on return (column j = map j).
 *   stats: [k] DEVICE structs, the conjugate-gradient runs of the column systems (in the order
 *          of the transformed columns).
 *   relres_true: DEVICE double or NULL: ||b - G x||_2 / ||b||_2 of eq. (Axb) for the result.
 * Copies tau, A and t to the host (the k x k decompositions are computed there), synchronises
 * `stream`, and refuses a capturing stream. */
size_t sylv_kohler_workspace_bytes(const sylv_sep_problem *prob, int32_t decouple,
                                   const sylv_pcg_opts *opts);
int sylv_kohler_solve(const sylv_sep_problem *prob, const double *Y, double *X,
                      int32_t decouple, const sylv_pcg_opts *opts, sylv_pcg_stats *stats,
                      double *relres_true, void *ws, size_t ws_bytes, void *stream);

/* ---- autotuning of the solver configuration --------------------------------------------- */

/* Result of sylv_autotune: the configuration to copy into sylv_pcg_opts. */
typedef struct sylv_tune_result {
    int32_t block;         /* 0: independent CG, 1: block CG                                    */
    int32_t block_size;    /* columns per block (block = 1), else 0                             */
    int32_t apply_rows;    /* rows per lane of the operator applies (independent CG), else 0    */
    int32_t candidates;    /* configurations timed                                              */
    double  ms;            /* time to tolerance of the chosen configuration                     */
    double  ms_given;      /* time to tolerance with the configuration of `opts` as given        */
} sylv_tune_result;

/* Time whole solves of this batch (same arguments as sylv_pcg_solve) under every candidate
 * configuration and report the fastest that converges for every right-hand side: independent CG
 * with 2, 4 and 8 output rows per lane of the applies, and block CG with every block size in
 * {2, 4, 8} that divides nrhs.  Each candidate is solved twice from x0 = 0 and timed with HIP
 * events around the whole call (set-up included); the shorter run counts.  X and stats are
 * scratch: X is zeroed before every solve and holds the last candidate's solution on return.
 * ws must hold sylv_workspace_bytes(probs, nprob, nrhs, opts) bytes (the same for every
 * candidate).  Synchronises `stream`; not capturable.  Intended to run once per batch shape,
 * with the result kept by the caller. */
int sylv_autotune(const sylv_problem *probs, int32_t nprob, int32_t nrhs, const double *Y,
                  const double *Bextra, double *X, const sylv_pcg_opts *opts,
                  sylv_pcg_stats *stats, sylv_tune_result *out, void *ws, size_t ws_bytes,
                  void *stream);

/* Human-readable name of a status or return code (static string). */
const char *sylv_status_string(int code);

/* Description of the last argument error of the calling thread (static per-thread buffer). */
const char *sylv_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SYLV_H */
