// Internal declarations shared by the HIP kernels (sylv_kernels.hip) and the host driver
// (sylv_api.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sylv {

constexpr int kMaxK = 8;
constexpr int kMaxF = 16;
constexpr int kCoefStride = 8;   // per component: c0, c1, cd, c2, diag, kappa, tau, unused
constexpr int kBlock = 256;      // threads per workgroup (4 wavefronts of 64)
constexpr int kTileX = 64;       // apply tile width = one wavefront across x
constexpr int kWavesY = 4;       // wavefronts stacked in y inside an apply tile
constexpr int kChunk = 1024;     // pixels per workgroup in streaming kernels (4 per thread)

// Reduction quantities in an instance's `partial` array (kNumSlots planes of `nred` doubles,
// one value per producing workgroup).  A kernel that needs a reduced value re-reduces the
// producer's partials itself, in a fixed order, at its start: kernel boundaries make them
// visible without any device-wide fence, and every workgroup obtains bitwise the same scalar.
// SLOT_FRZ: <r, z> of the Fourier preconditioner, one partial per column workgroup of its
// column pass (the update and start kernels then leave SLOT_RZ at zero).
enum Slot { SLOT_PQ = 0, SLOT_RZ = 1, SLOT_RR = 2, SLOT_RES_RR = 3, SLOT_RES_BB = 4, SLOT_FRZ = 5 };
constexpr int kNumSlots = 6;
constexpr int kMaxRestarts = 3;   // residual replacements of a float64 run
constexpr int kUploadWords = 512; // 32-bit words per table-upload launch (2 KiB of arguments)
constexpr int kMaxFixedIters = 65536;   // iterations one fixed-schedule call may queue
// Every workgroup of a consuming CG kernel re-reduces the producer's per-workgroup partials in a
// fixed order (no atomics, bitwise repeatable).  That read grows with the square of the
// workgroup count, so instances with more partials than this fold them first in a separate
// one-workgroup-per-instance kernel.  Measured: folding 1024 partials (1024^2 at 4 rows per lane)
// costs more in launches than it saves; 2048 (a 1024^2 face at 2 rows) and up gain.
constexpr int kPreReduce = 1024;
// Largest rows per lane of the apply kernels that keeps their register window without spills.
constexpr int apply_rows_cap(bool f64, int k) {
    return f64 ? (k <= 2 ? 8 : k <= 3 ? 4 : 2) : (k <= 2 ? 8 : k <= 5 ? 4 : 2);
}
// Mixed precision: a float32 inner run asks for safety * sqrt(threshold / ||r||^2) of its
// starting residual, so that the refinement step lands below the outer threshold with margin.
// The float64 residual after the step tracks the float32 recursive one to a few per cent at these
// levels (it lands at about safety * tol), so 0.7 keeps a 30 % margin; smaller factors only
// overshoot the tolerance at the price of extra iterations (0.3: 4 more at 1024^2, 7 at 2048^2).
constexpr double kInnerSafety = 0.7;

// Solver state of one conjugate-gradient run, in device memory.  The scalars of the recurrence
// (Alg. 2: alpha, beta, <r, z>, ||r||) are formed on the device; the host only reads `done`.
// Fields written during the loop are written by one workgroup of a kernel and read by later
// kernels only (rho is double-buffered by iteration parity for that reason).
struct DevState {
    double rho[2];   // <r, z> of iterations with even / odd index
    double alpha[2]; // step lengths of iterations with even / odd index (x is advanced by the
                     // next iteration's apply, which already reads that direction)
    double rr;       // ||r||^2 at the last test
    double rr0;      // ||r_0||^2
    double bb;       // ||b||^2
    double thresh;   // stop when rr <= thresh
    double tol;      // relative tolerance of this run
    double rel_true; // ||b - G x|| / ||b|| from the last float64 residual pass
    double rr_prev;  // previous refinement residual (stagnation test of the mixed path)
    int32_t iter;    // iterations done by this run
    int32_t max_iter;
    int32_t status;  // SYLV_OK / SYLV_NOT_CONVERGED / SYLV_BREAKDOWN / SYLV_NONFINITE / ...
    int32_t done;    // 1 once the run stopped; every kernel of the loop returns early then
    int32_t total_iter;  // accumulated over inner runs (mixed precision)
    int32_t outer;   // refinement steps
    int32_t pend;    // stopping decision of the last apply (-1: continue); the apply's own
                     // workgroups must all finish it (x update), so `done` is only set by the
                     // following update kernel
    int32_t ref;     // stopping reference: SYLV_STOP_R0 or SYLV_STOP_B
};

// One solve instance = one (problem, right-hand side) pair.  Pointers are into the caller's
// buffers or into the workspace.
struct Inst {
    int32_t ny, nx, n_pix;
    int32_t tiles_x;     // apply tiles across x
    int32_t ntiles;      // float64 apply tiles in this instance
    int32_t ntiles32;    // float32 apply tiles (rows per lane may differ by precision)
    int32_t nchunks;     // streaming chunks in this instance
    int32_t nred;        // stride between reduction quantities in `partial`
    int32_t pc;          // preconditioner kind (SYLV_PC_*)
    int32_t vec4;        // 1 if n_pix % 4 == 0 and every plane is 16-byte aligned
    int32_t f;           // maps of the problem
    int32_t pre;         // 1: the CG reductions are folded by k_prereduce before their
                         // consumers, which then read one value (large grids, see kPreReduce)
    const double *coef;  // [K * kCoefStride]
    const double *A;     // [f * K]
    const double *W;     // [f * n_pix]
    const double *Y;     // [f * n_pix] or null
    const double *bext;  // [K * n_pix] extra right-hand side or null
    const double *M64;   // packed mixing blocks [K(K+1)/2][n_pix]
    const float *M32;
    const double *P64;   // packed preconditioner blocks
    const float *P32;
    const unsigned short *P16;   // bfloat16 factor G = L^-1 of the blocks (CG runs)
    // float64 vectors.  The search direction is double-buffered: the apply of iteration i reads
    // the previous direction from p[i & 1] (including stencil halos owned by other workgroups)
    // and writes the new one to p[(i + 1) & 1], so no workgroup overwrites a value another one
    // may still read.
    double *b, *x, *r, *z, *p[2], *q;
    // float32 vectors of the inner runs of the mixed path; d = inner solution
    float *r32, *z32, *p32[2], *q32, *d32;
    DevState *st;        // float64 run (or outer refinement state)
    DevState *st_in;     // float32 inner run
    double *partial;     // [kNumSlots][nred]
    // Fourier preconditioner (pc == SYLV_PC_FOURIER, periodic grids with power-of-two sides)
    double *fs;          // half spectrum S[k][nx/2 + 1][ny], complex (float64 or float32 pairs)
    const double *fsym;  // Fourier region: Mbar [kMaxK][kMaxK], kappa_j^2 [kMaxK], tau_j
                         // [kMaxK], then eigenvalue and FFT stage tables
    const double *fsc64; // SYLV_PC_FOURIER_DIAG: 1 / s [k][n_pix] (s^2 = diag(G) / diag(Q + I
    const float *fsc32;  // (x) Mbar)); SYLV_PC_FOURIER_BLOCK: T [k(k+1)/2][n_pix] (packed lower
                         // triangle); float64 and float32; null for the plain preconditioner
    int32_t lognx, logny;
    int32_t frb;         // grid rows per workgroup of the row passes
    int32_t nfft;        // column workgroups = nx/2 (partials of <r, z>)
    int32_t nrr;         // partials of ||r||^2 in SLOT_RR: streaming chunks, or in float32 runs
                         // with the Fourier preconditioner its row-pass workgroups k ny / frb
};

// Launch-time view of the instances: a device table plus prefix sums that map a flat
// workgroup id to (instance, tile) for apply kernels or (instance, chunk) for streaming ones.
struct InstSet {
    const Inst *table;    // device array [ninst]
    const int *tprefix;   // device [ninst + 1] prefix sums of float64 apply tiles
    const int *tprefix32; // device [ninst + 1] prefix sums of float32 apply tiles
    const int *cprefix;   // device [ninst + 1] prefix sums of streaming chunks
    int ninst;
    int total_tiles;
    int total_tiles32;
    int total_chunks;
    int rows64, rows32;   // rows per lane of the float64 / float32 apply kernels
    int any_pre;          // some instance has Inst::pre set
    int bc;               // SYLV_BC_* of every instance (face grids use 2 rows per lane)
    int stream;           // 1: the working set exceeds the last-level cache, so the CG kernels
                          // stream their once-touched planes with non-temporal accesses
    // Fourier preconditioner: prefix sums of the row-pass and column-pass workgroups
    const int *fprefa, *fprefb;
    int total_fa, total_fb;
    int fourier;          // pc == SYLV_PC_FOURIER
    size_t fp_lds_rows, fp_lds_cols;  // dynamic LDS of the row and column passes (largest over
                                      // the set's instances)
    int fp_cols_gtw;      // length classes (fp_radix_bit of ny) whose column pass reads its
                          // twiddles from global memory
    int fp_rmask_x, fp_rmask_y;   // final FFT radices present (fp_radix_bit) along x and y
    int fp_scaled;        // SYLV_PC_FOURIER_DIAG: the row passes apply the diagonal scale
    int fp_block;         // SYLV_PC_FOURIER_BLOCK: the block-scaled row passes (all components)
    int fp_blk_gtw;       // ... of the length classes (fp_radix_bit of nx) reading their
                          // twiddles from global memory (float64, wide bands)
};

inline int packed_size(int k) { return k * (k + 1) / 2; }

// ---- block conjugate gradients over the s right-hand sides of one grid ----------------------
constexpr int kMaxS = 8;                           // right-hand sides per group
constexpr int kGramQ = kMaxS * (kMaxS + 1) / 2;    // packed s x s Gram entries
constexpr int kBlockQ = kGramQ + kMaxS;            // + per-column ||r||^2
constexpr int kBlockPix = 256;                     // smallest streaming chunk of the block kernels
// Rows per lane of the block apply, which keeps every column's direction at its output pixels
// in registers for the P^T Q Gram.
constexpr int kBlockRows = 2;
// Pixels per thread of the streaming block kernels (one 8-byte access per plane and lane):
// chunks of kBlock * block_vec pixels.
constexpr int block_vec(bool f64) { return f64 ? 1 : 2; }
enum BlockMode { BM_BLOCK = 0, BM_DIAG = 1 };

// State of one block-CG run of a group (device memory, written only by the Gram kernel).
struct GroupState {
    double rz[kMaxS][kMaxS];     // R^T Z of the current residual block
    double alpha[kMaxS][kMaxS];  // X += P alpha, R -= Q alpha (row: direction, column: rhs)
    double beta[kMaxS][kMaxS];   // P <- Z + P beta
    double rr[kMaxS], rr0[kMaxS], thresh[kMaxS];
    int32_t active[kMaxS];       // 1 while column r iterates (deflated once converged)
    int32_t mode;                // BM_BLOCK, or BM_DIAG (independent CG) after a Gram breakdown
    int32_t restart;             // next direction update restarts (beta = 0)
    int32_t iter, done;
};

struct Group {
    int32_t inst0;               // instance of right-hand side 0 (the group's s instances follow)
    int32_t ntiles, ntiles32;    // apply tiles (float64 / float32 rows per lane)
    int32_t nchunks;             // streaming chunks (kBlock * block_vec pixels)
    int32_t nred;                // partial stride
    int32_t vec;                 // 1: n_pix is a multiple of block_vec (wide plane accesses)
    GroupState *gs;
    double *partial;             // [kBlockQ][nred]
};

struct GroupSet {
    const Inst *table;
    const Group *groups;         // device [ngroup]
    const int *gtprefix;         // device [ngroup + 1] float64 apply tiles
    const int *gtprefix32;       // device [ngroup + 1] float32 apply tiles
    const int *gcprefix;         // device [ngroup + 1] chunks
    int ngroup, s;
    int total_tiles, total_tiles32, total_chunks;
    int bc;
    int stream;                  // as InstSet::stream
};

// ---- launchers (sylv_kernels.hip) -------------------------------------------------------
// Every launcher returns the hipError_t of its launch.
int apply_rows_valid(int rows);
// Rows per lane of the apply kernels for k components and element type dtype; `request` (2, 4
// or 8; 0 = default) is capped where the register window would overflow.
int apply_rows_for(int k, int dtype, int request);
hipError_t launch_coef(const double *kappa, const double *tau, int k, int ny, int nx,
                       double *coef, hipStream_t s);
hipError_t launch_setup(const double *W, const double *A, int f, int ny, int nx, int bc,
                        const double *coef, int pc, double *M64, float *M32, double *P64,
                        float *P32, unsigned short *P16, int exact, int k, hipStream_t s);
hipError_t launch_rhs(const double *W, const double *Y, const double *A, int f, int n_pix,
                      const double *bext, double *b, int k, hipStream_t s);
hipError_t launch_apply_plain(const Inst *table0, int k, int dtype, int rows, int bc, int stream,
                              int ny, int nx, int nrhs, const void *in, void *out, hipStream_t s);
// ---- Fourier preconditioner (sylv_fourier.hip) ------------------------------------------------
// Supported shapes: periodic or face grids with ny and nx powers of two in [4, 4096], k x ny
// within the column pass's LDS (why: the reason otherwise).
bool fp_supported(int ny, int nx, int k, int dtype, char *why, size_t why_len);
int fp_rows_per_block(int nx, int ny, int dtype);
size_t fp_setup_partials(int n_pix, int f);
// Bytes of a problem's Fourier region: the symbol block (Mbar, kappa^2, tau), the Laplacian
// eigenvalues of both grid sides and the FFT stage tables.
size_t fp_table_bytes(int nx, int ny);
// The Fourier region of a problem, fsym (part: fp_setup_partials doubles of scratch); face grids
// (face = 1) take the cosine basis.  scale = 1 (SYLV_PC_FOURIER_DIAG): also the diagonal scale
// 1 / s [k][n_pix] into sc64 / sc32; scale = 2 (SYLV_PC_FOURIER_BLOCK): the block scale T
// [k(k+1)/2][n_pix]; both from the mixing blocks M64 (packed, as k_setup writes them); a null
// sc64 or sc32 skips that precision.
hipError_t launch_fp_setup(const double *W, const double *A, int f, int k, int nx, int ny,
                           int face, const double *coef, double *part, double *fsym,
                           const double *M64, int scale, double *sc64, float *sc32,
                           hipStream_t s);
// Grid rows per workgroup of the block-scaled row passes (0: k nx too large for them).
int fp_rows_per_block_blk(int nx, int ny, int k, int dtype);
// Whether those passes read their stage twiddles from global memory, and their dynamic LDS bytes.
bool fp_blk_global_twiddles(int nx, int k, int dtype);
size_t fp_lds_bytes_blk(int nx, int k, int dtype, bool gtw);
// z = Fourier preconditioner of r for every instance of the set, in float32 (f32) or float64;
// inner = 1: the float32 inner runs of the mixed path, 0: the float64 runs, -1: the stand-alone
// preconditioner (one instance without run state: r read from rin, z written to zout).  upd
// (runs only): 1 = start of a run (the ||r||^2 partials of r), 2 = CG iteration it, whose update
// r -= alpha q (alpha from the apply's <p, q> partials) the forward row pass performs.
hipError_t launch_fp_apply(const InstSet &set, int k, int f32, int inner, const void *rin,
                           void *zout, int upd, int it, hipStream_t s);
// Dynamic LDS bytes of a row pass (pass 0: m rows of length n) or of the column pass (pass 1:
// m components of length n) in precision dtype.
size_t fp_lds_bytes(int pass, int n, int m, int dtype);
// Whether the column pass reads its FFT twiddles from global memory (its column and the table
// do not both fit in LDS).
bool fp_cols_global_twiddles(int ny, int k, int dtype);
// Bit of a transform length's final-radix class in InstSet.fp_rmask_x / fp_rmask_y.
int fp_radix_bit(int logn);

// Working sets above this many bytes are streamed past the last-level cache (256 MB on MI355X).
constexpr double kStreamBytes = 256.0 * (1 << 20);
hipError_t launch_precond_plain(const Inst *table0, int k, int dtype, int n_pix, int nrhs,
                                const void *in, void *out, hipStream_t s);
// residual r = b - G x (float64); phase 0: initial (sets ||b||, ||r0||, threshold),
// 1: final true residual only, 2: refinement step of the mixed path
hipError_t launch_resid(const InstSet &set, int k, int phase, hipStream_t s);
hipError_t launch_resid_fin(const InstSet &set, int phase, hipStream_t s);
hipError_t launch_pinit(const InstSet &set, int k, int mixed, double inner_tol, double safety,
                        int max_iter, hipStream_t s);
hipError_t launch_cg_apply(const InstSet &set, int k, int mixed, int it, hipStream_t s);
hipError_t launch_cg_update(const InstSet &set, int k, int mixed, int it, hipStream_t s);
hipError_t launch_refine_axpy(const InstSet &set, int k, hipStream_t s);
hipError_t launch_state_init(const InstSet &set, double tol, int max_iter, int ref,
                             hipStream_t s);
hipError_t launch_count_running(const InstSet &set, int inner, int *out, hipStream_t s);
// Copy `bytes` (a multiple of 4) of host memory to device memory `dst` in stream order, through
// kernel arguments (kUploadWords words per launch).  `src` may be freed on return.
hipError_t launch_upload(void *dst, const void *src, size_t bytes, hipStream_t s);
// Fold the partials of <p, q> (after a CG apply) or of <r, z>, ||r||^2 (after an update or a
// run start) of the instances with Inst::pre set; a no-op launch is skipped when none has it.
hipError_t launch_prereduce_pq(const InstSet &set, int mixed, hipStream_t s);
hipError_t launch_prereduce_rz(const InstSet &set, hipStream_t s);
hipError_t launch_stats(const InstSet &set, void *stats, int mixed, hipStream_t s);
hipError_t launch_po(const double *kappa, const double *tau, const double *A, const double *W,
                     const double *xi, const double *zeta, double *eta, int k, int f, int ny,
                     int nx, int bc, int nrhs, hipStream_t s);
hipError_t launch_grad(const double *coef, const double *A, const double *W, const double *Y,
                       const double *X, const double *Lm, int k, int f, int ny, int nx, int bc,
                       double *dkappa, double *dtau, double *dA, double *dW, double *dY,
                       double *partial, hipStream_t s);
int grad_blocks(int n_pix);
int grad_nv(int k, int f);

// block CG (sylv_block.hip); s in {2, 4, 8}
int block_rhs_supported(int s);
hipError_t launch_bpinit(const GroupSet &g, int k, int mixed, hipStream_t st);
hipError_t launch_bgram(const GroupSet &g, int phase, int mixed, double inner_tol, double safety,
                        int max_iter, hipStream_t st);
hipError_t launch_bdir(const GroupSet &g, int k, int mixed, int it, hipStream_t st);
hipError_t launch_bapply(const GroupSet &g, int k, int mixed, int it, hipStream_t st);
hipError_t launch_bupdate(const GroupSet &g, int k, int mixed, int it, hipStream_t st);

// ---- Lanczos-Sylvester (sylv_lanczos.hip) ----------------------------------------------------
// Small matrices of one solve, computed on the host before the first launch.
struct LzConst {
    double coef[4];               // c0, c1, cd, c2 of the 13-point stencil of (kappa^2 - Lap)^2
    double tap[kMaxK][kMaxF];     // t_f A[f][j] / tau_j: Yhat_p[j] = sum_f Y[f][p] tap[j][f]
    double tau[kMaxK];
    double ata[kMaxK][kMaxK];     // A^T T A
    double U[kMaxK][kMaxK];       // Lhat = U diag(rho) U^-1, U^T P^-1 U = I (Lemma 2)
    double rho[kMaxK];
    double tol;
    double kappa2;                // kappa^2 (face grids: per-pixel stencil coefficients)
};
// Device state of one solve (written only by the one-workgroup finishing kernels).
struct LzState {
    double nb0;                   // ||B_0||_F
    double thresh;                // tol * ||B_0||_F
    double gamma;                 // Alg. 5's residual estimate after the last step
    double rr, bb;                // ||b - G x||^2 and ||b||^2 of the final check
    int32_t iter;                 // Lanczos steps whose coefficients are complete
    int32_t done, status, max_iter;
    double S[kMaxK][kMaxK][kMaxK];   // per column l: Schur complement of T_i + rho_l I
    double y[kMaxK][kMaxK];          // per column l: forward-eliminated right-hand side
};
constexpr int kLzStride = kMaxK * kMaxK;   // one k x k coefficient block (row-major, ld kMaxK)
// Kernel argument block of every Lanczos-Sylvester kernel.
struct LzArgs {
    int ny, nx, n_pix, k, f, tiles_x, ntiles, nchunks, nred, rows, bc;
    const LzConst *c;
    LzState *st;
    double *H;                    // [max_iter] blocks: H_1 .. (symmetric part)
    double *B;                    // [max_iter + 1] blocks: B_0, B_2, B_3, .. (upper triangular)
    double *Binv;                 // their inverses
    double *hist;                 // [max_iter] sqrt(gamma_i) / ||B_0||_F
    double *partial;              // [kLzSlots][nred]: per-workgroup partials of a pass
    double *partial2;             // [kLzSlots]: the final sums of a pass
    const double *n, *Y;
    double *Yh, *Wa0, *Wa1, *basis, *X;
    const double *G;              // [iters] blocks of the solution coefficients Z
    int ring;                     // 0: basis block i in slot i (all kept); 1: two slots, i & 1
                                  // (the solution is assembled by a second Lanczos pass)
};
// P = V^T N Wa (k^2), C = V^T N V and E = Wa^T N Wa (k(k+1)/2 each), plus one count
constexpr int kLzSlots = kMaxK * kMaxK + kMaxK * (kMaxK + 1) + 1;
hipError_t lz_launch_init(const LzArgs &a, int max_iter, hipStream_t s);
hipError_t lz_launch_start(const LzArgs &a, hipStream_t s);
hipError_t lz_launch_step(const LzArgs &a, int it, hipStream_t s);
hipError_t lz_launch_flag(const LzArgs &a, int *host_running, hipStream_t s);
hipError_t lz_launch_finish(const LzArgs &a, int iters, hipStream_t s);
// Step `it` of the second Lanczos pass (a.ring = 1): regenerate V_it from the kept H, B blocks
// and add V_it G_(it-1) into a.X.
hipError_t lz_launch_replay(const LzArgs &a, int it, hipStream_t s);
// Residual pass of eq. (Axb) for a.X (stencil pass, reduction, ||r||^2 and ||b||^2 into a.st);
// needs the start block a.Yh (lz_launch_start).
hipError_t lz_launch_resid(const LzArgs &a, hipStream_t s);
int lz_tiles(int ny, int nx, int rows);

// ---- sparse-dense Sylvester solver, Alg. 3 (sylv_kohler.hip) -------------------------------
// Right-hand sides of the shifted column systems: b_i = n (.) (Yh Fw e_i - sum_(l<i) Rc[l][i] xhat_l)
struct KhCoef {
    double Fw[kMaxK][kMaxK];      // F -> F W (column transform of the right-hand side)
    double Rc[kMaxK][kMaxK];      // strictly upper part of R (zero when decoupled)
};
struct KhBack {
    double T[kMaxK][kMaxK];       // M = Xhat T, T = W^-1
};
hipError_t kh_launch_rhs(const double *Yh, const double *n, const double *Xh, const KhCoef &c,
                         int k, int i0, int i1, int n_pix, double *b, hipStream_t s);
hipError_t kh_launch_back(const double *Xh, const KhBack &t, int k, int n_pix, double *X,
                          hipStream_t s);
hipError_t kh_launch_zero(double *x, long n, hipStream_t s);
hipError_t kh_launch_relres(const LzState *st, double *out, hipStream_t s);
int lz_rows_valid(int k, int rows);

}  // namespace sylv
