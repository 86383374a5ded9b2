// Host side of libsylv: argument validation, workspace layout, and the driver loops of the
// preconditioned CG solve (Alg. 2 plus preconditioner; float64 or mixed precision with float64
// iterative refinement) and of its adjoint.  Everything numerical runs in the kernels of
// sylv_kernels.hip; the host only enqueues launches and, every `check_every` iterations, reads
// one integer (how many runs are still going) to decide whether to enqueue more.

#include "sylv.h"
#include "sylv_internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <utility>
#include <vector>

using namespace sylv;

// The workspace of sylv_pcg_solve_noalloc.  Each device the library runs on holds its own copy
// from the first use until the process ends.  In host code `scratch` names a host-side stand-in,
// never device memory: kernels receive the device address from hipGetSymbolAddress.
static_assert(SYLV_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size is a multiple of 256");
static __device__ __align__(256) unsigned char scratch[SYLV_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local char g_err[512] = "";

void set_err(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

constexpr size_t kAlign = 256;
// Prefix-sum arrays of the instance table: float64 and float32 apply tiles, streaming chunks,
// and the Fourier preconditioner's row-pass and column-pass workgroups.
constexpr int kPrefixArrays = 5;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Optional override of the apply kernels' rows per lane (2, 4 or 8) for tuning experiments.
// Partial count above which an instance's CG reductions are folded separately: kPreReduce, or
// SYLV_PREREDUCE_MIN from the environment (read at every solve call; tests set 0 to force it).
int prereduce_min() {
    const char *e = getenv("SYLV_PREREDUCE_MIN");
    if (!e || !*e) return kPreReduce;
    const int v = atoi(e);
    return v >= 0 ? v : kPreReduce;
}

// Safety factor of the inner tolerance of mixed runs: kInnerSafety, or SYLV_INNER_SAFETY from
// the environment (in (0, 1], read at every solve call).
double inner_safety() {
    const char *e = getenv("SYLV_INNER_SAFETY");
    if (!e || !*e) return kInnerSafety;
    const double v = atof(e);
    return (v > 0.0 && v <= 1.0) ? v : kInnerSafety;
}

// Whether kernels stream their once-touched planes past the last-level cache: when the bytes a
// solve (or apply) keeps touching exceed kStreamBytes, or as SYLV_STREAM (0 or 1) forces for
// experiments (read at every call).
int stream_policy(double working_set_bytes) {
    const char *e = getenv("SYLV_STREAM");
    if (e && (e[0] == '0' || e[0] == '1') && e[1] == 0) return e[0] - '0';
    return working_set_bytes > kStreamBytes ? 1 : 0;
}

int apply_rows_request() {
    static int rows = -1;
    if (rows < 0) {
        const char *e = getenv("SYLV_APPLY_ROWS");
        const int v = e ? atoi(e) : 0;
        rows = apply_rows_valid(v) ? v : 0;
    }
    return rows;
}

// Rows per lane of the Lanczos-Sylvester stencil kernels (2, or 4 for k <= 4); SYLV_LZ_ROWS
// overrides the default for tuning experiments.
int lz_rows_for(int k) {
    static int req = -1;
    if (req < 0) {
        const char *e = getenv("SYLV_LZ_ROWS");
        req = e ? atoi(e) : 0;
    }
    if (req > 0 && lz_rows_valid(k, req)) return req;
    return 2;
}

int tiles_for(int ny, int nx, int rows) {
    const int tx = (nx + kTileX - 1) / kTileX;
    const int ty = (ny + kWavesY * rows - 1) / (kWavesY * rows);
    return tx * ty;
}
int chunks_for(int n_pix) { return (n_pix + kChunk - 1) / kChunk; }


struct ProbLayout {
    size_t coef, M64, M32, P64, P32, P16;
    size_t fsym, fpart;   // Fourier preconditioner: symbol block and the weight-mean partials
    size_t fsc64, fsc32;  // its diagonal or block scale, on Fourier grids only
};
struct InstLayout {
    size_t st, partial, b, r, z, p, p2, q, r32, z32, p32, p32b, q32, d32;
    size_t fs;            // Fourier preconditioner: half spectrum (0 = none)
    int nred;
};
struct Layout {
    std::vector<ProbLayout> prob;
    std::vector<InstLayout> inst;
    std::vector<size_t> gstate, gpart;   // block CG: per-group state and partials
    std::vector<int> gnred;
    size_t groups = 0, gprefix = 0;
    size_t table = 0, tprefix = 0, count = 0, gpartial = 0;
    size_t fs1 = 0;       // stand-alone Fourier preconditioner's half spectrum (0 = none)
    size_t total = 0;
};

// Whether a grid can take the Fourier preconditioner in some precision (the stand-alone
// workspace then holds its spectrum), and the spectrum's bytes (complex float64 half spectrum;
// the cosine coefficients of face grids take less).
// The Fourier-basis preconditioners (plain, diagonally scaled, block scaled).
bool is_fourier(int pc) {
    return pc == SYLV_PC_FOURIER || pc == SYLV_PC_FOURIER_DIAG || pc == SYLV_PC_FOURIER_BLOCK;
}

bool fp_grid(const sylv_problem &p) {
    char why[160];
    return fp_supported((int)p.ny, (int)p.nx, p.k, SYLV_F32, why, sizeof(why));
}
size_t fp_spectrum_bytes(const sylv_problem &p) {
    return (size_t)16 * p.k * (size_t)(p.nx / 2 + 1) * (size_t)p.ny;
}

bool check_problem(const sylv_problem *p, int idx) {
    if (!p) { set_err("problem %d: null pointer", idx); return false; }
    if (p->k < 1 || p->k > kMaxK) { set_err("problem %d: k=%d outside [1, %d]", idx, p->k, kMaxK); return false; }
    if (p->f < 1 || p->f > kMaxF) { set_err("problem %d: f=%d outside [1, %d]", idx, p->f, kMaxF); return false; }
    if (p->ny < 1 || p->nx < 1) { set_err("problem %d: grid %lld x %lld", idx, (long long)p->ny, (long long)p->nx); return false; }
    if (p->ny * p->nx >= (int64_t)1 << 29) { set_err("problem %d: n_pix >= 2^29", idx); return false; }
    if (!p->kappa || !p->tau || !p->A || !p->W) { set_err("problem %d: null parameter pointer", idx); return false; }
    if (p->boundary != SYLV_BC_PERIODIC && p->boundary != SYLV_BC_FACE) { set_err("problem %d: boundary %d", idx, p->boundary); return false; }
    return true;
}

// Block CG groups a problem's right-hand sides into blocks of 2, 4 or 8 columns.
int max_groups_per_problem(int nrhs) { return nrhs % 2 == 0 ? nrhs / 2 : 0; }
int block_size_for(int nrhs, int requested) { return requested > 0 ? requested : nrhs; }
bool block_size_ok(int nrhs, int bs) { return block_rhs_supported(bs) && nrhs % bs == 0; }

// Workspace: per-problem operator regions first (so that the layout of the operator of a single
// problem does not depend on the call), then the instance table and prefixes, the run states,
// reduction partials, solver vectors and the gradient partials.
bool make_layout(const sylv_problem *probs, int nprob, int nrhs, bool solve, Layout &L,
                 int pc = SYLV_PC_BLOCK) {
    size_t off = 0;
    L.prob.resize(nprob);
    for (int g = 0; g < nprob; ++g) {
        const size_t n = (size_t)probs[g].ny * probs[g].nx;
        const size_t mk = (size_t)packed_size(probs[g].k);
        ProbLayout &P = L.prob[g];
        P.coef = off; off = align_up(off + sizeof(double) * kCoefStride * kMaxK);
        P.M64 = off;  off = align_up(off + sizeof(double) * mk * n);
        P.M32 = off;  off = align_up(off + sizeof(float) * mk * n);
        P.P64 = off;  off = align_up(off + sizeof(double) * mk * n);
        P.P32 = off;  off = align_up(off + sizeof(float) * mk * n);
        P.P16 = off;  off = align_up(off + sizeof(unsigned short) * mk * n);
        P.fsym = off; off = align_up(off + fp_table_bytes((int)probs[g].nx, (int)probs[g].ny));
        P.fpart = off; off = align_up(off + sizeof(double) * fp_setup_partials((int)n, probs[g].f));
        P.fsc64 = P.fsc32 = 0;
        // a solve lays out its operator for itself: the scale planes only for the scaled kinds;
        // the stand-alone layout (one problem, any later sylv_precond kind) always on these grids
        const bool scaled = pc == SYLV_PC_FOURIER_DIAG || pc == SYLV_PC_FOURIER_BLOCK;
        if (fp_grid(probs[g]) && (!solve || scaled)) {
            const size_t vk = (size_t)packed_size(probs[g].k) * n;   // block: k(k+1)/2 planes
            P.fsc64 = off; off = align_up(off + sizeof(double) * vk);
            P.fsc32 = off; off = align_up(off + sizeof(float) * vk);
        }
    }
    if (!solve && nprob == 1 && fp_grid(probs[0])) {
        L.fs1 = off;
        off = align_up(off + fp_spectrum_bytes(probs[0]));
    }
    const int ninst = solve ? nprob * nrhs : 1;
    L.table = off;   off = align_up(off + sizeof(Inst) * ninst);
    L.tprefix = off; off = align_up(off + sizeof(int) * kPrefixArrays * (ninst + 1));
    L.count = off;   off = align_up(off + sizeof(int) * 4);
    if (solve) {
        L.inst.resize(ninst);
        for (int g = 0; g < nprob; ++g) {
            const int ny = (int)probs[g].ny, nx = (int)probs[g].nx, k = probs[g].k;
            const size_t n = (size_t)ny * nx;
            const size_t vk = (size_t)k * n;
            for (int r = 0; r < nrhs; ++r) {
                InstLayout &I = L.inst[(size_t)g * nrhs + r];
                I.nred = std::max(std::max(tiles_for(ny, nx, 2), chunks_for((int)n)),
                                  std::max(nx / 2 + 1, k * ny / 2));
                I.st = off;      off = align_up(off + 2 * sizeof(DevState));
                I.partial = off; off = align_up(off + sizeof(double) * kNumSlots * I.nred);
                I.b = off;   off = align_up(off + sizeof(double) * vk);
                I.r = off;   off = align_up(off + sizeof(double) * vk);
                I.z = off;   off = align_up(off + sizeof(double) * vk);
                I.p = off;   off = align_up(off + sizeof(double) * vk);
                I.p2 = off;  off = align_up(off + sizeof(double) * vk);
                I.q = off;   off = align_up(off + sizeof(double) * vk);
                I.r32 = off; off = align_up(off + sizeof(float) * vk);
                I.z32 = off; off = align_up(off + sizeof(float) * vk);
                I.p32 = off; off = align_up(off + sizeof(float) * vk);
                I.p32b = off; off = align_up(off + sizeof(float) * vk);
                I.q32 = off; off = align_up(off + sizeof(float) * vk);
                I.d32 = off; off = align_up(off + sizeof(float) * vk);
                I.fs = 0;
                if (is_fourier(pc)) {
                    I.fs = off;
                    off = align_up(off + fp_spectrum_bytes(probs[g]));
                }
            }
        }
        // block CG tables, sized whenever a call could use them: up to nrhs / 2 groups (blocks
        // of 2 columns) per problem, group (g, b) at index g * (nrhs / 2) + b
        const int gpp = max_groups_per_problem(nrhs);
        const int ng = nprob * gpp;
        L.groups = off; off = align_up(off + sizeof(Group) * std::max(ng, 1));
        L.gprefix = off; off = align_up(off + sizeof(int) * 3 * (ng + 1));
        L.gstate.resize(ng);
        L.gpart.resize(ng);
        L.gnred.resize(ng);
        for (int g = 0; g < nprob; ++g) {
            const int ny = (int)probs[g].ny, nx = (int)probs[g].nx;
            const int n = ny * nx;
            for (int b = 0; b < gpp; ++b) {
                const int i = g * gpp + b;
                L.gnred[i] = std::max(tiles_for(ny, nx, kBlockRows), (n + kBlockPix - 1) / kBlockPix);
                L.gstate[i] = off; off = align_up(off + sizeof(GroupState));
                L.gpart[i] = off;  off = align_up(off + sizeof(double) * kBlockQ * L.gnred[i]);
            }
        }
        if (nprob == 1 && nrhs == 1) {
            const int n_pix = (int)(probs[0].ny * probs[0].nx);
            L.gpartial = off;
            off = align_up(off + sizeof(double) * grad_nv(probs[0].k, probs[0].f) *
                                     grad_blocks(n_pix));
        }
    }
    L.total = off;
    return true;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            set_err("%s failed: %s", #expr, hipGetErrorString(e_));                     \
            return SYLV_E_HIP;                                                          \
        }                                                                               \
    } while (0)

Inst operator_inst(const sylv_problem &p, const ProbLayout &P, char *base, int pc) {
    Inst I;
    memset(&I, 0, sizeof(I));
    I.ny = (int)p.ny;
    I.nx = (int)p.nx;
    I.n_pix = (int)(p.ny * p.nx);
    I.tiles_x = (I.nx + kTileX - 1) / kTileX;
    I.pc = is_fourier(pc) ? SYLV_PC_FOURIER : pc;   // the kernels tell the two apart by fsc64
    if (pc == SYLV_PC_FOURIER_DIAG || pc == SYLV_PC_FOURIER_BLOCK) {
        I.fsc64 = reinterpret_cast<const double *>(base + P.fsc64);
        I.fsc32 = reinterpret_cast<const float *>(base + P.fsc32);
    }
    I.f = p.f;
    I.coef = reinterpret_cast<const double *>(base + P.coef);
    I.A = p.A;
    I.W = p.W;
    I.M64 = reinterpret_cast<const double *>(base + P.M64);
    I.M32 = reinterpret_cast<const float *>(base + P.M32);
    I.P64 = reinterpret_cast<const double *>(base + P.P64);
    I.P32 = reinterpret_cast<const float *>(base + P.P32);
    I.P16 = reinterpret_cast<const unsigned short *>(base + P.P16);
    return I;
}

// exact = 1 also stores the exact block inverses (float64 and float32) that the stand-alone
// sylv_precond reads; CG runs read only the bfloat16 factor.
// prec: which precisions of the Fourier scales to make (bit 0 float32, bit 1 float64; a solve
// makes the one its runs read, the stand-alone set-up both).
int prepare_operator(const sylv_problem &p, const ProbLayout &P, char *base, int pc, int exact,
                     hipStream_t s, int prec = 3) {
    double *coef = reinterpret_cast<double *>(base + P.coef);
    HIP_TRY(launch_coef(p.kappa, p.tau, p.k, (int)p.ny, (int)p.nx, coef, s));
    HIP_TRY(launch_setup(p.W, p.A, p.f, (int)p.ny, (int)p.nx, p.boundary, coef, pc,
                         reinterpret_cast<double *>(base + P.M64),
                         reinterpret_cast<float *>(base + P.M32),
                         reinterpret_cast<double *>(base + P.P64),
                         reinterpret_cast<float *>(base + P.P32),
                         reinterpret_cast<unsigned short *>(base + P.P16), exact, p.k, s));
    if (is_fourier(pc)) {
        const int scale = pc == SYLV_PC_FOURIER_DIAG ? 1 : pc == SYLV_PC_FOURIER_BLOCK ? 2 : 0;
        HIP_TRY(launch_fp_setup(p.W, p.A, p.f, p.k, (int)p.nx, (int)p.ny,
                                p.boundary == SYLV_BC_FACE ? 1 : 0, coef,
                                reinterpret_cast<double *>(base + P.fpart),
                                reinterpret_cast<double *>(base + P.fsym),
                                reinterpret_cast<const double *>(base + P.M64), scale,
                                scale && (prec & 2) ? reinterpret_cast<double *>(base + P.fsc64)
                                                    : nullptr,
                                scale && (prec & 1) ? reinterpret_cast<float *>(base + P.fsc32)
                                                    : nullptr, s));
    }
    return SYLV_OK;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

int check_ws(void *ws, size_t ws_bytes, size_t need) {
    if (!ws) { set_err("null workspace"); return SYLV_E_INVALID; }
    if (((uintptr_t)ws & (kAlign - 1)) != 0) { set_err("workspace not 256-byte aligned"); return SYLV_E_INVALID; }
    if (ws_bytes < need) {
        set_err("workspace of %zu bytes, %zu needed", ws_bytes, need);
        return SYLV_E_WORKSPACE;
    }
    return SYLV_OK;
}

int check_opts(const sylv_pcg_opts *o) {
    if (!o) { set_err("null opts"); return SYLV_E_INVALID; }
    if (!(o->tol > 0.0) || !(o->tol < 1.0)) { set_err("tol must be in (0, 1)"); return SYLV_E_INVALID; }
    if (o->max_iter < 1) { set_err("max_iter must be >= 1"); return SYLV_E_INVALID; }
    if (o->precision != SYLV_PREC_F64 && o->precision != SYLV_PREC_MIXED) { set_err("bad precision"); return SYLV_E_INVALID; }
    if (o->precond < SYLV_PC_NONE || o->precond > SYLV_PC_FOURIER_BLOCK) { set_err("bad precond"); return SYLV_E_INVALID; }
    if (o->inner_tol < 0.0 || o->inner_tol >= 1.0) { set_err("inner_tol must be in [0, 1)"); return SYLV_E_INVALID; }
    if (o->refine_max < 0 || o->check_every < 0) { set_err("negative refine_max/check_every"); return SYLV_E_INVALID; }
    if (o->stop_ref != SYLV_STOP_R0 && o->stop_ref != SYLV_STOP_B) { set_err("bad stop_ref"); return SYLV_E_INVALID; }
    if (o->schedule != SYLV_SCHED_ADAPTIVE && o->schedule != SYLV_SCHED_FIXED) { set_err("bad schedule"); return SYLV_E_INVALID; }
    if (o->block_size != 0 && !block_rhs_supported(o->block_size)) { set_err("block_size must be 0, 2, 4 or 8"); return SYLV_E_INVALID; }
    if (o->apply_rows != 0 && !apply_rows_valid(o->apply_rows)) { set_err("apply_rows must be 0, 2, 4 or 8"); return SYLV_E_INVALID; }
    if (o->schedule == SYLV_SCHED_FIXED) {
        // every queued iteration is a few launches (graph nodes when captured): keep it bounded
        const long long steps = o->precision == SYLV_PREC_MIXED ? (o->refine_max > 0 ? o->refine_max : 8) : 1;
        const long long queued = ((long long)o->max_iter + 1) * steps;
        if (queued > kMaxFixedIters) {
            set_err("fixed schedule: (max_iter + 1) * refinement steps = %lld exceeds %d; set "
                    "max_iter and refine_max near what the solve needs",
                    queued, kMaxFixedIters);
            return SYLV_E_INVALID;
        }
    }
    return SYLV_OK;
}

// A call that must synchronise refuses a stream under graph capture (a wait there would fail
// half-way through the enqueued work).
int refuse_capture(hipStream_t s, const char *what) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone) {
        set_err("%s synchronises with the host and cannot be captured", what);
        return SYLV_E_INVALID;
    }
    return SYLV_OK;
}

// Host-side completion flags: the count kernel writes the number of unfinished runs straight
// into pinned host memory and an event marks when it is valid.  One small pinned block and a few
// events per host thread, created on first use and kept for the life of the thread.
struct HostFlags {
    static constexpr int kSlots = 4;
    static constexpr int kStride = 4;   // ints per slot (the completion report of k_count_running)
    int *pinned = nullptr;
    hipEvent_t ev[kSlots] = {};
    bool ready = false;
    ~HostFlags() {
        if (!ready) return;
        for (int i = 0; i < kSlots; ++i) (void)hipEventDestroy(ev[i]);
        (void)hipHostFree(pinned);
    }
};
thread_local HostFlags g_flags;

int host_flags(HostFlags *&out) {
    HostFlags &f = g_flags;
    if (!f.ready) {
        HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&f.pinned),
                              sizeof(int) * HostFlags::kSlots * HostFlags::kStride,
                              hipHostMallocDefault));
        for (int i = 0; i < HostFlags::kSlots; ++i)
            HIP_TRY(hipEventCreateWithFlags(&f.ev[i], hipEventDisableTiming));
        f.ready = true;
    }
    out = &f;
    return SYLV_OK;
}

// Enqueue "how many runs are unfinished" into slot `slot` (inner = 1: the float32 inner runs).
int post_count(const InstSet &set, int inner, HostFlags *f, int slot, hipStream_t s) {
    HIP_TRY(launch_count_running(set, inner, f->pinned + slot * HostFlags::kStride, s));
    HIP_TRY(hipEventRecord(f->ev[slot], s));
    return SYLV_OK;
}

struct Report {
    int running;   // runs not finished
    int iter;      // latest iteration tested among them
    double gap;    // max log2(rr / thresh) among them (0: unknown)
    double gap0;   // max log2(rr0 / thresh) among them, at their start (0: unknown)
};

int wait_report(HostFlags *f, int slot, Report &r) {
    HIP_TRY(hipEventSynchronize(f->ev[slot]));
    const volatile int *p = f->pinned + slot * HostFlags::kStride;
    r.running = p[0];
    r.iter = p[1];
    r.gap = p[2] / 256.0;
    r.gap0 = p[3] / 256.0;
    return SYLV_OK;
}

int wait_count(HostFlags *f, int slot, int &value) {
    HIP_TRY(hipEventSynchronize(f->ev[slot]));
    value = *reinterpret_cast<volatile int *>(f->pinned + slot * HostFlags::kStride);
    return SYLV_OK;
}

// Iterations still to queue after those already queued (indices below `queued`): the gap to the
// threshold shrinks about linearly in log scale, so the slowest run stops near iteration
// iter + gap / rate, the rate taken from the last two completion reports or, after the first,
// from the gap at the start of the run.  Returns a quarter batch (at least one iteration: enough
// queued work to cover the host's round trip) while no rate is known, 0 when the queued
// iterations should already finish every run, and otherwise the estimate plus one, never more
// than `chunk`.  A short estimate costs one more host round trip, an over-estimate a few
// early-exit launches; the result of the solve does not depend on it.  (het_1024 with the
// block-scaled Fourier preconditioner, whose runs take 6-7 iterations: half-batch blind queues
// and a margin of two took 1.36 ms mixed, this 1.33 ms; block-Jacobi unchanged.)
int next_batch(const Report &prev, const Report &cur, bool have_prev, bool have_cur, int queued,
               int chunk) {
    double rate = 0.0;
    if (have_cur && have_prev && cur.iter > prev.iter && cur.gap > 0.0 && prev.gap > cur.gap)
        rate = (prev.gap - cur.gap) / (cur.iter - prev.iter);
    else if (have_cur && cur.iter > 0 && cur.gap > 0.0 && cur.gap0 > cur.gap)
        rate = (cur.gap0 - cur.gap) / cur.iter;
    if (!(rate > 0.0)) return std::max(1, chunk / 4);
    const double stop = cur.iter + cur.gap / rate;
    const double left = stop - (queued - 1);
    if (left <= 0.0) return 0;
    const int n = (int)ceil(left * 1.1) + 1;
    return n < chunk ? n : chunk;
}

// Conjugate-gradient iterations in batches of `chunk`, with one batch always queued ahead of the
// completion check so that the GPU never waits for the host.  Iteration `it` is apply(it)
// (stopping test on the residual of update(it-1), new direction, q = G p) followed by
// update(it); a run that has stopped turns every later kernel of the loop into a no-op, and
// apply(max_iter) always stops it, so the loop ends.
static_assert(sizeof(Inst) % 4 == 0 && sizeof(Group) % 4 == 0, "tables upload as 32-bit words");

// The Fourier preconditioner's three passes (z and <r, z> of every unfinished run).
// With the Fourier preconditioner, in the float32 inner runs of the mixed path the forward row
// pass also performs the CG update of iteration `it` (upd = 2) and, at the start of a run, takes
// the ||r||^2 partials of r (upd = 1); float64 runs keep the streaming update (fused, the float64
// row pass took longer than the two kernels apart: 42 against 22 + 18 us at 1024^2, k = 3).
int fourier_apply(const InstSet &set, int k, int mixed, int upd, int it, hipStream_t s) {
    HIP_TRY(launch_fp_apply(set, k, mixed, mixed, nullptr, nullptr, mixed ? upd : 0, it, s));
    return SYLV_OK;
}

int cg_iteration(const InstSet &set, int k, int mixed, int it, hipStream_t s) {
    HIP_TRY(launch_cg_apply(set, k, mixed, it, s));
    HIP_TRY(launch_prereduce_pq(set, mixed, s));
    if (!(set.fourier && mixed)) HIP_TRY(launch_cg_update(set, k, mixed, it, s));
    if (set.fourier) {
        const int rc = fourier_apply(set, k, mixed, 2, it, s);
        if (rc) return rc;
    }
    HIP_TRY(launch_prereduce_rz(set, s));
    return SYLV_OK;
}

int run_cg_loop(const InstSet &set, int k, int mixed, int chunk, int max_iter, HostFlags *f,
                hipStream_t s) {
    int it = 0, rc;
    if (!f) {   // fixed schedule: every iteration up to the cap, no host check
        for (; it <= max_iter; ++it)
            if ((rc = cg_iteration(set, k, mixed, it, s))) return rc;
        return SYLV_OK;
    }
    // batches queued and not yet waited for, oldest first, in slots 0 and 1 used alternately
    int pend[2], npend = 0, next_slot = 0;
    auto enqueue_batch = [&](int n) -> int {
        for (int c = 0; c < n && it <= max_iter; ++c, ++it)
            if (int e = cg_iteration(set, k, mixed, it, s)) return e;
        pend[npend++] = next_slot;
        const int slot = next_slot;
        next_slot ^= 1;
        return post_count(set, mixed, f, slot, s);
    };
    Report prev{}, cur{};
    bool have_prev = false, have_cur = false;
    if ((rc = enqueue_batch(chunk))) return rc;
    for (;;) {
        // keep one batch queued ahead of the report being waited for, sized by the estimate
        if (it <= max_iter && npend < 2) {
            int n = next_batch(prev, cur, have_prev, have_cur, it, chunk);
            if (npend == 0 && n < 4) n = 4;   // the estimate fell short: the run goes on
            if (n > 0 && (rc = enqueue_batch(n))) return rc;
        }
        if (npend == 0) break;   // every iteration up to max_iter has been waited for
        const int slot = pend[0];
        pend[0] = pend[1];
        --npend;
        prev = cur;
        have_prev = have_cur;
        if ((rc = wait_report(f, slot, cur))) return rc;
        have_cur = true;
        if (cur.running == 0) {
            while (npend > 0) {   // drain the lookahead (its kernels returned at once)
                Report r;
                if ((rc = wait_report(f, pend[0], r))) return rc;
                pend[0] = pend[1];
                --npend;
            }
            break;
        }
    }
    return SYLV_OK;
}

// Block-CG iterations: P = Z + P beta (from the second iteration), Q = G P with the P^T Q
// Gram, alpha, the block update with the R^T Z Gram, beta and the per-column stopping test.
int block_iteration(const GroupSet &gset, int k, int mixed, int it, int max_iter,
                    hipStream_t s) {
    if (it > 0) HIP_TRY(launch_bdir(gset, k, mixed, it, s));
    HIP_TRY(launch_bapply(gset, k, mixed, it, s));
    HIP_TRY(launch_bgram(gset, 1, mixed, 0.0, 0.0, max_iter, s));
    HIP_TRY(launch_bupdate(gset, k, mixed, it, s));
    HIP_TRY(launch_bgram(gset, 2, mixed, 0.0, 0.0, max_iter, s));
    return SYLV_OK;
}

int run_block_loop(const GroupSet &gset, const InstSet &set, int k, int mixed, int chunk,
                   int max_iter, HostFlags *f, hipStream_t s) {
    int it = 0, rc;
    if (!f) {   // fixed schedule
        for (; it <= max_iter; ++it)
            if ((rc = block_iteration(gset, k, mixed, it, max_iter, s))) return rc;
        return SYLV_OK;
    }
    auto enqueue_batch = [&](int slot) -> int {
        for (int c = 0; c < chunk && it <= max_iter; ++c, ++it)
            if (int e = block_iteration(gset, k, mixed, it, max_iter, s)) return e;
        return post_count(set, mixed, f, slot, s);
    };
    if ((rc = enqueue_batch(0))) return rc;
    for (int cur = 0;; cur ^= 1) {
        const bool more = it <= max_iter;
        if (more && (rc = enqueue_batch(cur ^ 1))) return rc;
        int running = 0;
        if ((rc = wait_count(f, cur, running))) return rc;
        if (running == 0 || !more) {
            if (more && (rc = wait_count(f, cur ^ 1, running))) return rc;
            break;
        }
    }
    return SYLV_OK;
}

int solve_impl(const sylv_problem *probs, int nprob, int nrhs, const double *Y,
               const double *Bextra, double *X, const sylv_pcg_opts *opts,
               sylv_pcg_stats *stats, void *ws, size_t ws_bytes, hipStream_t s, Layout &L) {
    if (nprob < 1 || nrhs < 1) { set_err("nprob and nrhs must be >= 1"); return SYLV_E_INVALID; }
    for (int g = 0; g < nprob; ++g)
        if (!check_problem(&probs[g], g)) return SYLV_E_INVALID;
    const int k = probs[0].k;
    for (int g = 1; g < nprob; ++g)
        if (probs[g].k != k) { set_err("all problems of a call must share k"); return SYLV_E_INVALID; }
    const int bc = probs[0].boundary;
    for (int g = 1; g < nprob; ++g)
        if (probs[g].boundary != bc) { set_err("all problems of a call must share the boundary"); return SYLV_E_INVALID; }
    int rc = check_opts(opts);
    if (rc) return rc;
    if (!X || !stats) { set_err("null X or stats"); return SYLV_E_INVALID; }
    const bool fixed = opts->schedule == SYLV_SCHED_FIXED;
    if (!Y && !Bextra) { set_err("need Y or Bextra"); return SYLV_E_INVALID; }
    const bool block = opts->block != 0;
    const int bsize = block_size_for(nrhs, opts->block_size);
    if (block && !block_size_ok(nrhs, bsize)) {
        set_err("block CG needs a block size in {2, 4, 8} dividing nrhs (block %d, nrhs %d)",
                bsize, nrhs);
        return SYLV_E_INVALID;
    }
    const int fourier = is_fourier(opts->precond);
    int blk_gtw = 0;   // length classes (fp_radix_bit) whose block-scaled row passes read global
                       // twiddles
    if (fourier) {
        if (block) { set_err("block CG takes the per-pixel preconditioners only"); return SYLV_E_INVALID; }
        const int dt = opts->precision == SYLV_PREC_MIXED ? SYLV_F32 : SYLV_F64;
        for (int g = 0; g < nprob; ++g) {
            char why[200];
            if (!fp_supported((int)probs[g].ny, (int)probs[g].nx, k, dt, why, sizeof(why))) {
                set_err("problem %d: %s", g, why);
                return SYLV_E_INVALID;
            }
            if (opts->precond == SYLV_PC_FOURIER_BLOCK &&
                !fp_rows_per_block_blk((int)probs[g].nx, (int)probs[g].ny, k, dt)) {
                set_err("problem %d: the block-scaled Fourier preconditioner's row passes hold "
                        "every component of two grid rows: k * nx = %d > 8192", g,
                        k * (int)probs[g].nx);
                return SYLV_E_INVALID;
            }
        }
    }
    make_layout(probs, nprob, nrhs, true, L, opts->precond);
    rc = check_ws(ws, ws_bytes, L.total);
    if (rc) return rc;
    if (!fixed && (rc = refuse_capture(s, "the adaptive schedule"))) return rc;
    char *base = reinterpret_cast<char *>(ws);
    const int mixed = opts->precision == SYLV_PREC_MIXED;
    // face grids run the apply kernels with 2 rows per lane
    const int rreq = opts->apply_rows > 0 ? opts->apply_rows : apply_rows_request();
    const int rows64 = bc == SYLV_BC_FACE ? 2 : apply_rows_for(k, SYLV_F64, rreq);
    const int rows32 = bc == SYLV_BC_FACE ? 2 : apply_rows_for(k, SYLV_F32, rreq);
    const int pc = opts->precond;

    // instance table
    const int ninst = nprob * nrhs;
    std::vector<Inst> tab(ninst);
    std::vector<int> pre(kPrefixArrays * (ninst + 1));
    int *tpre = pre.data(), *tpre32 = tpre + (ninst + 1), *cpre = tpre32 + (ninst + 1);
    int *fpa = cpre + (ninst + 1), *fpb = fpa + (ninst + 1);
    size_t fp_lds_rows = 0, fp_lds_cols = 0;
    int fp_cols_gtw = 0, fp_rmask_x = 0, fp_rmask_y = 0;
    size_t xoff = 0, yoff = 0;
    int any_pre = 0;
    const int pre_min = prereduce_min();
    tpre[0] = tpre32[0] = cpre[0] = fpa[0] = fpb[0] = 0;
    for (int g = 0; g < nprob; ++g) {
        const sylv_problem &p = probs[g];
        const size_t n = (size_t)p.ny * p.nx;
        for (int r = 0; r < nrhs; ++r) {
            const int i = g * nrhs + r;
            const InstLayout &IL = L.inst[i];
            Inst I = operator_inst(p, L.prob[g], base, pc);
            I.ntiles = tiles_for(I.ny, I.nx, rows64);
            I.ntiles32 = tiles_for(I.ny, I.nx, rows32);
            I.nchunks = chunks_for(I.n_pix);
            I.nrr = I.nchunks;
            I.nred = IL.nred;
            I.Y = Y ? Y + yoff : nullptr;
            I.bext = Bextra ? Bextra + xoff + (size_t)r * k * n : nullptr;
            I.b = reinterpret_cast<double *>(base + IL.b);
            I.x = X + xoff + (size_t)r * k * n;
            I.r = reinterpret_cast<double *>(base + IL.r);
            I.z = reinterpret_cast<double *>(base + IL.z);
            I.p[0] = reinterpret_cast<double *>(base + IL.p);
            I.p[1] = reinterpret_cast<double *>(base + IL.p2);
            I.q = reinterpret_cast<double *>(base + IL.q);
            I.r32 = reinterpret_cast<float *>(base + IL.r32);
            I.z32 = reinterpret_cast<float *>(base + IL.z32);
            I.p32[0] = reinterpret_cast<float *>(base + IL.p32);
            I.p32[1] = reinterpret_cast<float *>(base + IL.p32b);
            I.q32 = reinterpret_cast<float *>(base + IL.q32);
            I.d32 = reinterpret_cast<float *>(base + IL.d32);
            I.st = reinterpret_cast<DevState *>(base + IL.st);
            I.st_in = I.st + 1;
            I.partial = reinterpret_cast<double *>(base + IL.partial);
            I.vec4 = (I.n_pix % 4 == 0) && aligned16(I.x) ? 1 : 0;
            int nfa = 0, nfb = 0;
            if (fourier) {
                I.fs = reinterpret_cast<double *>(base + IL.fs);
                I.fsym = reinterpret_cast<const double *>(base + L.prob[g].fsym);
                I.lognx = __builtin_ctz((unsigned)I.nx);
                I.logny = __builtin_ctz((unsigned)I.ny);
                const bool blk = pc == SYLV_PC_FOURIER_BLOCK;
                I.frb = blk ? fp_rows_per_block_blk(I.nx, I.ny, k, mixed ? SYLV_F32 : SYLV_F64)
                            : fp_rows_per_block(I.nx, I.ny, mixed ? SYLV_F32 : SYLV_F64);
                I.nfft = I.nx / 2;
                nfa = blk ? I.ny / I.frb : k * (I.ny / I.frb);
                I.nrr = mixed ? nfa : I.nchunks;   // the producer of ||r||^2 (see fourier_apply)
                nfb = I.nfft;
                const int dt = mixed ? SYLV_F32 : SYLV_F64;
                // global twiddles are chosen per length class: a class with any instance that
                // needs them reads them so for all its instances (right for every length of the
                // class; the LDS is sized for the largest need)
                const bool rg = blk && fp_blk_global_twiddles(I.nx, k, dt);
                if (rg) blk_gtw |= fp_radix_bit(I.lognx);
                fp_lds_rows = std::max(fp_lds_rows, blk ? fp_lds_bytes_blk(I.nx, k, dt, rg)
                                                        : fp_lds_bytes(0, I.nx, I.frb, dt));
                fp_lds_cols = std::max(fp_lds_cols, fp_lds_bytes(1, I.ny, k, dt));
                if (fp_cols_global_twiddles(I.ny, k, dt)) fp_cols_gtw |= fp_radix_bit(I.logny);
                fp_rmask_x |= fp_radix_bit(I.lognx);
                fp_rmask_y |= fp_radix_bit(I.logny);
            }
            I.pre = std::max(std::max(I.ntiles, I.ntiles32), I.nchunks) > pre_min ? 1 : 0;
            any_pre |= I.pre;
            tab[i] = I;
            tpre[i + 1] = tpre[i] + I.ntiles;
            tpre32[i + 1] = tpre32[i] + I.ntiles32;
            cpre[i + 1] = cpre[i] + I.nchunks;
            fpa[i + 1] = fpa[i] + nfa;
            fpb[i + 1] = fpb[i] + nfb;
        }
        xoff += (size_t)nrhs * k * n;
        yoff += (size_t)p.f * n;
    }
    HIP_TRY(launch_upload(base + L.table, tab.data(), sizeof(Inst) * ninst, s));
    HIP_TRY(launch_upload(base + L.tprefix, pre.data(), sizeof(int) * kPrefixArrays * (ninst + 1), s));
    InstSet set;
    set.table = reinterpret_cast<const Inst *>(base + L.table);
    set.tprefix = reinterpret_cast<const int *>(base + L.tprefix);
    set.tprefix32 = set.tprefix + (ninst + 1);
    set.cprefix = set.tprefix32 + (ninst + 1);
    set.ninst = ninst;
    set.total_tiles = tpre[ninst];
    set.total_tiles32 = tpre32[ninst];
    set.total_chunks = cpre[ninst];
    set.rows64 = rows64;
    set.rows32 = rows32;
    set.bc = bc;
    set.any_pre = any_pre;
    set.fourier = fourier;
    set.fp_scaled = opts->precond == SYLV_PC_FOURIER_DIAG ? 1 : 0;
    set.fp_block = opts->precond == SYLV_PC_FOURIER_BLOCK ? 1 : 0;
    set.fp_blk_gtw = blk_gtw;
    set.fprefa = set.cprefix + (ninst + 1);
    set.fprefb = set.fprefa + (ninst + 1);
    set.total_fa = fpa[ninst];
    set.total_fb = fpb[ninst];
    set.fp_lds_rows = fp_lds_rows;
    set.fp_lds_cols = fp_lds_cols;
    set.fp_cols_gtw = fp_cols_gtw;
    set.fp_rmask_x = fp_rmask_x;
    set.fp_rmask_y = fp_rmask_y;
    {
        // bytes the CG loop keeps touching: per problem the mixing blocks and the bfloat16
        // preconditioner factor, per instance x, r, z, two directions and q
        const double es = mixed ? 4.0 : 8.0;
        double wsb = 0.0;
        for (int g = 0; g < nprob; ++g) {
            const double n = (double)probs[g].ny * probs[g].nx, mk = packed_size(k);
            wsb += n * (mk * es + 2.0 * mk) + n * nrhs * 6.0 * k * es;
        }
        set.stream = stream_policy(wsb);
    }

    // block CG groups: nrhs / bsize per problem, each bsize consecutive instances
    GroupSet gset;
    memset(&gset, 0, sizeof(gset));
    if (block) {
        const int per = nrhs / bsize, gpp = max_groups_per_problem(nrhs);
        const int ngroup = nprob * per;
        std::vector<Group> grp(ngroup);
        std::vector<int> gpre(3 * (ngroup + 1));
        int *gt = gpre.data(), *gt32 = gt + (ngroup + 1), *gc = gt32 + (ngroup + 1);
        gt[0] = gt32[0] = gc[0] = 0;
        for (int g = 0; g < nprob; ++g) {
            const int ny = (int)probs[g].ny, nx = (int)probs[g].nx;
            for (int b = 0; b < per; ++b) {
                const int gi = g * per + b, slot = g * gpp + b;
                Group G;
                memset(&G, 0, sizeof(G));
                G.inst0 = g * nrhs + b * bsize;
                G.ntiles = tiles_for(ny, nx, kBlockRows);
                G.ntiles32 = tiles_for(ny, nx, kBlockRows);
                const int bv = kBlock * block_vec(!mixed);
                G.nchunks = (ny * nx + bv - 1) / bv;
                G.vec = (ny * nx) % block_vec(!mixed) == 0 ? 1 : 0;
                G.nred = L.gnred[slot];
                G.gs = reinterpret_cast<GroupState *>(base + L.gstate[slot]);
                G.partial = reinterpret_cast<double *>(base + L.gpart[slot]);
                grp[gi] = G;
                gt[gi + 1] = gt[gi] + G.ntiles;
                gt32[gi + 1] = gt32[gi] + G.ntiles32;
                gc[gi + 1] = gc[gi] + G.nchunks;
            }
        }
        HIP_TRY(launch_upload(base + L.groups, grp.data(), sizeof(Group) * ngroup, s));
        HIP_TRY(launch_upload(base + L.gprefix, gpre.data(), sizeof(int) * 3 * (ngroup + 1), s));
        gset.table = set.table;
        gset.groups = reinterpret_cast<const Group *>(base + L.groups);
        gset.gtprefix = reinterpret_cast<const int *>(base + L.gprefix);
        gset.gtprefix32 = gset.gtprefix + (ngroup + 1);
        gset.gcprefix = gset.gtprefix32 + (ngroup + 1);
        gset.ngroup = ngroup;
        gset.s = bsize;
        gset.total_tiles = gt[ngroup];
        gset.total_tiles32 = gt32[ngroup];
        gset.total_chunks = gc[ngroup];
        gset.bc = bc;
        gset.stream = set.stream;
    }

    // operator set-up and right-hand sides
    for (int g = 0; g < nprob; ++g) {
        rc = prepare_operator(probs[g], L.prob[g], base, pc, 0, s,
                              opts->precision == SYLV_PREC_MIXED ? 1 : 2);
        if (rc) return rc;
    }
    HIP_TRY(launch_state_init(set, opts->tol, opts->max_iter, opts->stop_ref, s));
    for (int i = 0; i < ninst; ++i) {
        const Inst &I = tab[i];
        HIP_TRY(launch_rhs(I.W, I.Y, I.A, I.f, I.n_pix, I.bext, I.b, k, s));
    }
    // Fourier-preconditioned runs take about ten iterations or fewer: shorter batches leave
    // fewer early-exit iterations queued past a run's end (het_1024, block-scaled, mixed: 1.39
    // ms with batches of 8, 1.33 ms with 4; float64 runs are insensitive)
    const int chunk = opts->check_every > 0 ? opts->check_every : fourier ? 4 : 8;
    HostFlags *flags = nullptr;   // stays null under the fixed schedule
    if (!fixed && (rc = host_flags(flags))) return rc;
    HIP_TRY(launch_resid(set, k, 0, s));   // r0 = b - G x0, ||b||, ||r0||
    HIP_TRY(launch_resid_fin(set, 0, s));
    const double inner_tol = opts->inner_tol > 0.0 ? opts->inner_tol : 1e-5;
    const double safety = inner_safety();
    auto start_run = [&]() -> int {
        if (block) {
            HIP_TRY(launch_bpinit(gset, k, mixed, s));
            HIP_TRY(launch_bgram(gset, 0, mixed, inner_tol, safety, opts->max_iter, s));
        } else {
            HIP_TRY(launch_pinit(set, k, mixed, inner_tol, safety, opts->max_iter, s));
            if (fourier) {
                const int rc2 = fourier_apply(set, k, mixed, 1, 0, s);
                if (rc2) return rc2;
            }
            HIP_TRY(launch_prereduce_rz(set, s));
        }
        return SYLV_OK;
    };
    auto loop = [&]() -> int {
        return block ? run_block_loop(gset, set, k, mixed, chunk, opts->max_iter, flags, s)
                     : run_cg_loop(set, k, mixed, chunk, opts->max_iter, flags, s);
    };
    if (!mixed) {
        // CG, then the recomputed residual; runs whose recomputed residual misses the threshold
        // are restarted from their current x (residual replacement, at most kMaxRestarts times)
        for (int run = 0; run <= kMaxRestarts; ++run) {
            if ((rc = start_run())) return rc;
            if ((rc = loop())) return rc;
            HIP_TRY(launch_resid(set, k, 1, s));   // true residual of the result
            HIP_TRY(launch_resid_fin(set, 1, s));
            if (fixed) break;   // no restart: a reopened run reports SYLV_NOT_CONVERGED
            if ((rc = post_count(set, 0, flags, 2, s))) return rc;
            int reopened = 0;
            if ((rc = wait_count(flags, 2, reopened))) return rc;
            if (reopened == 0) break;
        }
    } else {
        const int refine_max = opts->refine_max > 0 ? opts->refine_max : 8;
        // One refinement step: float32 inner PCG on the current float64 residual, x += d, new
        // float64 residual.  Steps of finished instances are no-ops on the device, so the next
        // step is queued before the host learns whether this one finished.
        if ((rc = start_run())) return rc;
        for (int o = 0; o < refine_max; ++o) {
            if ((rc = loop())) return rc;
            HIP_TRY(launch_refine_axpy(set, k, s));
            HIP_TRY(launch_resid(set, k, 2, s));   // float64 residual of the new x
            HIP_TRY(launch_resid_fin(set, 2, s));
            if (fixed) {
                if (o + 1 < refine_max && (rc = start_run())) return rc;
                continue;
            }
            if ((rc = post_count(set, 0, flags, 2, s))) return rc;
            if (o + 1 < refine_max && (rc = start_run())) return rc;
            int running = 0;
            if ((rc = wait_count(flags, 2, running))) return rc;
            if (running == 0) break;
        }
    }
    HIP_TRY(launch_stats(set, stats, mixed, s));
    return SYLV_OK;
}


// ---- Lanczos-Sylvester (Section 3.3, Alg. 4 and Alg. 5) ---------------------------------------

struct LzLayout {
    size_t cst, state, H, B, Binv, hist, G, partial, partial2, Yh, Wa0, Wa1, basis, total;
    int nred;
};

bool check_sep(const sylv_sep_problem *p) {
    if (!p) { set_err("null problem"); return false; }
    if (p->k < 1 || p->k > kMaxK) { set_err("k=%d outside [1, %d]", p->k, kMaxK); return false; }
    if (p->f < 1 || p->f > kMaxF) { set_err("f=%d outside [1, %d]", p->f, kMaxF); return false; }
    if (p->ny < 1 || p->nx < 1) { set_err("grid %lld x %lld", (long long)p->ny, (long long)p->nx); return false; }
    if (p->ny * p->nx >= (int64_t)1 << 29) { set_err("n_pix >= 2^29"); return false; }
    if (!(p->kappa >= 0.0) || !isfinite(p->kappa)) { set_err("kappa must be finite and >= 0"); return false; }
    if (!p->tau || !p->A || !p->t || !p->n) { set_err("null parameter pointer"); return false; }
    if (p->boundary != SYLV_BC_PERIODIC && p->boundary != SYLV_BC_FACE) { set_err("boundary %d", p->boundary); return false; }
    return true;
}

bool check_lz_opts(const sylv_lanczos_opts *o) {
    if (!o) { set_err("null opts"); return false; }
    if (!(o->tol > 0.0) || !(o->tol < 1.0)) { set_err("tol must be in (0, 1)"); return false; }
    if (o->max_iter < 1 || o->max_iter > 100000) { set_err("max_iter must be in [1, 100000]"); return false; }
    if (o->check_every < 0) { set_err("negative check_every"); return false; }
    if (o->assembly != SYLV_LZ_KEEP_BASIS && o->assembly != SYLV_LZ_RERUN) { set_err("assembly must be SYLV_LZ_KEEP_BASIS or SYLV_LZ_RERUN"); return false; }
    return true;
}

bool make_lz_layout(const sylv_sep_problem *p, const sylv_lanczos_opts *o, LzLayout &L) {
    const size_t n = (size_t)p->ny * p->nx, k = (size_t)p->k, mi = (size_t)o->max_iter;
    const int nt = lz_tiles((int)p->ny, (int)p->nx, 2), nc = chunks_for((int)n);   // 2 rows: most tiles
    L.nred = std::max(nt, nc);
    const size_t vb = sizeof(double) * k * n;
    if (vb && mi > ((size_t)1 << 62) / vb) { set_err("basis size overflows"); return false; }
    size_t off = 0;
    L.cst = off;     off = align_up(off + sizeof(LzConst));
    L.state = off;   off = align_up(off + sizeof(LzState));
    L.H = off;       off = align_up(off + sizeof(double) * kLzStride * mi);
    L.B = off;       off = align_up(off + sizeof(double) * kLzStride * (mi + 1));
    L.Binv = off;    off = align_up(off + sizeof(double) * kLzStride * (mi + 1));
    L.hist = off;    off = align_up(off + sizeof(double) * mi);
    L.G = off;       off = align_up(off + sizeof(double) * kLzStride * mi);
    L.partial = off; off = align_up(off + sizeof(double) * kLzSlots * L.nred);
    L.partial2 = off; off = align_up(off + sizeof(double) * kLzSlots);
    L.Yh = off;      off = align_up(off + vb);
    L.Wa0 = off;     off = align_up(off + vb);
    L.Wa1 = off;     off = align_up(off + vb);
    L.basis = off;   off = align_up(off + vb * (o->assembly == SYLV_LZ_RERUN ? 2 : mi));
    L.total = off;
    return true;
}

// Eigenvalues and orthonormal eigenvectors of a symmetric m x m matrix (cyclic Jacobi
// rotations), ascending.  a is overwritten; v[i][j] is component i of eigenvector j.
void sym_eig(int m, double a[kMaxK][kMaxK], double w[kMaxK], double v[kMaxK][kMaxK]) {
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) v[i][j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                tot += a[i][j] * a[i][j];
                if (i != j) off += a[i][j] * a[i][j];
            }
        if (off <= 1e-32 * tot) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                if (a[p][q] == 0.0) continue;
                const double th = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
                const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                for (int r = 0; r < m; ++r) {   // columns p, q
                    const double arp = a[r][p], arq = a[r][q];
                    a[r][p] = c * arp - sn * arq;
                    a[r][q] = sn * arp + c * arq;
                }
                for (int r = 0; r < m; ++r) {   // rows p, q
                    const double apr = a[p][r], aqr = a[q][r];
                    a[p][r] = c * apr - sn * aqr;
                    a[q][r] = sn * apr + c * aqr;
                }
                for (int r = 0; r < m; ++r) {
                    const double vrp = v[r][p], vrq = v[r][q];
                    v[r][p] = c * vrp - sn * vrq;
                    v[r][q] = sn * vrp + c * vrq;
                }
            }
    }
    int idx[kMaxK];
    for (int i = 0; i < m; ++i) { idx[i] = i; w[i] = a[i][i]; }
    std::sort(idx, idx + m, [&](int x, int y) { return w[x] < w[y]; });
    double ws[kMaxK], vs[kMaxK][kMaxK];
    for (int j = 0; j < m; ++j) {
        ws[j] = w[idx[j]];
        for (int i = 0; i < m; ++i) vs[i][j] = v[i][idx[j]];
    }
    for (int j = 0; j < m; ++j) {
        w[j] = ws[j];
        for (int i = 0; i < m; ++i) v[i][j] = vs[i][j];
    }
}

// Small dense SPD helpers for the projected equation (host, m <= 8, row-major ld kMaxK).
bool host_chol(int m, const double *a, double *r) {   // a = r^T r, r upper
    for (int i = 0; i < m * kMaxK; ++i) r[i] = 0.0;
    for (int i = 0; i < m; ++i) {
        double d = a[i * kMaxK + i];
        for (int q = 0; q < i; ++q) d -= r[q * kMaxK + i] * r[q * kMaxK + i];
        if (!(d > 0.0)) return false;
        r[i * kMaxK + i] = sqrt(d);
        for (int j = i + 1; j < m; ++j) {
            double v = a[i * kMaxK + j];
            for (int q = 0; q < i; ++q) v -= r[q * kMaxK + i] * r[q * kMaxK + j];
            r[i * kMaxK + j] = v / r[i * kMaxK + i];
        }
    }
    return true;
}
void host_chol_solve(int m, const double *r, const double *b, double *x) {
    double y[kMaxK];
    for (int i = 0; i < m; ++i) {
        double v = b[i];
        for (int q = 0; q < i; ++q) v -= r[q * kMaxK + i] * y[q];
        y[i] = v / r[i * kMaxK + i];
    }
    for (int i = m - 1; i >= 0; --i) {
        double v = y[i];
        for (int q = i + 1; q < m; ++q) v -= r[i * kMaxK + q] * x[q];
        x[i] = v / r[i * kMaxK + i];
    }
}

// Coefficients of the Galerkin approximation M = sum_j V_j G_j after `it` steps: the solution Z
// of the projected equation T Z + Z Lhat = E_1 B_0 (eq. (Sylv-small)).  With Lhat = U R U^-1 the
// columns decouple, Z U = [(T + rho_l I)^-1 E_1 B_0 U e_l]_l (eq. (soln-constr) without forming
// the eigenvectors of T), each a block tridiagonal SPD solve (block elimination, then back
// substitution); Z = (Z U) U^T P^-1.  Returns false if an elimination pivot is not positive.
bool lz_coefficients(int m, int it, const std::vector<double> &H, const std::vector<double> &B,
                     const double U[kMaxK][kMaxK], const double *rho, const double *tau,
                     std::vector<double> &G) {
    const int S = kLzStride;
    std::vector<double> ZU((size_t)it * kMaxK * kMaxK, 0.0);   // [block j][row r][column l]
    std::vector<double> Sc((size_t)it * S), Rc((size_t)it * S), g((size_t)it * kMaxK);
    for (int l = 0; l < m; ++l) {
        // forward elimination: S_1 = H_1 + rho I, g_1 = B_0 U e_l; S_j = H_j + rho I - B_j S_(j-1)^-1 B_j^T,
        // g_j = -B_j S_(j-1)^-1 g_(j-1)
        for (int j = 0; j < it; ++j) {
            double *Sj = &Sc[(size_t)j * S];
            for (int r = 0; r < m; ++r)
                for (int q = 0; q < m; ++q) Sj[r * kMaxK + q] = H[(size_t)j * S + r * kMaxK + q] + (r == q ? rho[l] : 0.0);
            double *gj = &g[(size_t)j * kMaxK];
            if (j == 0) {
                for (int r = 0; r < m; ++r) {
                    double v = 0.0;
                    for (int q = 0; q < m; ++q) v += B[r * kMaxK + q] * U[q][l];
                    gj[r] = v;
                }
            } else {
                const double *Bj = &B[(size_t)j * S];          // B_(j+1) in 1-based names
                const double *Rp = &Rc[(size_t)(j - 1) * S];
                double X[kMaxK][kMaxK];
                for (int q = 0; q < m; ++q) {
                    double bcol[kMaxK], xcol[kMaxK];
                    for (int r = 0; r < m; ++r) bcol[r] = Bj[q * kMaxK + r];
                    host_chol_solve(m, Rp, bcol, xcol);
                    for (int r = 0; r < m; ++r) X[r][q] = xcol[r];
                }
                for (int r = 0; r < m; ++r)
                    for (int q = 0; q < m; ++q) {
                        double v = Sj[r * kMaxK + q];
                        for (int a = 0; a < m; ++a) v -= Bj[r * kMaxK + a] * X[a][q];
                        Sj[r * kMaxK + q] = v;
                    }
                for (int r = 0; r < m; ++r)
                    for (int q = r + 1; q < m; ++q) {
                        const double v = 0.5 * (Sj[r * kMaxK + q] + Sj[q * kMaxK + r]);
                        Sj[r * kMaxK + q] = v;
                        Sj[q * kMaxK + r] = v;
                    }
                double z[kMaxK];
                host_chol_solve(m, Rp, &g[(size_t)(j - 1) * kMaxK], z);
                for (int r = 0; r < m; ++r) {
                    double v = 0.0;
                    for (int q = 0; q < m; ++q) v -= Bj[r * kMaxK + q] * z[q];
                    gj[r] = v;
                }
            }
            if (!host_chol(m, Sj, &Rc[(size_t)j * S])) return false;
        }
        // back substitution: x_it = S_it^-1 g_it, x_j = S_j^-1 (g_j - B_(j+1)^T x_(j+1))
        std::vector<double> x((size_t)it * kMaxK);
        for (int j = it - 1; j >= 0; --j) {
            double rhs[kMaxK];
            for (int r = 0; r < m; ++r) rhs[r] = g[(size_t)j * kMaxK + r];
            if (j + 1 < it) {
                const double *Bn = &B[(size_t)(j + 1) * S];
                for (int r = 0; r < m; ++r)
                    for (int q = 0; q < m; ++q) rhs[r] -= Bn[q * kMaxK + r] * x[(size_t)(j + 1) * kMaxK + q];
            }
            host_chol_solve(m, &Rc[(size_t)j * S], rhs, &x[(size_t)j * kMaxK]);
        }
        for (int j = 0; j < it; ++j)
            for (int r = 0; r < m; ++r) ZU[((size_t)j * kMaxK + r) * kMaxK + l] = x[(size_t)j * kMaxK + r];
    }
    // Z = (Z U) U^T P^-1
    G.assign((size_t)it * S, 0.0);
    for (int j = 0; j < it; ++j)
        for (int r = 0; r < m; ++r)
            for (int c = 0; c < m; ++c) {
                double v = 0.0;
                for (int l = 0; l < m; ++l) v += ZU[((size_t)j * kMaxK + r) * kMaxK + l] * U[c][l];
                G[(size_t)j * S + r * kMaxK + c] = v / tau[c];
            }
    return true;
}

// Small matrices of a separable problem, on the host: the stencil coefficients of D2, t_f A/tau,
// A^T T A and Lemma 2's P^-1/2 A^T T A P^-1/2 = V diag(rho) V^T with U = P^1/2 V (so that
// Lhat = U diag(rho) U^-1).  Copies tau, A and t to the host (synchronises s).
int sep_constants(const sylv_sep_problem *p, LzConst &C, double tau[kMaxK],
                  double Vm[kMaxK][kMaxK], hipStream_t s) {
    const int k = p->k, f = p->f;
    double A[kMaxF * kMaxK], t[kMaxF];
    HIP_TRY(hipMemcpyAsync(tau, p->tau, sizeof(double) * k, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(A, p->A, sizeof(double) * f * k, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(t, p->t, sizeof(double) * f, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int j = 0; j < k; ++j)
        if (!(tau[j] > 0.0) || !isfinite(tau[j])) { set_err("tau[%d] must be finite and > 0", j); return SYLV_E_INVALID; }
    for (int i = 0; i < f; ++i)
        if (!(t[i] > 0.0) || !isfinite(t[i])) { set_err("t[%d] must be finite and > 0", i); return SYLV_E_INVALID; }
    memset(&C, 0, sizeof(C));
    const double ks = p->kappa * p->kappa;
    C.coef[0] = (ks + 4.0) * (ks + 4.0) + 4.0;
    C.coef[1] = -2.0 * (ks + 4.0);
    C.coef[2] = 2.0;
    C.coef[3] = 1.0;
    for (int j = 0; j < k; ++j) {
        C.tau[j] = tau[j];
        for (int i = 0; i < f; ++i) C.tap[j][i] = t[i] * A[i * k + j] / tau[j];
        for (int q = 0; q < k; ++q) {
            double v = 0.0;
            for (int i = 0; i < f; ++i) v += A[i * k + j] * t[i] * A[i * k + q];
            C.ata[j][q] = v;
        }
    }
    double Sm[kMaxK][kMaxK];
    for (int j = 0; j < k; ++j)
        for (int q = 0; q < k; ++q) Sm[j][q] = C.ata[j][q] / sqrt(tau[j] * tau[q]);
    sym_eig(k, Sm, C.rho, Vm);
    if (!(C.rho[0] > 0.0)) { set_err("A^T T A is not positive definite (A must have full column rank)"); return SYLV_E_INVALID; }
    for (int j = 0; j < k; ++j)
        for (int q = 0; q < k; ++q) C.U[j][q] = sqrt(tau[j]) * Vm[j][q];
    C.kappa2 = ks;
    return SYLV_OK;
}

int lanczos_impl(const sylv_sep_problem *p, const double *Y, double *X,
                 const sylv_lanczos_opts *o, sylv_lanczos_stats *stats, void *ws,
                 size_t ws_bytes, hipStream_t s) {
    const int k = p->k, f = p->f;
    LzLayout L;
    if (!make_lz_layout(p, o, L)) return SYLV_E_INVALID;
    int rc = check_ws(ws, ws_bytes, L.total);
    if (rc) return rc;
    if ((rc = refuse_capture(s, "sylv_lanczos_solve"))) return rc;
    char *base = reinterpret_cast<char *>(ws);
    LzConst C;
    double tau[kMaxK], Vm[kMaxK][kMaxK];
    if ((rc = sep_constants(p, C, tau, Vm, s))) return rc;
    C.tol = o->tol;

    LzArgs a;
    memset(&a, 0, sizeof(a));
    a.ny = (int)p->ny; a.nx = (int)p->nx; a.n_pix = (int)(p->ny * p->nx); a.k = k; a.f = f;
    a.tiles_x = (a.nx + kTileX - 1) / kTileX;
    a.bc = p->boundary;
    a.rows = a.bc == SYLV_BC_FACE ? 2 : lz_rows_for(k);
    a.ntiles = lz_tiles(a.ny, a.nx, a.rows);
    a.nchunks = chunks_for(a.n_pix);
    a.nred = L.nred;
    a.c = reinterpret_cast<const LzConst *>(base + L.cst);
    a.st = reinterpret_cast<LzState *>(base + L.state);
    a.H = reinterpret_cast<double *>(base + L.H);
    a.B = reinterpret_cast<double *>(base + L.B);
    a.Binv = reinterpret_cast<double *>(base + L.Binv);
    a.hist = reinterpret_cast<double *>(base + L.hist);
    a.partial = reinterpret_cast<double *>(base + L.partial);
    a.partial2 = reinterpret_cast<double *>(base + L.partial2);
    a.n = p->n;
    a.Y = Y;
    a.Yh = reinterpret_cast<double *>(base + L.Yh);
    a.Wa0 = reinterpret_cast<double *>(base + L.Wa0);
    a.Wa1 = reinterpret_cast<double *>(base + L.Wa1);
    a.basis = reinterpret_cast<double *>(base + L.basis);
    a.X = X;
    a.G = reinterpret_cast<const double *>(base + L.G);
    a.ring = o->assembly == SYLV_LZ_RERUN ? 1 : 0;

    HIP_TRY(hipMemcpyAsync(base + L.cst, &C, sizeof(C), hipMemcpyHostToDevice, s));
    HIP_TRY(lz_launch_init(a, o->max_iter, s));
    HIP_TRY(lz_launch_start(a, s));
    HostFlags *fl = nullptr;
    if ((rc = host_flags(fl))) return rc;
    // Lanczos steps in batches, one batch always queued ahead of the completion check
    const int chunk = o->check_every > 0 ? o->check_every : 8;
    int it = 1;
    auto enqueue_batch = [&](int slot) -> int {
        for (int c = 0; c < chunk && it <= o->max_iter; ++c, ++it) HIP_TRY(lz_launch_step(a, it, s));
        HIP_TRY(lz_launch_flag(a, fl->pinned + slot * HostFlags::kStride, s));
        HIP_TRY(hipEventRecord(fl->ev[slot], s));
        return SYLV_OK;
    };
    if ((rc = enqueue_batch(0))) return rc;
    for (int cur = 0;; cur ^= 1) {
        const bool more = it <= o->max_iter;
        if (more && (rc = enqueue_batch(cur ^ 1))) return rc;
        int running = 0;
        if ((rc = wait_count(fl, cur, running))) return rc;
        if (running == 0 || !more) {
            if (more && (rc = wait_count(fl, cur ^ 1, running))) return rc;
            break;
        }
    }
    // coefficients of the approximation from H and B (host), then assemble and check on the device
    LzState st;
    HIP_TRY(hipMemcpyAsync(&st, base + L.state, sizeof(LzState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int iters = std::max(0, std::min(st.iter, o->max_iter));
    int status = st.done ? st.status : SYLV_NOT_CONVERGED;
    std::vector<double> Hh((size_t)iters * kLzStride), Bh((size_t)(iters + 1) * kLzStride), Gh;
    if (iters > 0) {
        HIP_TRY(hipMemcpyAsync(Hh.data(), base + L.H, sizeof(double) * Hh.size(), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(Bh.data(), base + L.B, sizeof(double) * Bh.size(), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (!lz_coefficients(k, iters, Hh, Bh, C.U, C.rho, tau, Gh)) {
            status = SYLV_BREAKDOWN;
            iters = 0;
        } else {
            HIP_TRY(hipMemcpyAsync(base + L.G, Gh.data(), sizeof(double) * Gh.size(), hipMemcpyHostToDevice, s));
        }
    }
    if (a.ring && iters > 0) {
        // Alg. 5's second pass: the recurrence again from Yhat with the kept H, B blocks, adding
        // V_i G_(i-1) into X step by step; then the residual pass
        for (int i = 1; i <= iters; ++i) HIP_TRY(lz_launch_replay(a, i, s));
        HIP_TRY(lz_launch_resid(a, s));
    } else {
        HIP_TRY(lz_launch_finish(a, iters, s));
    }
    HIP_TRY(hipMemcpyAsync(&st, base + L.state, sizeof(LzState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (stats) {
        stats->status = status;
        stats->iters = iters;
        stats->relres_est = (st.nb0 > 0.0 && st.gamma >= 0.0) ? sqrt(st.gamma) / st.nb0 : (st.nb0 > 0.0 ? NAN : 0.0);
        stats->relres_true = st.bb > 0.0 ? sqrt(st.rr / st.bb) : 0.0;
    }
    return SYLV_OK;
}

// ---- sparse-dense Sylvester solver (Section 3.3.1, Alg. 3) ----------------------------------

// Workspace: the shifted column problems' small parameters, the Lanczos start / residual state
// (F = Yhat is the start block of Alg. 5, and its residual pass checks eq. (Axb)), Xhat, the
// column right-hand sides, then the conjugate-gradient workspace of the column solves.
struct KhLayout {
    size_t par, cst, state, H, B, Binv, hist, G, partial, partial2, Yh, Xh, rhs, solve, total;
    int nred;
};

// The column systems as one-component problems: kappa = the common kappa, tau = 1, A = sqrt of
// the shift, W = n, so that the operator is D2 + shift * N.  Device pointers into `par`
// (par[0] = kappa, par[1] = 1, par[2 + i] = sqrt(shift_i)).
void kh_problems(const sylv_sep_problem *p, const double *par, sylv_problem q[kMaxK]) {
    for (int i = 0; i < p->k; ++i) {
        sylv_problem &c = q[i];
        memset(&c, 0, sizeof(c));
        c.ny = p->ny; c.nx = p->nx; c.k = 1; c.f = 1;
        c.kappa = par; c.tau = par + 1; c.A = par + 2 + i; c.W = p->n;
        c.boundary = p->boundary;
    }
}

bool make_kh_layout(const sylv_sep_problem *p, int decouple, const sylv_pcg_opts *o,
                    KhLayout &L) {
    const size_t n = (size_t)p->ny * p->nx, k = (size_t)p->k;
    L.nred = std::max(lz_tiles((int)p->ny, (int)p->nx, 2), chunks_for((int)n));
    const size_t vb = sizeof(double) * k * n;
    size_t off = 0;
    L.par = off;      off = align_up(off + sizeof(double) * (2 + kMaxK));
    L.cst = off;      off = align_up(off + sizeof(LzConst));
    L.state = off;    off = align_up(off + sizeof(LzState));
    L.H = off;        off = align_up(off + sizeof(double) * kLzStride * 2);
    L.B = off;        off = align_up(off + sizeof(double) * kLzStride * 2);
    L.Binv = off;     off = align_up(off + sizeof(double) * kLzStride * 2);
    L.hist = off;     off = align_up(off + sizeof(double) * 2);
    L.G = off;        off = align_up(off + sizeof(double) * kLzStride * 2);
    L.partial = off;  off = align_up(off + sizeof(double) * kLzSlots * L.nred);
    L.partial2 = off; off = align_up(off + sizeof(double) * kLzSlots);
    L.Yh = off;       off = align_up(off + vb);
    L.Xh = off;       off = align_up(off + vb);
    L.rhs = off;      off = align_up(off + vb);
    L.solve = off;
    // the conjugate-gradient workspace depends only on sizes: lay it out with stand-in pointers
    sylv_problem q[kMaxK];
    kh_problems(p, reinterpret_cast<const double *>(kAlign), q);
    Layout S;
    make_layout(q, decouple ? p->k : 1, 1, true, S, o ? o->precond : SYLV_PC_BLOCK);
    (void)o;
    L.total = align_up(off + S.total);
    return true;
}

// Real Schur form of Lhat from Lemma 2's eigenvectors: U = Wq Ru (QR, Wq orthogonal, Ru upper
// triangular) gives Lhat = U diag(rho) U^-1 = Wq (Ru diag(rho) Ru^-1) Wq^T with
// R = Ru diag(rho) Ru^-1 upper triangular and R_ii = rho_i.  Modified Gram-Schmidt, applied
// twice.  Returns false if U is numerically singular.
bool schur_from_eigvecs(int m, const double U[kMaxK][kMaxK], const double rho[kMaxK],
                        double Wq[kMaxK][kMaxK], double R[kMaxK][kMaxK]) {
    double Ru[kMaxK][kMaxK] = {};
    for (int j = 0; j < m; ++j) {
        double v[kMaxK];
        for (int i = 0; i < m; ++i) v[i] = U[i][j];
        for (int pass = 0; pass < 2; ++pass)
            for (int l = 0; l < j; ++l) {
                double d = 0.0;
                for (int i = 0; i < m; ++i) d += Wq[i][l] * v[i];
                for (int i = 0; i < m; ++i) v[i] -= d * Wq[i][l];
                Ru[l][j] += d;
            }
        double nrm = 0.0;
        for (int i = 0; i < m; ++i) nrm += v[i] * v[i];
        nrm = sqrt(nrm);
        if (!(nrm > 1e-300)) return false;
        Ru[j][j] = nrm;
        for (int i = 0; i < m; ++i) Wq[i][j] = v[i] / nrm;
    }
    // Ru^-1 (upper triangular), then R = Ru diag(rho) Ru^-1
    double Ri[kMaxK][kMaxK] = {};
    for (int j = 0; j < m; ++j) {
        Ri[j][j] = 1.0 / Ru[j][j];
        for (int i = j - 1; i >= 0; --i) {
            double v = 0.0;
            for (int l = i + 1; l <= j; ++l) v += Ru[i][l] * Ri[l][j];
            Ri[i][j] = -v / Ru[i][i];
        }
    }
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            double v = 0.0;
            for (int l = i; l <= j; ++l) v += Ru[i][l] * rho[l] * Ri[l][j];
            R[i][j] = (j >= i) ? v : 0.0;
        }
    return true;
}

int kohler_impl(const sylv_sep_problem *p, const double *Y, double *X, int decouple,
                const sylv_pcg_opts *o, sylv_pcg_stats *stats, double *relres, void *ws,
                size_t ws_bytes, hipStream_t s) {
    const int k = p->k;
    KhLayout L;
    make_kh_layout(p, decouple, o, L);
    int rc = check_ws(ws, ws_bytes, L.total);
    if (rc) return rc;
    if ((rc = refuse_capture(s, "sylv_kohler_solve"))) return rc;
    char *base = reinterpret_cast<char *>(ws);
    LzConst C;
    double tau[kMaxK], Vm[kMaxK][kMaxK];
    if ((rc = sep_constants(p, C, tau, Vm, s))) return rc;
    C.tol = o->tol;

    // the column transform W, the triangular R and the back-transform W^-1
    KhCoef cf;
    KhBack bk;
    memset(&cf, 0, sizeof(cf));
    memset(&bk, 0, sizeof(bk));
    double shift[kMaxK];
    if (decouple) {
        // Lemma 2: Lhat = U diag(rho) U^-1 with U = P^1/2 V, U^-1 = V^T P^-1/2
        for (int i = 0; i < k; ++i) {
            shift[i] = C.rho[i];
            for (int j = 0; j < k; ++j) {
                cf.Fw[j][i] = C.U[j][i];
                bk.T[i][j] = Vm[j][i] / sqrt(tau[j]);
            }
        }
    } else {
        double Wq[kMaxK][kMaxK], R[kMaxK][kMaxK];
        if (!schur_from_eigvecs(k, C.U, C.rho, Wq, R)) {
            set_err("Schur vectors of Lhat are singular");
            return SYLV_E_INVALID;
        }
        for (int i = 0; i < k; ++i) {
            shift[i] = R[i][i];
            for (int j = 0; j < k; ++j) {
                cf.Fw[j][i] = Wq[j][i];
                bk.T[i][j] = Wq[j][i];
                cf.Rc[j][i] = (j < i) ? R[j][i] : 0.0;
            }
        }
    }
    for (int i = 0; i < k; ++i)
        if (!(shift[i] > 0.0)) { set_err("shift %d of the column systems is not positive", i); return SYLV_E_INVALID; }
    double par[2 + kMaxK];
    par[0] = p->kappa;
    par[1] = 1.0;
    for (int i = 0; i < k; ++i) par[2 + i] = sqrt(shift[i]);
    HIP_TRY(launch_upload(base + L.par, par, sizeof(double) * (2 + k), s));
    HIP_TRY(launch_upload(base + L.cst, &C, sizeof(C), s));

    // F = Y^T T A P^-1 into Yh (the Lanczos start kernel), on the Lanczos argument block
    LzArgs a;
    memset(&a, 0, sizeof(a));
    a.ny = (int)p->ny; a.nx = (int)p->nx; a.n_pix = (int)(p->ny * p->nx); a.k = k; a.f = p->f;
    a.tiles_x = (a.nx + kTileX - 1) / kTileX;
    a.bc = p->boundary;
    a.rows = 2;
    a.ntiles = lz_tiles(a.ny, a.nx, a.rows);
    a.nchunks = chunks_for(a.n_pix);
    a.nred = L.nred;
    a.c = reinterpret_cast<const LzConst *>(base + L.cst);
    a.st = reinterpret_cast<LzState *>(base + L.state);
    a.H = reinterpret_cast<double *>(base + L.H);
    a.B = reinterpret_cast<double *>(base + L.B);
    a.Binv = reinterpret_cast<double *>(base + L.Binv);
    a.hist = reinterpret_cast<double *>(base + L.hist);
    a.partial = reinterpret_cast<double *>(base + L.partial);
    a.partial2 = reinterpret_cast<double *>(base + L.partial2);
    a.n = p->n;
    a.Y = Y;
    a.Yh = reinterpret_cast<double *>(base + L.Yh);
    a.X = X;
    a.G = reinterpret_cast<const double *>(base + L.G);
    HIP_TRY(lz_launch_init(a, 1, s));
    HIP_TRY(lz_launch_start(a, s));

    const size_t n = (size_t)a.n_pix;
    double *Xh = reinterpret_cast<double *>(base + L.Xh);
    double *rhs = reinterpret_cast<double *>(base + L.rhs);
    sylv_problem q[kMaxK];
    kh_problems(p, reinterpret_cast<const double *>(base + L.par), q);
    void *sws = base + L.solve;
    const size_t sbytes = ws_bytes - L.solve;
    HIP_TRY(kh_launch_zero(Xh, (long)(k * n), s));
    if (decouple) {
        // every column at once: k independent one-component problems in one batched solve
        HIP_TRY(kh_launch_rhs(a.Yh, p->n, Xh, cf, k, 0, k, a.n_pix, rhs, s));
        Layout S;
        if ((rc = solve_impl(q, k, 1, nullptr, rhs, Xh, o, stats, sws, sbytes, s, S))) return rc;
    } else {
        // Alg. 3: column i after columns 0 .. i-1
        for (int i = 0; i < k; ++i) {
            HIP_TRY(kh_launch_rhs(a.Yh, p->n, Xh, cf, k, i, i + 1, a.n_pix, rhs, s));
            Layout S;
            if ((rc = solve_impl(&q[i], 1, 1, nullptr, rhs + i * n, Xh + i * n, o, stats + i,
                                 sws, sbytes, s, S)))
                return rc;
        }
    }
    HIP_TRY(kh_launch_back(Xh, bk, k, a.n_pix, X, s));
    HIP_TRY(lz_launch_resid(a, s));
    if (relres) HIP_TRY(kh_launch_relres(a.st, relres, s));
    return SYLV_OK;
}

// ---- solves without allocation: a static per-device scratch array as the workspace ---------

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Device address of the current device's scratch array, looked up once per device.
int scratch_address(void **out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_err("device index %d outside [0, %d)", dev, kMaxDevices);
        return SYLV_E_INVALID;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr || ((uintptr_t)ptr & (kAlign - 1)) != 0) {
            set_err("scratch array of device %d at an unaligned address", dev);
            return SYLV_E_HIP;
        }
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return SYLV_OK;
}

int solve_noalloc_impl(const sylv_problem *probs, int nprob, int nrhs, const double *Y,
                       const double *Bextra, double *X, const sylv_pcg_opts *opts,
                       sylv_pcg_stats *stats, hipStream_t s) {
    if (!probs || nprob < 1 || nrhs < 1) { set_err("null problems or nprob, nrhs < 1"); return SYLV_E_INVALID; }
    if (!opts) { set_err("null opts"); return SYLV_E_INVALID; }
    if (opts->schedule != SYLV_SCHED_FIXED) {
        set_err("the no-allocation solve runs the fixed schedule only (the adaptive schedule "
                "needs pinned host memory for its convergence checks)");
        return SYLV_E_INVALID;
    }
    for (int g = 0; g < nprob; ++g)
        if (!check_problem(&probs[g], g)) return SYLV_E_INVALID;
    Layout L;
    make_layout(probs, nprob, nrhs, true, L, opts->precond);
    if (L.total > SYLV_NOALLOC_SCRATCH_BYTES) {
        set_err("the batch needs %zu bytes of workspace; the no-allocation solve has %zu "
                "(use sylv_pcg_solve with a caller workspace)",
                L.total, (size_t)SYLV_NOALLOC_SCRATCH_BYTES);
        return SYLV_E_WORKSPACE;
    }
    void *ws = nullptr;
    int rc = scratch_address(&ws);
    if (rc) return rc;
    Layout L2;
    return solve_impl(probs, nprob, nrhs, Y, Bextra, X, opts, stats, ws,
                      SYLV_NOALLOC_SCRATCH_BYTES, s, L2);
}

// ---- autotuning (configuration choice by timing whole solves) --------------------------------

struct EventPair {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~EventPair() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

// One solve from x0 = 0 under `o`, timed with events around the whole call; `ok` when every
// right-hand side converged.
int timed_solve(const sylv_problem *probs, int nprob, int nrhs, const double *Y,
                const double *Bextra, double *X, size_t xbytes, const sylv_pcg_opts &o,
                sylv_pcg_stats *stats, void *ws, size_t ws_bytes, hipStream_t s, EventPair &ev,
                double &ms, bool &ok) {
    HIP_TRY(hipMemsetAsync(X, 0, xbytes, s));
    HIP_TRY(hipEventRecord(ev.e0, s));
    Layout L;
    const int rc = solve_impl(probs, nprob, nrhs, Y, Bextra, X, &o, stats, ws, ws_bytes, s, L);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(ev.e1, s));
    HIP_TRY(hipEventSynchronize(ev.e1));
    float t = 0.0f;
    HIP_TRY(hipEventElapsedTime(&t, ev.e0, ev.e1));
    ms = t;
    std::vector<sylv_pcg_stats> h((size_t)nprob * nrhs);
    HIP_TRY(hipMemcpy(h.data(), stats, sizeof(sylv_pcg_stats) * h.size(), hipMemcpyDeviceToHost));
    ok = true;
    for (const sylv_pcg_stats &st : h) ok = ok && st.status == SYLV_OK;
    return SYLV_OK;
}

int autotune_impl(const sylv_problem *probs, int nprob, int nrhs, const double *Y,
                  const double *Bextra, double *X, const sylv_pcg_opts *opts,
                  sylv_pcg_stats *stats, sylv_tune_result *out, void *ws, size_t ws_bytes,
                  hipStream_t s) {
    if (!probs || nprob < 1 || nrhs < 1) { set_err("null problems or nprob, nrhs < 1"); return SYLV_E_INVALID; }
    if (!out || !X || !stats) { set_err("null X, stats or out"); return SYLV_E_INVALID; }
    int rc = check_opts(opts);
    if (rc) return rc;
    for (int g = 0; g < nprob; ++g)
        if (!check_problem(&probs[g], g)) return SYLV_E_INVALID;
    if ((rc = refuse_capture(s, "sylv_autotune"))) return rc;
    size_t xbytes = 0;
    for (int g = 0; g < nprob; ++g)
        xbytes += sizeof(double) * (size_t)nrhs * probs[g].k * probs[g].ny * probs[g].nx;
    EventPair ev;
    HIP_TRY(hipEventCreate(&ev.e0));
    HIP_TRY(hipEventCreate(&ev.e1));

    // candidates: independent CG at each distinct effective tiling, block CG at each block size
    struct Cand { int block, bsize, rows; };
    std::vector<Cand> cands;
    const int k = probs[0].k;
    const bool face = probs[0].boundary == SYLV_BC_FACE;
    std::vector<std::pair<int, int>> tilings;
    for (int rows : {2, 4, 8}) {
        const std::pair<int, int> t = face ? std::make_pair(2, 2)
                                           : std::make_pair(apply_rows_for(k, SYLV_F64, rows),
                                                            apply_rows_for(k, SYLV_F32, rows));
        if (std::find(tilings.begin(), tilings.end(), t) != tilings.end()) continue;
        tilings.push_back(t);
        cands.push_back({0, 0, rows});
    }
    for (int bs : {2, 4, 8})
        if (block_size_ok(nrhs, bs)) cands.push_back({1, bs, 0});

    // the configuration as given first (it also warms up the allocator and the code paths)
    double ms_given = -1.0, best = -1.0;
    bool ok = false;
    Cand pick{0, 0, 0};
    {
        double t0 = 0.0, t1 = 0.0;
        if ((rc = timed_solve(probs, nprob, nrhs, Y, Bextra, X, xbytes, *opts, stats, ws, ws_bytes,
                              s, ev, t0, ok)))
            return rc;
        if ((rc = timed_solve(probs, nprob, nrhs, Y, Bextra, X, xbytes, *opts, stats, ws, ws_bytes,
                              s, ev, t1, ok)))
            return rc;
        ms_given = ok ? std::min(t0, t1) : -1.0;
    }
    for (const Cand &c : cands) {
        sylv_pcg_opts o = *opts;
        o.block = c.block;
        o.block_size = c.bsize;
        o.apply_rows = c.rows;
        double t = 1e300;
        bool all_ok = true;
        for (int rep = 0; rep < 2; ++rep) {
            double ms = 0.0;
            if ((rc = timed_solve(probs, nprob, nrhs, Y, Bextra, X, xbytes, o, stats, ws, ws_bytes,
                                  s, ev, ms, ok)))
                return rc;
            all_ok = all_ok && ok;
            t = std::min(t, ms);
        }
        if (all_ok && (best < 0.0 || t < best)) {
            best = t;
            pick = c;
        }
    }
    out->block = pick.block;
    out->block_size = pick.bsize;
    out->apply_rows = pick.rows;
    out->candidates = (int32_t)cands.size();
    out->ms = best;
    out->ms_given = ms_given;
    if (best < 0.0) {
        set_err("no candidate configuration converged for every right-hand side");
        return SYLV_NOT_CONVERGED;
    }
    return SYLV_OK;
}

}  // namespace

extern "C" {

size_t sylv_workspace_bytes(const sylv_problem *probs, int32_t nprob, int32_t nrhs,
                            const sylv_pcg_opts *opts) {
    if (!probs || nprob < 1 || nrhs < 1) return 0;
    for (int g = 0; g < nprob; ++g)
        if (!check_problem(&probs[g], g)) return 0;
    Layout L;
    if (!opts) {
        if (nprob != 1) return 0;
        make_layout(probs, 1, 1, false, L);
    } else {
        make_layout(probs, nprob, nrhs, true, L, opts->precond);
    }
    return L.total;
}

int sylv_prepare(const sylv_problem *prob, int32_t precond, void *ws, size_t ws_bytes,
                 void *stream) {
    if (!check_problem(prob, 0)) return SYLV_E_INVALID;
    if (precond < SYLV_PC_NONE || precond > SYLV_PC_FOURIER_BLOCK) { set_err("bad precond"); return SYLV_E_INVALID; }
    if (is_fourier(precond) && !fp_grid(*prob)) {
        set_err("the Fourier preconditioner needs grid sides that are powers of two in [4, 4096]");
        return SYLV_E_INVALID;
    }
    Layout L;
    make_layout(prob, 1, 1, false, L);
    int rc = check_ws(ws, ws_bytes, L.total);
    if (rc) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *base = reinterpret_cast<char *>(ws);
    rc = prepare_operator(*prob, L.prob[0], base, precond, 1, s);
    if (rc) return rc;
    Inst I = operator_inst(*prob, L.prob[0], base, precond);
    I.ntiles = 0;
    I.nchunks = chunks_for(I.n_pix);
    I.nrr = I.nchunks;
    HIP_TRY(launch_upload(base + L.table, &I, sizeof(Inst), s));
    return SYLV_OK;
}

int sylv_apply(const sylv_problem *prob, int32_t dtype, const void *X, void *Y, int32_t nrhs,
               int32_t prepared, void *ws, size_t ws_bytes, void *stream) {
    if (!check_problem(prob, 0)) return SYLV_E_INVALID;
    if (dtype != SYLV_F64 && dtype != SYLV_F32) { set_err("bad dtype"); return SYLV_E_INVALID; }
    if (!X || !Y || nrhs < 1) { set_err("null X/Y or nrhs < 1"); return SYLV_E_INVALID; }
    if (X == Y) { set_err("X and Y must not overlap"); return SYLV_E_INVALID; }
    Layout L;
    make_layout(prob, 1, 1, false, L);
    int rc = check_ws(ws, ws_bytes, L.total);
    if (rc) return rc;
    if (!prepared) {
        rc = sylv_prepare(prob, SYLV_PC_NONE, ws, ws_bytes, stream);
        if (rc) return rc;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *base = reinterpret_cast<char *>(ws);
    const double es = dtype == SYLV_F64 ? 8.0 : 4.0, n = (double)prob->ny * prob->nx;
    const int streamed = stream_policy(n * (2.0 * prob->k * nrhs + packed_size(prob->k)) * es);
    HIP_TRY(launch_apply_plain(reinterpret_cast<const Inst *>(base + L.table), prob->k, dtype,
                               apply_rows_for(prob->k, dtype, apply_rows_request()),
                               prob->boundary, streamed, (int)prob->ny, (int)prob->nx, nrhs, X,
                               Y, s));
    return SYLV_OK;
}

int sylv_precond(const sylv_problem *prob, int32_t dtype, int32_t precond, const void *R,
                 void *Z, int32_t nrhs, int32_t prepared, void *ws, size_t ws_bytes,
                 void *stream) {
    if (!check_problem(prob, 0)) return SYLV_E_INVALID;
    if (dtype != SYLV_F64 && dtype != SYLV_F32) { set_err("bad dtype"); return SYLV_E_INVALID; }
    if (precond < SYLV_PC_NONE || precond > SYLV_PC_FOURIER_BLOCK) { set_err("bad precond"); return SYLV_E_INVALID; }
    if (is_fourier(precond)) {
        char why[200];
        if (!fp_supported((int)prob->ny, (int)prob->nx, prob->k, dtype, why, sizeof(why))) { set_err("%s", why); return SYLV_E_INVALID; }
        if (precond == SYLV_PC_FOURIER_BLOCK &&
            !fp_rows_per_block_blk((int)prob->nx, (int)prob->ny, prob->k, dtype)) {
            set_err("the block-scaled Fourier preconditioner's row passes hold every component of "
                    "two grid rows: k * nx = %d > 8192", prob->k * (int)prob->nx);
            return SYLV_E_INVALID;
        }
    }
    if (!R || !Z || nrhs < 1) { set_err("null R/Z or nrhs < 1"); return SYLV_E_INVALID; }
    Layout L;
    make_layout(prob, 1, 1, false, L);
    int rc = check_ws(ws, ws_bytes, L.total);
    if (rc) return rc;
    if (!prepared) {
        rc = sylv_prepare(prob, precond, ws, ws_bytes, stream);
        if (rc) return rc;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *base = reinterpret_cast<char *>(ws);
    if (is_fourier(precond)) {
        // one instance without run state: its spectrum in the stand-alone region
        Inst I = operator_inst(*prob, L.prob[0], base, precond);
        I.nchunks = chunks_for(I.n_pix);
        I.nrr = I.nchunks;
        I.fs = reinterpret_cast<double *>(base + L.fs1);
        I.fsym = reinterpret_cast<const double *>(base + L.prob[0].fsym);
        I.lognx = __builtin_ctz((unsigned)I.nx);
        I.logny = __builtin_ctz((unsigned)I.ny);
        const int k = prob->k;
        const bool blk = precond == SYLV_PC_FOURIER_BLOCK;
        I.frb = blk ? fp_rows_per_block_blk(I.nx, I.ny, k, dtype)
                    : fp_rows_per_block(I.nx, I.ny, dtype);
        I.nfft = I.nx / 2;
        I.partial = nullptr;
        int pre[kPrefixArrays * 2] = {0, 0, 0, 0, 0, 0, 0, blk ? I.ny / I.frb : k * (I.ny / I.frb),
                                      0, I.nfft};
        HIP_TRY(launch_upload(base + L.table, &I, sizeof(Inst), s));
        HIP_TRY(launch_upload(base + L.tprefix, pre, sizeof(pre), s));
        InstSet set;
        memset(&set, 0, sizeof(set));
        set.table = reinterpret_cast<const Inst *>(base + L.table);
        set.tprefix = reinterpret_cast<const int *>(base + L.tprefix);
        set.tprefix32 = set.tprefix + 2;
        set.cprefix = set.tprefix32 + 2;
        set.fprefa = set.cprefix + 2;
        set.fprefb = set.fprefa + 2;
        set.ninst = 1;
        set.total_fa = pre[7];
        set.total_fb = pre[9];
        set.fourier = 1;
        set.fp_scaled = precond == SYLV_PC_FOURIER_DIAG ? 1 : 0;
        set.fp_block = blk ? 1 : 0;
        const bool rg = blk && fp_blk_global_twiddles(I.nx, k, dtype);
        set.fp_blk_gtw = rg ? fp_radix_bit(I.lognx) : 0;
        set.fp_lds_rows = blk ? fp_lds_bytes_blk(I.nx, k, dtype, rg)
                              : fp_lds_bytes(0, I.nx, I.frb, dtype);
        set.fp_lds_cols = fp_lds_bytes(1, I.ny, k, dtype);
        set.fp_cols_gtw = fp_cols_global_twiddles(I.ny, k, dtype) ? fp_radix_bit(I.logny) : 0;
        set.fp_rmask_x = fp_radix_bit(I.lognx);
        set.fp_rmask_y = fp_radix_bit(I.logny);
        set.bc = prob->boundary;
        const size_t es = dtype == SYLV_F64 ? 8 : 4, plane = (size_t)k * I.n_pix * es;
        for (int r = 0; r < nrhs; ++r)
            HIP_TRY(launch_fp_apply(set, k, dtype == SYLV_F32, -1,
                                    static_cast<const char *>(R) + r * plane,
                                    static_cast<char *>(Z) + r * plane, 0, 0, s));
        return SYLV_OK;
    }
    HIP_TRY(launch_precond_plain(reinterpret_cast<const Inst *>(base + L.table), prob->k, dtype,
                                 (int)(prob->ny * prob->nx), nrhs, R, Z, s));
    return SYLV_OK;
}

int sylv_rhs(const sylv_problem *prob, const double *Y, double *Bout, void *stream) {
    if (!check_problem(prob, 0)) return SYLV_E_INVALID;
    if (!Y || !Bout) { set_err("null Y or Bout"); return SYLV_E_INVALID; }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(launch_rhs(prob->W, Y, prob->A, prob->f, (int)(prob->ny * prob->nx), nullptr, Bout,
                       prob->k, s));
    return SYLV_OK;
}

int sylv_po_perturb(const sylv_problem *prob, const double *xi, const double *zeta, double *eta,
                    int32_t nrhs, void *stream) {
    if (!check_problem(prob, 0)) return SYLV_E_INVALID;
    if (!xi || !zeta || !eta || nrhs < 1) { set_err("null xi/zeta/eta or nrhs < 1"); return SYLV_E_INVALID; }
    if (nrhs > 65535) { set_err("nrhs > 65535"); return SYLV_E_INVALID; }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(launch_po(prob->kappa, prob->tau, prob->A, prob->W, xi, zeta, eta, prob->k, prob->f,
                      (int)prob->ny, (int)prob->nx, prob->boundary, nrhs, s));
    return SYLV_OK;
}

int sylv_pcg_solve(const sylv_problem *probs, int32_t nprob, int32_t nrhs, const double *Y,
                   const double *Bextra, double *X, const sylv_pcg_opts *opts,
                   sylv_pcg_stats *stats, void *ws, size_t ws_bytes, void *stream) {
    if (!probs) { set_err("null problems"); return SYLV_E_INVALID; }
    Layout L;
    return solve_impl(probs, nprob, nrhs, Y, Bextra, X, opts, stats, ws, ws_bytes,
                      reinterpret_cast<hipStream_t>(stream), L);
}

size_t sylv_kohler_workspace_bytes(const sylv_sep_problem *prob, int32_t decouple,
                                   const sylv_pcg_opts *opts) {
    if (!check_sep(prob) || check_opts(opts) || (decouple != 0 && decouple != 1)) return 0;
    KhLayout L;
    make_kh_layout(prob, decouple, opts, L);
    return L.total;
}

int sylv_kohler_solve(const sylv_sep_problem *prob, const double *Y, double *X,
                      int32_t decouple, const sylv_pcg_opts *opts, sylv_pcg_stats *stats,
                      double *relres_true, void *ws, size_t ws_bytes, void *stream) {
    if (!check_sep(prob)) return SYLV_E_INVALID;
    int rc = check_opts(opts);
    if (rc) return rc;
    if (decouple != 0 && decouple != 1) { set_err("decouple must be 0 or 1"); return SYLV_E_INVALID; }
    if (!Y || !X || !stats) { set_err("null Y, X or stats"); return SYLV_E_INVALID; }
    return kohler_impl(prob, Y, X, decouple, opts, stats, relres_true, ws, ws_bytes,
                       reinterpret_cast<hipStream_t>(stream));
}

int sylv_pcg_solve_noalloc(const sylv_problem *probs, int32_t nprob, int32_t nrhs,
                           const double *Y, const double *Bextra, double *X,
                           const sylv_pcg_opts *opts, sylv_pcg_stats *stats, void *stream) {
    return solve_noalloc_impl(probs, nprob, nrhs, Y, Bextra, X, opts, stats,
                              reinterpret_cast<hipStream_t>(stream));
}

int sylv_pcg_backward(const sylv_problem *prob, const double *Y, const double *Xstar,
                      const double *Gbar, double *Lambda, double *dkappa, double *dtau,
                      double *dA, double *dW, double *dY, const sylv_pcg_opts *opts,
                      sylv_pcg_stats *stats, void *ws, size_t ws_bytes, void *stream) {
    if (!check_problem(prob, 0)) return SYLV_E_INVALID;
    if (!Y || !Xstar || !Gbar || !Lambda) { set_err("null Y/Xstar/Gbar/Lambda"); return SYLV_E_INVALID; }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Layout L;
    int rc = solve_impl(prob, 1, 1, nullptr, Gbar, Lambda, opts, stats, ws, ws_bytes, s, L);
    if (rc) return rc;
    char *base = reinterpret_cast<char *>(ws);
    HIP_TRY(launch_grad(reinterpret_cast<const double *>(base + L.prob[0].coef), prob->A,
                        prob->W, Y, Xstar, Lambda, prob->k, prob->f, (int)prob->ny,
                        (int)prob->nx, prob->boundary, dkappa, dtau, dA, dW, dY,
                        reinterpret_cast<double *>(base + L.gpartial), s));
    return SYLV_OK;
}

int sylv_autotune(const sylv_problem *probs, int32_t nprob, int32_t nrhs, const double *Y,
                  const double *Bextra, double *X, const sylv_pcg_opts *opts,
                  sylv_pcg_stats *stats, sylv_tune_result *out, void *ws, size_t ws_bytes,
                  void *stream) {
    return autotune_impl(probs, nprob, nrhs, Y, Bextra, X, opts, stats, out, ws, ws_bytes,
                         reinterpret_cast<hipStream_t>(stream));
}

size_t sylv_lanczos_workspace_bytes(const sylv_sep_problem *prob, const sylv_lanczos_opts *opts) {
    if (!check_sep(prob) || !check_lz_opts(opts)) return 0;
    LzLayout L;
    if (!make_lz_layout(prob, opts, L)) return 0;
    return L.total;
}

int sylv_lanczos_solve(const sylv_sep_problem *prob, const double *Y, double *X,
                       const sylv_lanczos_opts *opts, sylv_lanczos_stats *stats, void *ws,
                       size_t ws_bytes, void *stream) {
    if (!check_sep(prob) || !check_lz_opts(opts)) return SYLV_E_INVALID;
    if (!Y || !X) { set_err("null Y or X"); return SYLV_E_INVALID; }
    return lanczos_impl(prob, Y, X, opts, stats, ws, ws_bytes, reinterpret_cast<hipStream_t>(stream));
}

const char *sylv_status_string(int code) {
    switch (code) {
        case SYLV_OK: return "ok";
        case SYLV_NOT_CONVERGED: return "not converged";
        case SYLV_BREAKDOWN: return "breakdown (operator or preconditioner not positive definite)";
        case SYLV_NONFINITE: return "non-finite value";
        case SYLV_STAGNATED: return "refinement stagnated";
        case SYLV_BAD_INPUT: return "invalid input values (n_p not a positive finite number)";
        case SYLV_E_INVALID: return "invalid argument";
        case SYLV_E_WORKSPACE: return "workspace too small";
        case SYLV_E_HIP: return "HIP runtime error";
        default: return "unknown code";
    }
}

const char *sylv_last_error(void) { return g_err; }

}  // extern "C"
