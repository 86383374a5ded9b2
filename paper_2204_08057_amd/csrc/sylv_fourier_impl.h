// Fourier preconditioner of the CG solver on periodic grids whose sides are powers of two:
//
//     z = (Q + I (x) Mbar)^-1 r,   Q = blockdiag_j tau_j (kappa_j^2 I - Lap)^2,
//     Mbar = sum_f mean_p(W[f, p]) a_f a_f^T,
//
// i.e. the operator of the system (eq. (Axb)) with the per-pixel noise weights replaced by their
// mean over the pixels.  Every prior block is a polynomial in the periodic Laplacian, so the 2-D
// DFT diagonalises Q: the mode with -Lap eigenvalue lam = 4 - 2 cos(2 pi u / nx) - 2 cos(2 pi v /
// ny) gets diag_j tau_j (kappa_j^2 + lam)^2, and one k x k symmetric positive definite block per
// mode remains.  A preconditioner only has to be fixed and SPD; this one is exact when the weights
// do not depend on the pixel, and otherwise removes the stencil prior's spread of scales that
// block-Jacobi leaves to CG.
//
// Three passes over the grid per application (r real [k][ny][nx] -> z real [k][ny][nx]):
//   A  forward FFT of every row (length nx), stored transposed as the half spectrum
//      S[j][c][y], c in [0, nx/2] (the rows of S are the columns of the grid's spectrum);
//   B  per column c of the half spectrum, all k components at once: forward FFT along y (length
//      ny), the k x k solve of every mode (its block formed and factored in registers), the
//      <r, z> partial by Parseval's identity, inverse FFT along y, back into S.  The columns
//      c = 0 and c = nx/2 are real (sums of real rows with weights +-1) and travel together as
//      one complex column, so that the pass has nx/2 workgroups;
//   C  per row: the full row spectrum from the half (Hermitian symmetry of a real row), inverse
//      FFT (length nx), the real part scaled by 1 / (nx ny) into z.
// Every FFT is a Stockham transform in LDS whose butterflies are DFTs of 16 points (8, 4 or 2 for
// the last stage) in registers; the first stage reads global memory and the last writes it where
// the layout allows.  Its twiddles come from per-stage tables made once at set-up (with the
// per-mode Laplacian eigenvalues) and copied into LDS, so a butterfly reads each twiddle once,
// from consecutive entries.  The row passes transform two real rows as one complex row.
// T = float for the inner runs of the mixed path, double for float64 runs.
//
// Face grids (zero-flux edges, the faces of the sky grid) take the same three passes with
// cosine transforms (DCT-II, which diagonalises the path Laplacian with Neumann ends: lam = 4 -
// 2 cos(pi u / nx) - 2 cos(pi v / ny)) in place of Fourier transforms, each computed by an FFT of
// the reordered sequence; all coefficients are real, so pass B takes two coefficient columns as
// one complex column.
//
// This header holds the kernels of the three passes and the launcher template; every
// (precision, grid type) pair is instantiated in a translation unit of its own
// (sylv_fourier_{f32,f64}_{periodic,face}.hip) so that they compile in parallel.  The set-up
// kernels and the host queries are in sylv_fourier.hip.
#pragma once

#include "sylv_device.h"

#include <stdio.h>

#include <algorithm>
#include <type_traits>

namespace sylv {
namespace {

using namespace dev;

template <typename T>
struct Cx {
    T x, y;
};
template <typename T>
__device__ __forceinline__ Cx<T> cadd(Cx<T> a, Cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ Cx<T> csub(Cx<T> a, Cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// LDS index with one padding slot per 32 entries (breaks the power-of-two strides of the
// Stockham stores across banks).
__device__ __forceinline__ int lpad(int i) { return i + (i >> 5); }
__host__ __device__ constexpr int lds_entries(int n) { return n + (n >> 5) + 1; }

// Workgroup shape of the three passes: 512 threads (8 wavefronts), and at most kFftCap complex
// entries of transform data per workgroup (64 KB in float32, 128 KB in float64; the device
// allows 160 KB of LDS per workgroup).  A thread holds at most kRegPts complex values between two
// LDS exchanges.
constexpr int kFT = 512;
constexpr int kRegPts = 16;
constexpr int kFftCap = kFT * kRegPts;
constexpr size_t kMaxLds = 163840;
static_assert(kFT == 8 * 64, "fp_block_sum sums eight wavefronts");

// ---- set-up tables (per problem, after the symbol block) --------------------------------------
// In doubles from the start of the problem's Fourier region:
//   [0, kSymDoubles)   Mbar [kMaxK][kMaxK], kappa_j^2 [kMaxK], tau_j [kMaxK]
//   lamx[u], u < nx, and lamy[v], v < ny: the Laplacian eigenvalue of each side's modes,
//   2 - 2 cos(2 pi u / nx) on periodic grids, 2 - 2 cos(pi u / nx) on face grids (cosines)
//   Stockham twiddles for n = nx and n = ny, complex double, then complex float (n - 1 entries
//   each, padded to n): stage s (radix R, ns = product of the earlier radices) holds
//   W_(ns R)^(r kk) at [off_s + (r - 1) ns + kk], r in [1, R), kk in [0, ns)
//   face grids: exp(-i pi u / 2n), u < n, for n = nx and n = ny, complex double then float (the
//   cosine transform's twiddles)
constexpr int kSymDoubles = kMaxK * kMaxK + 2 * kMaxK;
__host__ __device__ constexpr size_t round4(size_t v) { return (v + 3) & ~(size_t)3; }
struct FpTabs {
    size_t lamx, lamy, twx64, twy64, twx32, twy32, ctx64, cty64, ctx32, cty32, total;   // doubles
};
__host__ __device__ inline FpTabs fp_tabs(int nx, int ny) {
    FpTabs t;
    size_t o = round4(kSymDoubles);
    t.lamx = o;  o = round4(o + nx);
    t.lamy = o;  o = round4(o + ny);
    t.twx64 = o; o = round4(o + 2 * (size_t)nx);
    t.twy64 = o; o = round4(o + 2 * (size_t)ny);
    t.twx32 = o; o = round4(o + (size_t)nx);
    t.twy32 = o; o = round4(o + (size_t)ny);
    t.ctx64 = o; o = round4(o + 2 * (size_t)nx);
    t.cty64 = o; o = round4(o + 2 * (size_t)ny);
    t.ctx32 = o; o = round4(o + (size_t)nx);
    t.cty32 = o; o = round4(o + (size_t)ny);
    t.total = o;
    return t;
}
template <typename T>
__device__ __forceinline__ const Cx<T> *stage_table(const double *base, const FpTabs &t, bool x) {
    if (sizeof(T) == 8) return reinterpret_cast<const Cx<T> *>(base + (x ? t.twx64 : t.twy64));
    return reinterpret_cast<const Cx<T> *>(base + (x ? t.twx32 : t.twy32));
}

template <typename T>
__device__ __forceinline__ const Cx<T> *cos_table(const double *base, const FpTabs &t, bool x) {
    if (sizeof(T) == 8) return reinterpret_cast<const Cx<T> *>(base + (x ? t.ctx64 : t.cty64));
    return reinterpret_cast<const Cx<T> *>(base + (x ? t.ctx32 : t.cty32));
}

// The cosine transform (DCT-II, X[u] = sum_i x[i] cos(pi u (2i + 1) / 2n)) of a real sequence
// comes from one complex FFT of the reordered sequence v[m] = x[cos_src(m)] (even samples
// forward, odd samples backward): X[u] = Re(exp(-i pi u / 2n) V[u]).  The inverse forms
// V[u] = exp(i pi u / 2n) (X[u] - i X[n - u]) (X[n] = 0), transforms back and undoes the order.
__device__ __forceinline__ int cos_src(int m, int n) {
    return m < (n >> 1) ? 2 * m : 2 * (n - 1 - m) + 1;
}

// log2 of the radix of the stage that starts at log2-position lg of a length-2^logn transform:
// radix-16 stages, then one of radix fft_last_radix(logn).
__host__ __device__ constexpr int stage_log_radix(int logn, int lg) {
    return logn - lg >= 4 ? 4 : logn - lg;
}
__host__ __device__ constexpr int fft_last_radix(int logn) {
    return (logn & 3) == 0 ? 16 : 1 << (logn & 3);
}
// Kernel classes of a transform length: the lengths of the 1024^2 and 2048^2 grids get kernels
// of their own (class 100 + log2 n: every stage size, stride and LDS offset a compile-time
// constant), every other length the kernel of its final radix (class 2, 4, 8 or 16).
__host__ __device__ constexpr int fft_class(int logn) {
    return (logn == 10 || logn == 11) ? 100 + logn : fft_last_radix(logn);
}
__host__ __device__ constexpr int cls_fr(int cls) { return cls >= 100 ? fft_last_radix(cls - 100) : cls; }
__host__ __device__ constexpr int cls_ln(int cls) { return cls >= 100 ? cls - 100 : 0; }
// The bit of a class in the set masks (the same as fp_radix_bit of its lengths).
__host__ __device__ constexpr int cls_bit(int cls) { return cls >= 100 ? 16 << (cls - 110) : cls / 2; }

// ---- DFTs of R = 2, 4, 8, 16 points in registers, natural order in and out ----------------
// Forward: X[k] = sum_j x[j] exp(-2 pi i j k / R); INV = 1 uses exp(+2 pi i j k / R).
template <typename T, int INV>
__device__ __forceinline__ Cx<T> mul_mi(Cx<T> a) {   // a * (-i) forward, a * (+i) inverse
    return INV ? Cx<T>{-a.y, a.x} : Cx<T>{a.y, -a.x};
}
template <typename T, int INV>
__device__ __forceinline__ Cx<T> mul_w8(Cx<T> a, int e) {   // a * W_8^e, e in 0..3
    const T h = (T)0.70710678118654752440;                  // cos(pi/4)
    switch (e) {
        case 0: return a;
        case 1: return INV ? Cx<T>{h * (a.x - a.y), h * (a.x + a.y)}
                           : Cx<T>{h * (a.x + a.y), h * (a.y - a.x)};
        case 2: return mul_mi<T, INV>(a);
        default: return INV ? Cx<T>{-h * (a.x + a.y), h * (a.x - a.y)}
                            : Cx<T>{h * (a.y - a.x), -h * (a.x + a.y)};
    }
}
template <typename T, int INV>
__device__ __forceinline__ void dft4(Cx<T> &a0, Cx<T> &a1, Cx<T> &a2, Cx<T> &a3) {
    const Cx<T> s0 = cadd(a0, a2), d0 = csub(a0, a2);
    const Cx<T> s1 = cadd(a1, a3), d1 = mul_mi<T, INV>(csub(a1, a3));
    a0 = cadd(s0, s1);
    a1 = cadd(d0, d1);
    a2 = csub(s0, s1);
    a3 = csub(d0, d1);
}
template <typename T, int R, int INV>
__device__ __forceinline__ void dft(Cx<T> (&a)[R]) {
    if constexpr (R == 2) {
        const Cx<T> t = a[0];
        a[0] = cadd(t, a[1]);
        a[1] = csub(t, a[1]);
    } else if constexpr (R == 4) {
        dft4<T, INV>(a[0], a[1], a[2], a[3]);
    } else if constexpr (R == 8) {
        // even / odd halves (4 points each), then X[k] = E[k] + W_8^k O[k], X[k+4] = E[k] - ...
        dft4<T, INV>(a[0], a[2], a[4], a[6]);
        dft4<T, INV>(a[1], a[3], a[5], a[7]);
        Cx<T> o[8];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const Cx<T> e = a[2 * k], w = mul_w8<T, INV>(a[2 * k + 1], k);
            o[k] = cadd(e, w);
            o[k + 4] = csub(e, w);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] = o[k];
    } else {
        static_assert(R == 16, "radix 2, 4, 8 or 16");
        // 16 = 4 x 4: DFTs over j1 of x[4 j1 + j2], twiddle W_16^(j2 k1), DFTs over j2
        const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173;   // pi/8
        const T h = (T)0.70710678118654752440;
#pragma unroll
        for (int j2 = 0; j2 < 4; ++j2) dft4<T, INV>(a[j2], a[4 + j2], a[8 + j2], a[12 + j2]);
        // now a[4 k1 + j2] = Y[j2][k1]
        const T sg = INV ? (T)1 : (T)-1;                       // sign of the sine
        const Cx<T> w1 = {c1, sg * s1}, w2 = {h, sg * h}, w3 = {s1, sg * c1};
        const Cx<T> w6 = {-h, sg * h}, w9 = {-c1, -sg * s1};
        a[4 * 1 + 1] = cmul(a[4 * 1 + 1], w1);
        a[4 * 1 + 2] = cmul(a[4 * 1 + 2], w2);
        a[4 * 1 + 3] = cmul(a[4 * 1 + 3], w3);
        a[4 * 2 + 1] = cmul(a[4 * 2 + 1], w2);
        a[4 * 2 + 2] = mul_mi<T, INV>(a[4 * 2 + 2]);          // W_16^4
        a[4 * 2 + 3] = cmul(a[4 * 2 + 3], w6);
        a[4 * 3 + 1] = cmul(a[4 * 3 + 1], w3);
        a[4 * 3 + 2] = cmul(a[4 * 3 + 2], w6);
        a[4 * 3 + 3] = cmul(a[4 * 3 + 3], w9);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1)
            dft4<T, INV>(a[4 * k1], a[4 * k1 + 1], a[4 * k1 + 2], a[4 * k1 + 3]);
        // now a[4 k1 + k2] = X[k1 + 4 k2]: transpose the 4 x 4 index
        Cx<T> o[16];
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) o[k1 + 4 * k2] = a[4 * k1 + k2];
#pragma unroll
        for (int k = 0; k < 16; ++k) a[k] = o[k];
    }
}

// One Stockham stage of radix R over `rows` sequences of length n = 2^logn held at
// buf[lpad(row n + i)]; ns = 2^lgns is the product of the radices already applied and tws the
// stage's twiddle table in LDS.  Butterfly (row, j), j < m = n / R: inputs i = j + r m, twiddled
// by W_(ns R)^(r kk) (kk = j mod ns), an R-point DFT, outputs at (j - kk) R + kk + r ns.  gin: the
// inputs come from ldg(row, i) instead of LDS (first stage); gout: the outputs go to stg(row, i,
// v) (last stage, natural order).  Every read happens before the barrier, every write after it.
template <typename T, int R, int INV, typename LDG, typename STG>
__device__ __forceinline__ void fft_stage(Cx<T> *buf, const Cx<T> *tws, int logn, int rows,
                                          int lgns, bool gin, bool gout, const LDG &ldg,
                                          const STG &stg) {
    constexpr int LR = R == 16 ? 4 : R == 8 ? 3 : R == 4 ? 2 : 1;
    constexpr int MT = kRegPts / R;
    const int logm = logn - LR, m = 1 << logm, ntask = rows << logm, ns = 1 << lgns;
    Cx<T> v[MT][R];
#pragma unroll
    for (int q = 0; q < MT; ++q) {
        const int t = threadIdx.x + q * kFT;
        if (t < ntask) {
            const int row = t >> logm, j = t & (m - 1);
#pragma unroll
            for (int r = 0; r < R; ++r)
                v[q][r] = gin ? ldg(row, j + r * m) : buf[lpad((row << logn) + j + r * m)];
            const int kk = j & (ns - 1);
            if (kk) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    Cx<T> w = tws[((r - 1) << lgns) + kk];
                    if (INV) w.y = -w.y;
                    v[q][r] = cmul(v[q][r], w);
                }
            }
            dft<T, R, INV>(v[q]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MT; ++q) {
        const int t = threadIdx.x + q * kFT;
        if (t < ntask) {
            const int row = t >> logm, j = t & (m - 1), kk = j & (ns - 1);
            const int base = (j - kk) * R + kk;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (gout) stg(row, base + (r << lgns), v[q][r]);
                else buf[lpad((row << logn) + base + (r << lgns))] = v[q][r];
            }
        }
    }
    __syncthreads();
}

// FFTs (INV = 1: inverse, unnormalised) of `rows` sequences of length n = 2^logn, n <= 4096,
// rows n <= kFftCap, with the stage tables of n at tw: radix-16 stages, then one of radix FR
// (FR = fft_last_radix(logn), a template parameter so that only two stage bodies are inlined).
// The first stage reads through ldg when gin, the last writes through stg when gout; otherwise
// the data start and end in buf in natural order.
template <typename T, int INV, int FR, typename LDG, typename STG>
__device__ __forceinline__ void fft_run(Cx<T> *buf, const Cx<T> *tw, int logn, int rows, bool gin,
                                        const LDG &ldg, bool gout, const STG &stg) {
    constexpr int LFR = FR == 16 ? 4 : FR == 8 ? 3 : FR == 4 ? 2 : 1;
    const int n16 = (logn - LFR) >> 2;
    int off = 0, lg = 0;
    for (int st = 0; st < n16; ++st) {
        fft_stage<T, 16, INV>(buf, tw + off, logn, rows, lg, gin && st == 0, false, ldg, stg);
        off += 15 << lg;
        lg += 4;
    }
    fft_stage<T, FR, INV>(buf, tw + off, logn, rows, lg, gin && n16 == 0, gout, ldg, stg);
}
// Copy the n - 1 stage-table entries of a transform into LDS.
template <typename T>
__device__ __forceinline__ void load_table(Cx<T> *tw, const Cx<T> *src, int n) {
    for (int m = threadIdx.x; m < n - 1; m += kFT) tw[m] = src[m];
}

// The half spectrum S[j][c][y] of an instance: complex T as (re, im) pairs (the buffer is sized
// for complex float64).
typedef float fvec2 __attribute__((ext_vector_type(2)));
template <typename T>
using cvec_t = typename std::conditional<sizeof(T) == 8, dvec2, fvec2>::type;

template <typename T>
__device__ __forceinline__ GAS T *spectrum(const Inst &I) {
    return reinterpret_cast<GAS T *>(gp(I.fs));
}
// The diagonal scale 1 / s of SYLV_PC_FOURIER_DIAG in precision T (null: plain preconditioner).
template <typename T>
__device__ __forceinline__ const T *fscale(const Inst &I) {
    return sizeof(T) == 8 ? reinterpret_cast<const T *>(I.fsc64)
                          : reinterpret_cast<const T *>(I.fsc32);
}
template <typename T>
__device__ __forceinline__ void cstore(GAS T *S, size_t i, Cx<T> v) {
    cvec_t<T> w;
    w.x = v.x;
    w.y = v.y;
    reinterpret_cast<GAS cvec_t<T> *>(S)[i] = w;
}
template <typename T>
__device__ __forceinline__ Cx<T> cload(const GAS T *S, size_t i) {
    const cvec_t<T> w = reinterpret_cast<const GAS cvec_t<T> *>(S)[i];
    return {w.x, w.y};
}

// Sum over the workgroup in a fixed order (one value per thread).
__device__ __forceinline__ double fp_block_sum(double v) {
    __shared__ double sm[kFT / 64];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
    __syncthreads();
    return ((sm[0] + sm[1]) + (sm[2] + sm[3])) + ((sm[4] + sm[5]) + (sm[6] + sm[7]));
}

// Fixed-order sum of `count` partials of slot `slot` (every thread receives it): four running
// sums per thread, then the workgroup in a fixed order.
__device__ __forceinline__ double fp_consume(const double *partial, int nred, int slot,
                                             int count) {
    const GAS double *pp = gp(partial) + (size_t)slot * nred;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int b = threadIdx.x;
    for (; b + 3 * kFT < count; b += 4 * kFT) {
        a0 += pp[b];
        a1 += pp[b + kFT];
        a2 += pp[b + 2 * kFT];
        a3 += pp[b + 3 * kFT];
    }
    for (; b < count; b += kFT) a0 += pp[b];
    return fp_block_sum((a0 + a1) + (a2 + a3));
}

// Placeholders for the unused global side of fft_run.
template <typename T>
struct NoLoad {
    __device__ Cx<T> operator()(int, int) const { return {(T)0, (T)0}; }
};
template <typename T>
struct NoStore {
    __device__ void operator()(int, int, Cx<T>) const {}
};

// 1 / sqrt(x): the hardware estimate in float32 (the preconditioner only has to be a fixed SPD
// operator), a rounded division in float64.
__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_t(double x) { return 1.0 / sqrt(x); }

// The k x k block of a mode with Laplacian eigenvalue lam, factored as L L^T (lower, with the
// reciprocals of its diagonal), applied to one complex right-hand side: z = (L L^T)^-1 r.
template <typename T, int K>
struct ModeSolver {
    T mb[K][K], k2[K], ta[K];
    __device__ void load(const double *fd) {
#pragma unroll
        for (int a = 0; a < K; ++a) {
            k2[a] = (T)fd[kMaxK * kMaxK + a];
            ta[a] = (T)fd[kMaxK * kMaxK + kMaxK + a];
#pragma unroll
            for (int b = 0; b < K; ++b) mb[a][b] = (T)fd[a * kMaxK + b];
        }
    }
    // real right-hand side (cosine modes)
    __device__ void solve_re(T lam, const T (&rh)[K], T (&zh)[K]) const {
        T l[K][K], id[K];
        factor(lam, l, id);
#pragma unroll
        for (int a = 0; a < K; ++a) {
            T s = rh[a];
#pragma unroll
            for (int q = 0; q < a; ++q) s -= l[a][q] * zh[q];
            zh[a] = s * id[a];
        }
#pragma unroll
        for (int a = K - 1; a >= 0; --a) {
            T s = zh[a];
#pragma unroll
            for (int q = a + 1; q < K; ++q) s -= l[q][a] * zh[q];
            zh[a] = s * id[a];
        }
    }
    __device__ void factor(T lam, T (&l)[K][K], T (&id)[K]) const {
#pragma unroll
        for (int a = 0; a < K; ++a) {
#pragma unroll
            for (int b = 0; b <= a; ++b) {
                T s = mb[a][b];
                if (a == b) {
                    const T u = k2[a] + lam;
                    s += ta[a] * u * u;
                }
#pragma unroll
                for (int q = 0; q < b; ++q) s -= l[a][q] * l[b][q];
                if (a == b) id[a] = rsqrt_t(s);
                else l[a][b] = s * id[b];
            }
        }
    }
    __device__ void solve(T lam, const Cx<T> (&rh)[K], Cx<T> (&zh)[K]) const {
        T l[K][K], id[K];
#pragma unroll
        for (int a = 0; a < K; ++a) {
#pragma unroll
            for (int b = 0; b <= a; ++b) {
                T s = mb[a][b];
                if (a == b) {
                    const T u = k2[a] + lam;
                    s += ta[a] * u * u;
                }
#pragma unroll
                for (int q = 0; q < b; ++q) s -= l[a][q] * l[b][q];
                if (a == b) id[a] = rsqrt_t(s);
                else l[a][b] = s * id[b];
            }
        }
#pragma unroll
        for (int a = 0; a < K; ++a) {
            Cx<T> s = rh[a];
#pragma unroll
            for (int q = 0; q < a; ++q) { s.x -= l[a][q] * zh[q].x; s.y -= l[a][q] * zh[q].y; }
            zh[a] = {s.x * id[a], s.y * id[a]};
        }
#pragma unroll
        for (int a = K - 1; a >= 0; --a) {
            Cx<T> s = zh[a];
#pragma unroll
            for (int q = a + 1; q < K; ++q) { s.x -= l[q][a] * zh[q].x; s.y -= l[q][a] * zh[q].y; }
            zh[a] = {s.x * id[a], s.y * id[a]};
        }
    }
};

template <typename T, int K>
__device__ __forceinline__ double dot_r(const T (&a)[K], const T (&b)[K]) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < K; ++q) s += (double)a[q] * (double)b[q];
    return s;
}

template <typename T, int K>
__device__ __forceinline__ double dot_re(const Cx<T> (&a)[K], const Cx<T> (&b)[K]) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < K; ++q) s += (double)a[q].x * (double)b[q].x + (double)a[q].y * (double)b[q].y;
    return s;
}

// Run state at the start of a forward row pass (inner < 0: the stand-alone preconditioner, no
// state).  Returns false when the workgroup has nothing to do: the run has stopped, or, for
// upd == 2 (the CG update of iteration `it` fused into the pass), this iteration's apply stopped
// it (its pending status is recorded) or <p, q> from the apply's partials is not a positive
// finite number (breakdown recorded).  Otherwise alpha = rho / <p, q> for the update, recorded by
// workgroup 0 for the next apply.
template <typename T>
__device__ __forceinline__ bool fp_update_prologue(const Inst &I, int inner, int upd, int it,
                                                   int blk, T &alpha) {
    if (inner < 0) return true;
    DevState *st = inner ? I.st_in : I.st;
    if (st->done) return false;
    if (upd != 2) return true;
    const int pend = st->pend;
    if (pend >= 0) {   // this iteration's apply stopped the run
        if (blk == 0 && threadIdx.x == 0) {
            st->status = pend;
            st->done = 1;
            st->total_iter += it;
        }
        return false;
    }
    const double pq = fp_consume(I.partial, I.nred, SLOT_PQ,
                                 I.pre ? 1 : (sizeof(T) == 4 ? I.ntiles32 : I.ntiles));
    int status = -1;
    if (!finite_d(pq)) status = SYLV_NONFINITE;
    else if (!(pq > 0.0)) status = SYLV_BREAKDOWN;
    const double alpha_d = st->rho[it & 1] / pq;
    if (blk == 0 && threadIdx.x == 0) {
        if (status >= 0) {
            st->status = status;
            st->done = 1;
            st->total_iter += it;
        } else {
            st->alpha[it & 1] = alpha_d;
        }
    }
    if (status >= 0) return false;
    alpha = (T)alpha_d;
    return true;
}

// Pass A: forward FFT of rows y0 .. y0 + rb of component j of r (rb even), half spectrum stored
// transposed: S[j][c][y], c in [0, nx/2].  Two real rows travel as one complex row, u = r_2q +
// i r_(2q+1) (the first stage reads them from global memory); their spectra separate by
// Hermitian symmetry, R_2q[c] = (U[c] + conj U[-c]) / 2 and R_(2q+1)[c] = (U[c] - conj U[-c]) /
// 2i.  The rb rows of one column c are consecutive in S, so the stores come in runs of rb
// complex values.
// In a CG run the pass also takes the ||r||^2 partials of its rows (upd = 1, start of a run) and
// first performs the update of iteration `it` (upd = 2): alpha = rho / <p, q> from the apply's
// partials (stop and breakdown handled as the streaming update kernel does), r -= alpha q as
// the first stage loads r and q, r written back.
// DCT (face grids): the rows' cosine transforms instead, from the reordered rows; the nx real
// coefficients of each row are stored transposed, S[j][u][y], u < nx, two rows per 8-byte store.
template <typename T, int CLS, bool DCT, bool SC>
__global__ __launch_bounds__(kFT) void k_fp_rows_fwd(const Inst *__restrict__ tab,
                                                     const int *__restrict__ fpre, int ninst,
                                                     int nb, int inner,
                                                     const T *__restrict__ rin, int use_in,
                                                     int upd, int it) {
    extern __shared__ __align__(16) unsigned char fp_lds[];
    const int L = xcd_remap(blockIdx.x, nb);
    const int ii = find_inst(fpre, ninst, L);
    const Inst &I = tab[ii];
    if (fft_class(I.lognx) != CLS) return;                         // another launch's instance
    constexpr int FR = cls_fr(CLS), LN = cls_ln(CLS);
    const int blk = L - fpre[ii];
    T alpha = (T)0;
    if (!fp_update_prologue(I, inner, upd, it, blk, alpha)) return;
    const int ln = LN ? LN : I.lognx, nx = 1 << ln;
    const int ny = I.ny, rb = I.frb, nc = nx / 2 + 1, h = rb / 2;
    const int lrb = __builtin_ctz((unsigned)rb), nrb = ny >> lrb;
    const int j = blk / nrb, y0 = (blk - j * nrb) << lrb;
    Cx<T> *tw = reinterpret_cast<Cx<T> *>(fp_lds);
    Cx<T> *buf = tw + nx;
    const FpTabs tb = fp_tabs(nx, ny);
    load_table<T>(tw, stage_table<T>(I.fsym, tb, true), nx);
    __syncthreads();
    const uint32_t np = (uint32_t)I.n_pix;
    GAS T *r = (use_in ? gp(const_cast<T *>(rin)) : Sel<T>::r(I)) + (size_t)j * I.n_pix;
    const GAS T *qv = Sel<T>::q(I) + (size_t)j * I.n_pix;
    const uint32_t o0 = (uint32_t)y0 * (uint32_t)nx;
    // SC (SYLV_PC_FOURIER_DIAG): the transforms take S^-1 r
    const GAS T *sc = gp(fscale<T>(I)) + (SC ? (size_t)j * I.n_pix : 0);
    double rr = 0.0;
    const auto ldg = [&](int q, int i) -> Cx<T> {
        const uint32_t o = o0 + ((uint32_t)(2 * q) << ln) + (uint32_t)(DCT ? cos_src(i, nx) : i);
        T a = bld(r, np, o), b = bld(r, np, o + (uint32_t)nx);
        if (upd == 2) {
            a -= alpha * bld(qv, np, o);
            b -= alpha * bld(qv, np, o + (uint32_t)nx);
            bst(r, np, o, a);
            bst(r, np, o + (uint32_t)nx, b);
        }
        rr += (double)a * (double)a + (double)b * (double)b;
        if constexpr (SC) {
            a *= bld(sc, np, o);
            b *= bld(sc, np, o + (uint32_t)nx);
        }
        return {a, b};
    };
    fft_run<T, 0, FR>(buf, tw, ln, h, true, ldg, false, NoStore<T>());
    if (upd) {   // the ||r||^2 partial of this workgroup's rows
        const double tot = fp_block_sum(rr);
        if (threadIdx.x == 0) gp(I.partial)[(size_t)SLOT_RR * I.nred + blk] = tot;
    }
    if (DCT) {
        // rows 2q, 2q+1: V_2q[u] = (U[u] + conj U[-u]) / 2, V_(2q+1)[u] = (U[u] - conj U[-u]) / 2i,
        // X[u] = Re(exp(-i pi u / 2nx) V[u])
        GAS T *Sr = spectrum<T>(I) + (size_t)j * nx * ny;
        const Cx<T> *ct = cos_table<T>(I.fsym, tb, true);
        const int lh = lrb - 1;
        const T hf = (T)0.5;
        for (int e = threadIdx.x; e < (nx << lh); e += kFT) {
            const int u = e >> lh, q = e & (h - 1);
            const Cx<T> U = buf[lpad((q << ln) + u)];
            const Cx<T> M = buf[lpad((q << ln) + ((nx - u) & (nx - 1)))];
            const Cx<T> va = {hf * (U.x + M.x), hf * (U.y - M.y)};
            const Cx<T> vb = {hf * (U.y + M.y), hf * (M.x - U.x)};
            const Cx<T> w = ct[u];
            cstore(Sr, ((size_t)u * ny + y0) / 2 + q,
                   Cx<T>{w.x * va.x - w.y * va.y, w.x * vb.x - w.y * vb.y});
        }
        return;
    }
    GAS T *S = spectrum<T>(I) + (size_t)2 * j * nc * ny;
    const T half = (T)0.5;
    for (int e = threadIdx.x; e < rb * nc; e += kFT) {
        const int c = e >> lrb, yy = e & (rb - 1), q = yy >> 1;
        const Cx<T> U = buf[lpad((q << ln) + c)];
        const Cx<T> V = buf[lpad((q << ln) + ((nx - c) & (nx - 1)))];   // U[-c]
        const Cx<T> out = (yy & 1) ? Cx<T>{half * (U.y + V.y), half * (V.x - U.x)}
                                   : Cx<T>{half * (U.x + V.x), half * (U.y - V.y)};
        cstore(S, (size_t)c * ny + y0 + yy, out);
    }
}

// Pass B: column c of the half spectrum for every component: forward FFT along y (first stage
// from global memory), the per-mode k x k solve, the <r, z> partial (Parseval: each c in
// (0, nx/2) stands for itself and its conjugate partner), inverse FFT along y (last stage to
// global memory).  Workgroup 0 takes the two real columns c = 0 and c = nx/2 as w = S[.][0] + i
// S[.][nx/2]: with W its transform, F0[v] = (W[v] + conj W[-v]) / 2 and Fn[v] = (W[v] - conj
// W[-v]) / 2i are the two columns' spectra; each is solved with its own eigenvalues, Z0 + i Zn
// is transformed back, and its real and imaginary parts are the two columns.  A thread owns the
// modes v and -v together (Z[-v] = conj Z[v] for both columns), so no mode is shared.
// GTW: the stage twiddles are read from the set-up table in global memory (when the table and
// the column do not both fit in LDS; float64 columns of 8192 values).
// DCT (face grids): workgroup c takes the real coefficient columns u0 = 2c and u1 = 2c + 1 of
// pass A as one complex column, transforms it by the cosine transform along y (reordered, FFT,
// split into the two columns' spectra, twiddled), solves the real k x k system of each of the
// four modes (u0, v), (u0, -v), (u1, v), (u1, -v) a thread owns, and transforms back.  <r, z> by
// Parseval with the orthonormal weights (1 or 2) / n of each side.
template <typename T, int K, int CLS, bool GTW, bool DCT>
__global__ __launch_bounds__(kFT, (sizeof(T) == 8 || K > 5 || (DCT && K > 4)) ? 2 : 4) void k_fp_cols(
    const Inst *__restrict__ tab, const int *__restrict__ fpre, int ninst, int nb, int inner) {
    extern __shared__ __align__(16) unsigned char fp_lds[];
    const int L = xcd_remap(blockIdx.x, nb);
    const int ii = find_inst(fpre, ninst, L);
    const Inst &I = tab[ii];
    if (inner >= 0 && (inner ? I.st_in : I.st)->done) return;   // inner < 0: stand-alone
    if (fft_class(I.logny) != CLS) return;                         // another launch's instance
    constexpr int FR = cls_fr(CLS), LN = cls_ln(CLS);
    const int c = L - fpre[ii];
    const int ln = LN ? LN : I.logny, ny = 1 << ln;
    const int nx = I.nx, nc = nx / 2 + 1, cn = nx / 2;
    const FpTabs tb = fp_tabs(nx, ny);
    Cx<T> *buf = reinterpret_cast<Cx<T> *>(fp_lds) + (GTW ? 0 : ny);
    const Cx<T> *tw = stage_table<T>(I.fsym, tb, false);
    if (!GTW) {
        load_table<T>(reinterpret_cast<Cx<T> *>(fp_lds), tw, ny);
        tw = reinterpret_cast<const Cx<T> *>(fp_lds);
    }
    __syncthreads();
    GAS T *S = spectrum<T>(I);
    const double *lamy = I.fsym + tb.lamy;
    ModeSolver<T, K> ms;
    ms.load(I.fsym);
    double rz = 0.0;
    if constexpr (DCT) {
        const int u0 = 2 * c, u1 = 2 * c + 1;
        const size_t pl = (size_t)nx * ny;   // one component's coefficients
        const auto ldg = [&](int a, int y) -> Cx<T> {
            const size_t o = a * pl + cos_src(y, ny);
            return {S[o + (size_t)u0 * ny], S[o + (size_t)u1 * ny]};
        };
        fft_run<T, 0, FR>(buf, tw, ln, K, true, ldg, false, NoStore<T>());
        const Cx<T> *ct = cos_table<T>(I.fsym, tb, false);
        const T lx0 = (T)I.fsym[tb.lamx + u0], lx1 = (T)I.fsym[tb.lamx + u1];
        const double wx0 = (u0 == 0 ? 1.0 : 2.0) / nx, wx1 = 2.0 / nx;
        const T hf = (T)0.5;
        for (int v = threadIdx.x; v <= ny / 2; v += kFT) {
            const int w = (ny - v) & (ny - 1);
            const Cx<T> tv = ct[v], tw2 = ct[w];
            T c0v[K], c1v[K], c0w[K], c1w[K];
#pragma unroll
            for (int a = 0; a < K; ++a) {
                const Cx<T> P = buf[lpad((a << ln) + v)], M = buf[lpad((a << ln) + w)];
                const Cx<T> va = {hf * (P.x + M.x), hf * (P.y - M.y)};
                const Cx<T> vb = {hf * (P.y + M.y), hf * (M.x - P.x)};
                c0v[a] = tv.x * va.x - tv.y * va.y;     // Re(t_v V0[v])
                c1v[a] = tv.x * vb.x - tv.y * vb.y;
                c0w[a] = tw2.x * va.x + tw2.y * va.y;   // Re(t_w conj V0[v]) = Re(t_w V0[w])
                c1w[a] = tw2.x * vb.x + tw2.y * vb.y;
            }
            const T lyv = (T)lamy[v], lyw = (T)lamy[w];
            const double wyv = (v == 0 ? 1.0 : 2.0) / ny, wyw = (w == 0 ? 1.0 : 2.0) / ny;
            T z0v[K], z1v[K], z0w[K], z1w[K];
            ms.solve_re(lx0 + lyv, c0v, z0v);
            ms.solve_re(lx1 + lyv, c1v, z1v);
            rz += wx0 * wyv * dot_r<T, K>(c0v, z0v) + wx1 * wyv * dot_r<T, K>(c1v, z1v);
            if (w != v) {
                ms.solve_re(lx0 + lyw, c0w, z0w);
                ms.solve_re(lx1 + lyw, c1w, z1w);
                rz += wx0 * wyw * dot_r<T, K>(c0w, z0w) + wx1 * wyw * dot_r<T, K>(c1w, z1w);
            }
#pragma unroll
            for (int a = 0; a < K; ++a) {
                // V[v] = conj(t_v) (Z[v] - i Z[ny - v]) with Z[ny] = 0; U' = V0 + i V1
                const T m0 = v == 0 ? (T)0 : (w == v ? z0v[a] : z0w[a]);
                const T m1 = v == 0 ? (T)0 : (w == v ? z1v[a] : z1w[a]);
                const Cx<T> a0 = {tv.x * z0v[a] - tv.y * m0, -tv.y * z0v[a] - tv.x * m0};
                const Cx<T> a1 = {tv.x * z1v[a] - tv.y * m1, -tv.y * z1v[a] - tv.x * m1};
                buf[lpad((a << ln) + v)] = {a0.x - a1.y, a0.y + a1.x};
                if (w != v) {
                    const Cx<T> b0 = {tw2.x * z0w[a] - tw2.y * z0v[a], -tw2.y * z0w[a] - tw2.x * z0v[a]};
                    const Cx<T> b1 = {tw2.x * z1w[a] - tw2.y * z1v[a], -tw2.y * z1w[a] - tw2.x * z1v[a]};
                    buf[lpad((a << ln) + w)] = {b0.x - b1.y, b0.y + b1.x};
                }
            }
        }
        __syncthreads();
        const auto stg = [&](int a, int m, Cx<T> val) {
            const size_t o = a * pl + cos_src(m, ny);
            S[o + (size_t)u0 * ny] = val.x;
            S[o + (size_t)u1 * ny] = val.y;
        };
        fft_run<T, 1, FR>(buf, tw, ln, K, false, NoLoad<T>(), true, stg);
        const double tot = fp_block_sum(rz);
        if (I.partial && threadIdx.x == 0) gp(I.partial)[(size_t)SLOT_FRZ * I.nred + c] = tot;
        return;
    }
    // column c (c > 0), or the real columns 0 and nx/2 packed as re + i im (c = 0)
    const auto ldg = [&](int a, int y) -> Cx<T> {
        if (c > 0) return cload(S, ((size_t)a * nc + c) * ny + y);
        return {S[2 * (((size_t)a * nc) * ny + y)], S[2 * (((size_t)a * nc + cn) * ny + y)]};
    };
    fft_run<T, 0, FR>(buf, tw, ln, K, true, ldg, false, NoStore<T>());
    if (c > 0) {
        const T lx = (T)I.fsym[tb.lamx + c];
        for (int v = threadIdx.x; v < ny; v += kFT) {
            Cx<T> rh[K], zh[K];
#pragma unroll
            for (int a = 0; a < K; ++a) rh[a] = buf[lpad((a << ln) + v)];
            ms.solve(lx + (T)lamy[v], rh, zh);
            rz += 2.0 * dot_re<T, K>(rh, zh);
#pragma unroll
            for (int a = 0; a < K; ++a) buf[lpad((a << ln) + v)] = zh[a];
        }
    } else {
        const T lxn = (T)I.fsym[tb.lamx + cn];
        for (int v = threadIdx.x; v <= ny / 2; v += kFT) {
            const int w = (ny - v) & (ny - 1);
            Cx<T> f0[K], fn[K], z0[K], zn[K];
#pragma unroll
            for (int a = 0; a < K; ++a) {
                const Cx<T> P = buf[lpad((a << ln) + v)], M = buf[lpad((a << ln) + w)];
                f0[a] = {(T)0.5 * (P.x + M.x), (T)0.5 * (P.y - M.y)};
                fn[a] = {(T)0.5 * (P.y + M.y), (T)0.5 * (M.x - P.x)};
            }
            const T ly = (T)lamy[v];
            ms.solve(ly, f0, z0);
            ms.solve(lxn + ly, fn, zn);
            rz += (w == v ? 1.0 : 2.0) * (dot_re<T, K>(f0, z0) + dot_re<T, K>(fn, zn));
#pragma unroll
            for (int a = 0; a < K; ++a) {
                // U[v] = Z0 + i Zn, U[-v] = conj Z0 + i conj Zn
                buf[lpad((a << ln) + v)] = {z0[a].x - zn[a].y, z0[a].y + zn[a].x};
                if (w != v) buf[lpad((a << ln) + w)] = {z0[a].x + zn[a].y, zn[a].x - z0[a].y};
            }
        }
    }
    __syncthreads();
    const auto stg = [&](int a, int y, Cx<T> v) {
        if (c > 0) {
            cstore(S, ((size_t)a * nc + c) * ny + y, v);
        } else {
            cstore(S, ((size_t)a * nc) * ny + y, Cx<T>{v.x, (T)0});
            cstore(S, ((size_t)a * nc + cn) * ny + y, Cx<T>{v.y, (T)0});
        }
    };
    fft_run<T, 1, FR>(buf, tw, ln, K, false, NoLoad<T>(), true, stg);
    // <r, z> = rz / (nx ny): the partial of this workgroup (none for the stand-alone application)
    const double tot = fp_block_sum(rz);
    if (I.partial && threadIdx.x == 0)
        gp(I.partial)[(size_t)SLOT_FRZ * I.nred + c] = tot / ((double)nx * (double)ny);
}

// Pass C: rows y0 .. y0 + rb of component j, two real rows per complex inverse FFT: with R_2q
// and R_(2q+1) the half spectra of the two rows, U[c] = R_2q[c] + i R_(2q+1)[c] and U[-c] =
// conj R_2q[c] + i conj R_(2q+1)[c]; the inverse FFT of U is r_2q + i r_(2q+1) (times nx), and
// z = those parts / (nx ny), written by the last stage.
// DCT (face grids): the rows' inverse cosine transforms: U[u] = V_2q[u] + i V_(2q+1)[u] with
// V[u] = exp(i pi u / 2nx) (Z[u] - i Z[nx - u]), the inverse FFT, and the reorder undone as the
// last stage writes z.
template <typename T, int CLS, bool DCT, bool SC>
__global__ __launch_bounds__(kFT) void k_fp_rows_inv(const Inst *__restrict__ tab,
                                                     const int *__restrict__ fpre, int ninst,
                                                     int nb, int inner, T *__restrict__ zout,
                                                     int use_out) {
    extern __shared__ __align__(16) unsigned char fp_lds[];
    const int L = xcd_remap(blockIdx.x, nb);
    const int ii = find_inst(fpre, ninst, L);
    const Inst &I = tab[ii];
    if (inner >= 0 && (inner ? I.st_in : I.st)->done) return;   // inner < 0: stand-alone
    if (fft_class(I.lognx) != CLS) return;                         // another launch's instance
    constexpr int FR = cls_fr(CLS), LN = cls_ln(CLS);
    const int blk = L - fpre[ii];
    const int ln = LN ? LN : I.lognx, nx = 1 << ln;
    const int ny = I.ny, rb = I.frb, nc = nx / 2 + 1, h = rb / 2;
    const int lrb = __builtin_ctz((unsigned)rb), nrb = ny >> lrb;
    const int j = blk / nrb, y0 = (blk - j * nrb) << lrb;
    Cx<T> *tw = reinterpret_cast<Cx<T> *>(fp_lds);
    Cx<T> *buf = tw + nx;
    const FpTabs tb = fp_tabs(nx, ny);
    load_table<T>(tw, stage_table<T>(I.fsym, tb, true), nx);
    const int lh = lrb - 1;
    // SC (SYLV_PC_FOURIER_DIAG): z = S^-1 times the inverse transform
    const GAS T *sc = gp(fscale<T>(I)) + (SC ? (size_t)j * I.n_pix : 0);
    if (DCT) {
        const GAS T *Sr = spectrum<T>(I) + (size_t)j * nx * ny;
        const Cx<T> *ct = cos_table<T>(I.fsym, tb, true);
        for (int e = threadIdx.x; e < ((nx / 2 + 1) << lh); e += kFT) {
            const int u = e >> lh, q = e & (h - 1), um = (nx - u) & (nx - 1);
            const Cx<T> zu = cload(Sr, ((size_t)u * ny + y0) / 2 + q);   // (Z_2q[u], Z_2q+1[u])
            const Cx<T> zm = u == 0 ? Cx<T>{(T)0, (T)0} : cload(Sr, ((size_t)um * ny + y0) / 2 + q);
            const Cx<T> t = ct[u];
            const Cx<T> a0 = {t.x * zu.x - t.y * zm.x, -t.y * zu.x - t.x * zm.x};
            const Cx<T> a1 = {t.x * zu.y - t.y * zm.y, -t.y * zu.y - t.x * zm.y};
            buf[lpad((q << ln) + u)] = {a0.x - a1.y, a0.y + a1.x};
            if (u != 0 && um != u) {
                const Cx<T> tm = ct[um];
                const Cx<T> b0 = {tm.x * zm.x - tm.y * zu.x, -tm.y * zm.x - tm.x * zu.x};
                const Cx<T> b1 = {tm.x * zm.y - tm.y * zu.y, -tm.y * zm.y - tm.x * zu.y};
                buf[lpad((q << ln) + um)] = {b0.x - b1.y, b0.y + b1.x};
            }
        }
        __syncthreads();
        const T scale = (T)(1.0 / ((double)nx * (double)ny));
        const uint32_t np = (uint32_t)I.n_pix;
        GAS T *z = (use_out ? gp(zout) : gp(Sel<T>::z(I))) + (size_t)j * I.n_pix;
        const uint32_t o0 = (uint32_t)y0 * (uint32_t)nx;
        const auto stg = [&](int q, int m, Cx<T> v) {
            const uint32_t o = o0 + ((uint32_t)(2 * q) << ln) + (uint32_t)cos_src(m, nx);
            T s0 = scale, s1 = scale;
            if constexpr (SC) {
                s0 *= bld(sc, np, o);
                s1 *= bld(sc, np, o + (uint32_t)nx);
            }
            bst(z, np, o, v.x * s0);
            bst(z, np, o + (uint32_t)nx, v.y * s1);
        };
        fft_run<T, 1, FR>(buf, tw, ln, h, false, NoLoad<T>(), true, stg);
        return;
    }
    const GAS T *S = spectrum<T>(I) + (size_t)2 * j * nc * ny;
    // stage: unit u = rows 2q, 2q + 1 of column c = u / h (one 4-vector)
    const int units = nc << lh;
    constexpr int G = sizeof(T) == 8 ? 4 : 8;
    for (int u0 = 0; u0 < units; u0 += G * kFT) {
        T a[G][4];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int u = u0 + g * kFT + threadIdx.x;
            if (u < units) {
                const int c = u >> lh, q = u & (h - 1);
                ld4(S + 2 * ((size_t)c * ny + y0 + 2 * q), a[g]);
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int u = u0 + g * kFT + threadIdx.x;
            if (u < units) {
                const int c = u >> lh, q = u & (h - 1);
                const T ex = a[g][0], ey = a[g][1], ox = a[g][2], oy = a[g][3];
                buf[lpad((q << ln) + c)] = {ex - oy, ey + ox};
                if (c > 0 && 2 * c < nx) buf[lpad((q << ln) + nx - c)] = {ex + oy, ox - ey};
            }
        }
    }
    __syncthreads();
    const T scale = (T)(1.0 / ((double)nx * (double)ny));
    const uint32_t np = (uint32_t)I.n_pix;
    GAS T *z = (use_out ? gp(zout) : gp(Sel<T>::z(I))) + (size_t)j * I.n_pix;
    const uint32_t o0 = (uint32_t)y0 * (uint32_t)nx;
    const auto stg = [&](int q, int i, Cx<T> v) {
        const uint32_t o = o0 + ((uint32_t)(2 * q) << ln) + (uint32_t)i;
        T s0 = scale, s1 = scale;
        if constexpr (SC) {
            s0 *= bld(sc, np, o);
            s1 *= bld(sc, np, o + (uint32_t)nx);
        }
        bst(z, np, o, v.x * s0);
        bst(z, np, o + (uint32_t)nx, v.y * s1);
    };
    fft_run<T, 1, FR>(buf, tw, ln, h, false, NoLoad<T>(), true, stg);
}

// Block-scaled variant (SYLV_PC_FOURIER_BLOCK): z = T^T M0^-1 T r with T_p = L0_p Lp^-1 lower
// triangular per pixel (Lp Lp^T = G's k x k block of the pixel, L0_p L0_p^T that block of
// M0 = Q + I (x) Mbar), stored packed at tidx(a, b), a >= b, one plane per entry.  Its row passes
// transform all K components of rb grid rows in one workgroup (K rb / 2 complex rows: row pair qq
// of component j is complex row j rb / 2 + qq), so that T r before the forward transforms and
// T^T zhat after the inverse ones see every component of a pixel.  They stage the pixel products
// through LDS (the transforms start and end there); the column pass is the same as above.
__host__ __device__ constexpr int tidx(int a, int b) { return a * (a + 1) / 2 + b; }
// Inverse of cos_src: the transform index of sample x.
__device__ __forceinline__ int cos_dst(int x, int n) { return (x & 1) ? n - 1 - (x >> 1) : x >> 1; }
// Pixel pairs a thread of the block-scaled row passes has in flight at once: as many as about
// 96 (float32) or 48 (float64) loaded values allow, each pair holding 2 (K + K(K+1)/2) of them.
template <typename T, int K>
constexpr int blk_pairs() {
    constexpr int per = 2 * (K + K * (K + 1) / 2), cap = sizeof(T) == 8 ? 48 : 96;
    return per >= cap ? 1 : (cap / per > 4 ? 4 : cap / per);
}

// Pass A of the block-scaled variant: the update and ||r||^2 partials as k_fp_rows_fwd (upd), then
// u = T_p r_p at every pixel of the band, the forward row transforms of all components, and the
// half spectrum (or the cosine coefficients) of every component stored as k_fp_rows_fwd does.
template <typename T, int K, int CLS, bool DCT, bool GTW>
__global__ __launch_bounds__(kFT) void k_fp_rows_fwd_blk(const Inst *__restrict__ tab,
                                                         const int *__restrict__ fpre, int ninst,
                                                         int nb, int inner,
                                                         const T *__restrict__ rin, int use_in,
                                                         int upd, int it) {
    extern __shared__ __align__(16) unsigned char fp_lds[];
    const int L = xcd_remap(blockIdx.x, nb);
    const int ii = find_inst(fpre, ninst, L);
    const Inst &I = tab[ii];
    if (fft_class(I.lognx) != CLS) return;                         // another launch's instance
    constexpr int FR = cls_fr(CLS), LN = cls_ln(CLS);
    const int blk = L - fpre[ii];
    T alpha = (T)0;
    if (!fp_update_prologue(I, inner, upd, it, blk, alpha)) return;
    const int ln = LN ? LN : I.lognx, nx = 1 << ln;
    const int ny = I.ny, rb = I.frb, nc = nx / 2 + 1, hb = rb / 2;
    const int lrb = __builtin_ctz((unsigned)rb), lh = lrb - 1, y0 = blk << lrb;
    // GTW: the stage twiddles read from the set-up table in global memory (float64 bands whose
    // k complex rows and table do not both fit in LDS)
    Cx<T> *buf = reinterpret_cast<Cx<T> *>(fp_lds) + (GTW ? 0 : nx);
    const FpTabs tb = fp_tabs(nx, ny);
    const Cx<T> *tw = stage_table<T>(I.fsym, tb, true);
    if (!GTW) {
        load_table<T>(reinterpret_cast<Cx<T> *>(fp_lds), tw, nx);
        tw = reinterpret_cast<const Cx<T> *>(fp_lds);
    }
    const uint32_t np = (uint32_t)I.n_pix;
    const size_t pl = (size_t)I.n_pix;
    GAS T *r = use_in ? gp(const_cast<T *>(rin)) : Sel<T>::r(I);
    const GAS T *qv = Sel<T>::q(I);
    const GAS T *tp = gp(fscale<T>(I));
    double rr = 0.0;
    constexpr int NB = blk_pairs<T, K>(), KP = K * (K + 1) / 2;
    const int items = hb << ln;
    for (int e0 = threadIdx.x; e0 < items; e0 += NB * kFT) {
        // every load of NB pixel pairs first, then the products
        T v[NB][2][K], tt[NB][2][KP];
#pragma unroll
        for (int g = 0; g < NB; ++g) {
            const int e = e0 + g * kFT;
            if (e < items) {
                const int qq = e >> ln, x = e & (nx - 1);
#pragma unroll
                for (int w = 0; w < 2; ++w) {
                    const uint32_t o = (uint32_t)(y0 + 2 * qq + w) * (uint32_t)nx + (uint32_t)x;
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        v[g][w][j] = bld(r + j * pl, np, o);
                        if (upd == 2) v[g][w][j] -= alpha * bld(qv + j * pl, np, o);
                    }
#pragma unroll
                    for (int t = 0; t < KP; ++t) tt[g][w][t] = bld(tp + t * pl, np, o);
                }
            }
        }
#pragma unroll
        for (int g = 0; g < NB; ++g) {
            const int e = e0 + g * kFT;
            if (e < items) {
                const int qq = e >> ln, x = e & (nx - 1);
                T u[2][K];
#pragma unroll
                for (int w = 0; w < 2; ++w) {
                    if (upd == 2) {
                        const uint32_t o =
                            (uint32_t)(y0 + 2 * qq + w) * (uint32_t)nx + (uint32_t)x;
#pragma unroll
                        for (int j = 0; j < K; ++j) bst(r + j * pl, np, o, v[g][w][j]);
                    }
#pragma unroll
                    for (int j = 0; j < K; ++j) rr += (double)v[g][w][j] * (double)v[g][w][j];
#pragma unroll
                    for (int a = 0; a < K; ++a) {
                        T sacc = (T)0;
#pragma unroll
                        for (int b = 0; b <= a; ++b) sacc += tt[g][w][tidx(a, b)] * v[g][w][b];
                        u[w][a] = sacc;
                    }
                }
                const int i = DCT ? cos_dst(x, nx) : x;
#pragma unroll
                for (int a = 0; a < K; ++a)
                    buf[lpad(((a * hb + qq) << ln) + i)] = {u[0][a], u[1][a]};
            }
        }
    }
    __syncthreads();
    fft_run<T, 0, FR>(buf, tw, ln, K * hb, false, NoLoad<T>(), false, NoStore<T>());
    if (upd) {   // the ||r||^2 partial of this workgroup's rows (all components)
        const double tot = fp_block_sum(rr);
        if (threadIdx.x == 0) gp(I.partial)[(size_t)SLOT_RR * I.nred + blk] = tot;
    }
    if (DCT) {
        const Cx<T> *ct = cos_table<T>(I.fsym, tb, true);
        const T hf = (T)0.5;
        const int per = nx << lh;   // entries of one component
        for (int e = threadIdx.x; e < K * per; e += kFT) {
            const int j = e >> (ln + lh), e2 = e & (per - 1);
            const int u = e2 >> lh, q = j * hb + (e2 & (hb - 1));
            GAS T *Sr = spectrum<T>(I) + (size_t)j * nx * ny;
            const Cx<T> U = buf[lpad((q << ln) + u)];
            const Cx<T> M = buf[lpad((q << ln) + ((nx - u) & (nx - 1)))];
            const Cx<T> va = {hf * (U.x + M.x), hf * (U.y - M.y)};
            const Cx<T> vb = {hf * (U.y + M.y), hf * (M.x - U.x)};
            const Cx<T> w = ct[u];
            cstore(Sr, ((size_t)u * ny + y0) / 2 + (e2 & (hb - 1)),
                   Cx<T>{w.x * va.x - w.y * va.y, w.x * vb.x - w.y * vb.y});
        }
        return;
    }
    const T half = (T)0.5;
    const int per = rb * nc;
    for (int e = threadIdx.x; e < K * per; e += kFT) {
        const int j = e / per, e2 = e - j * per;
        const int c = e2 >> lrb, yy = e2 & (rb - 1), q = j * hb + (yy >> 1);
        GAS T *S = spectrum<T>(I) + (size_t)2 * j * nc * ny;
        const Cx<T> U = buf[lpad((q << ln) + c)];
        const Cx<T> V = buf[lpad((q << ln) + ((nx - c) & (nx - 1)))];   // U[-c]
        const Cx<T> out = (yy & 1) ? Cx<T>{half * (U.y + V.y), half * (V.x - U.x)}
                                   : Cx<T>{half * (U.x + V.x), half * (U.y - V.y)};
        cstore(S, (size_t)c * ny + y0 + yy, out);
    }
}

// Pass C of the block-scaled variant: the rows of every component rebuilt from the half spectrum
// (or the cosine coefficients) as k_fp_rows_inv does, the inverse row transforms, then
// z_p = T_p^T zhat_p / (nx ny) at every pixel of the band.
template <typename T, int K, int CLS, bool DCT, bool GTW>
__global__ __launch_bounds__(kFT) void k_fp_rows_inv_blk(const Inst *__restrict__ tab,
                                                         const int *__restrict__ fpre, int ninst,
                                                         int nb, int inner, T *__restrict__ zout,
                                                         int use_out) {
    extern __shared__ __align__(16) unsigned char fp_lds[];
    const int L = xcd_remap(blockIdx.x, nb);
    const int ii = find_inst(fpre, ninst, L);
    const Inst &I = tab[ii];
    if (inner >= 0 && (inner ? I.st_in : I.st)->done) return;   // inner < 0: stand-alone
    if (fft_class(I.lognx) != CLS) return;                         // another launch's instance
    constexpr int FR = cls_fr(CLS), LN = cls_ln(CLS);
    const int blk = L - fpre[ii];
    const int ln = LN ? LN : I.lognx, nx = 1 << ln;
    const int ny = I.ny, rb = I.frb, nc = nx / 2 + 1, hb = rb / 2;
    const int lrb = __builtin_ctz((unsigned)rb), lh = lrb - 1, y0 = blk << lrb;
    // GTW: the stage twiddles read from the set-up table in global memory (float64 bands whose
    // k complex rows and table do not both fit in LDS)
    Cx<T> *buf = reinterpret_cast<Cx<T> *>(fp_lds) + (GTW ? 0 : nx);
    const FpTabs tb = fp_tabs(nx, ny);
    const Cx<T> *tw = stage_table<T>(I.fsym, tb, true);
    if (!GTW) {
        load_table<T>(reinterpret_cast<Cx<T> *>(fp_lds), tw, nx);
        tw = reinterpret_cast<const Cx<T> *>(fp_lds);
    }
    if (DCT) {
        const Cx<T> *ct = cos_table<T>(I.fsym, tb, true);
        const int per = (nx / 2 + 1) << lh;
        for (int e = threadIdx.x; e < K * per; e += kFT) {
            const int j = e / per, e2 = e - j * per;
            const int u = e2 >> lh, qq = e2 & (hb - 1), q = j * hb + qq;
            const int um = (nx - u) & (nx - 1);
            const GAS T *Sr = spectrum<T>(I) + (size_t)j * nx * ny;
            const Cx<T> zu = cload(Sr, ((size_t)u * ny + y0) / 2 + qq);
            const Cx<T> zm = u == 0 ? Cx<T>{(T)0, (T)0} : cload(Sr, ((size_t)um * ny + y0) / 2 + qq);
            const Cx<T> t = ct[u];
            const Cx<T> a0 = {t.x * zu.x - t.y * zm.x, -t.y * zu.x - t.x * zm.x};
            const Cx<T> a1 = {t.x * zu.y - t.y * zm.y, -t.y * zu.y - t.x * zm.y};
            buf[lpad((q << ln) + u)] = {a0.x - a1.y, a0.y + a1.x};
            if (u != 0 && um != u) {
                const Cx<T> tm = ct[um];
                const Cx<T> b0 = {tm.x * zm.x - tm.y * zu.x, -tm.y * zm.x - tm.x * zu.x};
                const Cx<T> b1 = {tm.x * zm.y - tm.y * zu.y, -tm.y * zm.y - tm.x * zu.y};
                buf[lpad((q << ln) + um)] = {b0.x - b1.y, b0.y + b1.x};
            }
        }
    } else {
        // unit u = rows 2qq, 2qq + 1 of column c of component j (one 4-vector), G units of a
        // thread in flight at once
        const int per = nc << lh, units = K * per;
        constexpr int G = sizeof(T) == 8 ? 4 : 8;
        for (int u0 = 0; u0 < units; u0 += G * kFT) {
            T a[G][4];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int e = u0 + g * kFT + threadIdx.x;
                if (e < units) {
                    const int j = e / per, e2 = e - j * per;
                    const int c = e2 >> lh, qq = e2 & (hb - 1);
                    ld4(spectrum<T>(I) + (size_t)2 * j * nc * ny + 2 * ((size_t)c * ny + y0 + 2 * qq),
                        a[g]);
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int e = u0 + g * kFT + threadIdx.x;
                if (e < units) {
                    const int j = e / per, e2 = e - j * per;
                    const int c = e2 >> lh, q = j * hb + (e2 & (hb - 1));
                    buf[lpad((q << ln) + c)] = {a[g][0] - a[g][3], a[g][1] + a[g][2]};
                    if (c > 0 && 2 * c < nx)
                        buf[lpad((q << ln) + nx - c)] = {a[g][0] + a[g][3], a[g][2] - a[g][1]};
                }
            }
        }
    }
    __syncthreads();
    fft_run<T, 1, FR>(buf, tw, ln, K * hb, false, NoLoad<T>(), false, NoStore<T>());
    const T scale = (T)(1.0 / ((double)nx * (double)ny));
    const uint32_t np = (uint32_t)I.n_pix;
    const size_t pl = (size_t)I.n_pix;
    GAS T *z = use_out ? gp(zout) : gp(Sel<T>::z(I));
    const GAS T *tp = gp(fscale<T>(I));
    constexpr int NB = blk_pairs<T, K>(), KP = K * (K + 1) / 2;
    const int items = hb << ln;
    for (int e0 = threadIdx.x; e0 < items; e0 += NB * kFT) {
        T tt[NB][2][KP];
#pragma unroll
        for (int g = 0; g < NB; ++g) {
            const int e = e0 + g * kFT;
            if (e < items) {
                const int qq = e >> ln, x = e & (nx - 1);
#pragma unroll
                for (int w = 0; w < 2; ++w) {
                    const uint32_t o = (uint32_t)(y0 + 2 * qq + w) * (uint32_t)nx + (uint32_t)x;
#pragma unroll
                    for (int t = 0; t < KP; ++t) tt[g][w][t] = bld(tp + t * pl, np, o);
                }
            }
        }
#pragma unroll
        for (int g = 0; g < NB; ++g) {
            const int e = e0 + g * kFT;
            if (e < items) {
                const int qq = e >> ln, x = e & (nx - 1);
                const int i = DCT ? cos_dst(x, nx) : x;
                Cx<T> zh[K];
#pragma unroll
                for (int a = 0; a < K; ++a) zh[a] = buf[lpad(((a * hb + qq) << ln) + i)];
#pragma unroll
                for (int w = 0; w < 2; ++w) {
                    const uint32_t o = (uint32_t)(y0 + 2 * qq + w) * (uint32_t)nx + (uint32_t)x;
#pragma unroll
                    for (int b = 0; b < K; ++b) {   // z_b = sum over a >= b of T[a][b] zhat_a
                        T sacc = (T)0;
#pragma unroll
                        for (int a = b; a < K; ++a)
                            sacc += tt[g][w][tidx(a, b)] * (w ? zh[a].y : zh[a].x);
                        bst(z + b * pl, np, o, sacc * scale);
                    }
                }
            }
        }
    }
}

// LDS bytes of a row pass over rb real rows of length nx (rb / 2 complex rows) and of the column
// pass (k components of length ny), stage tables included.
template <typename T>
size_t rows_lds(int nx, int rb) {
    return sizeof(Cx<T>) * ((size_t)nx + lds_entries(rb / 2 * nx));
}
template <typename T>
size_t cols_lds(int ny, int k, bool table = true) {
    return sizeof(Cx<T>) * ((table ? (size_t)ny : 0) + lds_entries(k * ny));
}

// Static LDS of the passes (the column pass's reduction table) kept free beside the dynamic part.
constexpr size_t kLdsMargin = 1024;

// Grid rows per workgroup of the block-scaled row passes (all k components of each row): two,
// so that a pass has twice the workgroups of four-row bands (two per CU at 1024^2, k = 3) whose
// loads and transforms overlap; measured faster than four-row bands despite 16-byte runs in the
// transposed spectrum (float32 1024^2, k = 3: forward 21.5 against 23.5 us, inverse 14.4 against
// 15.6 us).  0 when the k complex rows exceed kFftCap or, without the stage table, the LDS.
template <typename T>
size_t rows_lds_blk(int nx, int k, bool table) {
    return sizeof(Cx<T>) * ((table ? (size_t)nx : 0) + lds_entries(k * nx));
}
template <typename T>
int rows_per_block_blk(int nx, int ny, int k) {
    (void)ny;
    const bool fits = k * nx <= kFftCap && rows_lds_blk<T>(nx, k, false) <= kMaxLds - kLdsMargin;
    return fits ? 2 : 0;
}
// Whether the block-scaled row passes read their stage twiddles from global memory (the band and
// the table do not both fit in LDS; float64 only: 2048 columns at k = 4, 4096 at k = 2).
template <typename T>
bool blk_global_twiddles(int nx, int k) {
    return rows_lds_blk<T>(nx, k, true) > kMaxLds - kLdsMargin;
}

template <typename T>
int rows_per_block(int nx, int ny) {
    // runs of at least 64 bytes per column in the transposed stores, at most kFftCap complex
    // entries, and the LDS of the workgroup within the device's limit
    int rb = 64 / (int)sizeof(Cx<T>);
    rb = std::min(rb, 2 * kFftCap / nx);
    rb = std::min(rb, ny);
    while (rb > 2 && rows_lds<T>(nx, rb) > kMaxLds - kLdsMargin) rb /= 2;
    return std::max(rb, 2);
}


// One application z = Fourier preconditioner of r for every instance of the set, in precision T
// (float for the inner runs of the mixed path, double otherwise), DCT on face grids.  inner: 1 =
// the float32 inner runs of the mixed path (their r, z and state), 0 = the float64 runs, -1 = the
// stand-alone preconditioner (one instance, no run state): r read from rin, z written to zout.
// upd: see k_fp_rows_fwd (runs only).
// The kernels are instantiated per length class (fft_class); a pass is launched once per class
// present in the set (mask bit fp_radix_bit), and workgroups of other classes return at once.
template <typename F>
hipError_t for_each_class(int mask, F &&fn) {
    hipError_t e = hipSuccess;
    if ((mask & 1) && (e = fn(std::integral_constant<int, 2>())) != hipSuccess) return e;
    if ((mask & 2) && (e = fn(std::integral_constant<int, 4>())) != hipSuccess) return e;
    if ((mask & 4) && (e = fn(std::integral_constant<int, 8>())) != hipSuccess) return e;
    if ((mask & 8) && (e = fn(std::integral_constant<int, 16>())) != hipSuccess) return e;
    if ((mask & 16) && (e = fn(std::integral_constant<int, 110>())) != hipSuccess) return e;
    if ((mask & 32) && (e = fn(std::integral_constant<int, 111>())) != hipSuccess) return e;
    return e;
}

template <typename T, bool DCT>
hipError_t fp_apply_impl(const InstSet &set, int k, int inner, const void *rin, void *zout,
                         int upd, int it, hipStream_t s) {
    const int mixed = inner;
    const size_t lr = set.fp_lds_rows, lc = set.fp_lds_cols;
    return dispatch_k(k, [&](auto tag) -> hipError_t {
        constexpr int K = decltype(tag)::value;
        hipError_t e = for_each_class(set.fp_rmask_x, [&](auto fr) -> hipError_t {
            constexpr int FR = decltype(fr)::value;   // the class
            if (set.fp_block) {
                if (sizeof(T) == 8 && (set.fp_blk_gtw & cls_bit(FR))) {
                    // only float64 bands of k nx = 8192 with nx = 2048 (k = 4) or 4096 (k = 2)
                    if constexpr (sizeof(T) == 8 && ((FR == 111 && K == 4) || (FR == 16 && K == 2)))
                        hipLaunchKernelGGL((k_fp_rows_fwd_blk<T, K, FR, DCT, true>),
                                           dim3(set.total_fa), dim3(kFT), lr, s, set.table,
                                           set.fprefa, set.ninst, set.total_fa, mixed,
                                           reinterpret_cast<const T *>(rin), rin ? 1 : 0,
                                           inner >= 0 ? upd : 0, it);
                    else
                        return hipErrorInvalidValue;
                } else {
                    hipLaunchKernelGGL((k_fp_rows_fwd_blk<T, K, FR, DCT, false>),
                                       dim3(set.total_fa), dim3(kFT), lr, s, set.table,
                                       set.fprefa, set.ninst, set.total_fa, mixed,
                                       reinterpret_cast<const T *>(rin), rin ? 1 : 0,
                                       inner >= 0 ? upd : 0, it);
                }
            } else if (set.fp_scaled)
                hipLaunchKernelGGL((k_fp_rows_fwd<T, FR, DCT, true>), dim3(set.total_fa),
                                   dim3(kFT), lr, s, set.table, set.fprefa, set.ninst,
                                   set.total_fa, mixed, reinterpret_cast<const T *>(rin),
                                   rin ? 1 : 0, inner >= 0 ? upd : 0, it);
            else
                hipLaunchKernelGGL((k_fp_rows_fwd<T, FR, DCT, false>), dim3(set.total_fa),
                                   dim3(kFT), lr, s, set.table, set.fprefa, set.ninst,
                                   set.total_fa, mixed, reinterpret_cast<const T *>(rin),
                                   rin ? 1 : 0, inner >= 0 ? upd : 0, it);
            return hipGetLastError();
        });
        if (e != hipSuccess) return e;
        e = for_each_class(set.fp_rmask_y, [&](auto fr) -> hipError_t {
            constexpr int FR = decltype(fr)::value;   // the class
            const dim3 g(set.total_fb), b(kFT);
            if (sizeof(T) == 8 && (set.fp_cols_gtw & cls_bit(FR))) {
                // only float64 columns of k ny = 8192 with ny = 2048 (k <= 4) or 4096 (k <= 2)
                // exceed the LDS with their table (fp_cols_global_twiddles)
                if constexpr (sizeof(T) == 8 && ((FR == 111 && K <= 4) || (FR == 16 && K <= 2)))
                    hipLaunchKernelGGL((k_fp_cols<T, K, FR, true, DCT>), g, b, lc, s, set.table,
                                       set.fprefb, set.ninst, set.total_fb, mixed);
                else
                    return hipErrorInvalidValue;
            } else {
                hipLaunchKernelGGL((k_fp_cols<T, K, FR, false, DCT>), g, b, lc, s, set.table,
                                   set.fprefb, set.ninst, set.total_fb, mixed);
            }
            return hipGetLastError();
        });
        if (e != hipSuccess) return e;
        return for_each_class(set.fp_rmask_x, [&](auto fr) -> hipError_t {
            constexpr int FR = decltype(fr)::value;   // the class
            if (set.fp_block) {
                if (sizeof(T) == 8 && (set.fp_blk_gtw & cls_bit(FR))) {
                    if constexpr (sizeof(T) == 8 && ((FR == 111 && K == 4) || (FR == 16 && K == 2)))
                        hipLaunchKernelGGL((k_fp_rows_inv_blk<T, K, FR, DCT, true>),
                                           dim3(set.total_fa), dim3(kFT), lr, s, set.table,
                                           set.fprefa, set.ninst, set.total_fa, mixed,
                                           reinterpret_cast<T *>(zout), zout ? 1 : 0);
                    else
                        return hipErrorInvalidValue;
                } else {
                    hipLaunchKernelGGL((k_fp_rows_inv_blk<T, K, FR, DCT, false>),
                                       dim3(set.total_fa), dim3(kFT), lr, s, set.table,
                                       set.fprefa, set.ninst, set.total_fa, mixed,
                                       reinterpret_cast<T *>(zout), zout ? 1 : 0);
                }
            } else if (set.fp_scaled)
                hipLaunchKernelGGL((k_fp_rows_inv<T, FR, DCT, true>), dim3(set.total_fa),
                                   dim3(kFT), lr, s, set.table, set.fprefa, set.ninst,
                                   set.total_fa, mixed, reinterpret_cast<T *>(zout),
                                   zout ? 1 : 0);
            else
                hipLaunchKernelGGL((k_fp_rows_inv<T, FR, DCT, false>), dim3(set.total_fa),
                                   dim3(kFT), lr, s, set.table, set.fprefa, set.ninst,
                                   set.total_fa, mixed, reinterpret_cast<T *>(zout),
                                   zout ? 1 : 0);
            return hipGetLastError();
        });
    });
}

}  // namespace

// The four instantiations of fp_apply_impl, one per translation unit.
hipError_t fp_apply_f32_periodic(const InstSet &set, int k, int inner, const void *rin,
                                 void *zout, int upd, int it, hipStream_t s);
hipError_t fp_apply_f32_face(const InstSet &set, int k, int inner, const void *rin, void *zout,
                             int upd, int it, hipStream_t s);
hipError_t fp_apply_f64_periodic(const InstSet &set, int k, int inner, const void *rin,
                                 void *zout, int upd, int it, hipStream_t s);
hipError_t fp_apply_f64_face(const InstSet &set, int k, int inner, const void *rin, void *zout,
                             int upd, int it, hipStream_t s);

}  // namespace sylv
