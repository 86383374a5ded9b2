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
//      <r, z> partial by Parseval's identity, inverse FFT along y, back into S;
//   C  per row: the full row spectrum from the half (Hermitian symmetry of a real row), inverse
//      FFT (length nx), the real part scaled by 1 / (nx ny) into z.
// Every FFT is a Stockham radix-4 (radix-2 for an odd power) transform in LDS with a twiddle table
// computed per workgroup from sincospi in float64.  T = float for the inner runs of the mixed
// path, double for float64 runs.

#include "sylv_device.h"

#include <stdio.h>

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
// a * conj(b)
template <typename T>
__device__ __forceinline__ Cx<T> cmulc(Cx<T> a, Cx<T> b) {
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

// LDS index with one padding slot per 32 entries (breaks the power-of-two strides of the
// Stockham stores across banks).
__device__ __forceinline__ int lpad(int i) { return i + (i >> 5); }
__host__ __device__ constexpr int lds_entries(int n) { return n + (n >> 5) + 1; }

// tw[m] = exp(-2 pi i m / n) for m in [0, n/2); W^m for m >= n/2 is -tw[m - n/2].
template <typename T>
__device__ __forceinline__ void make_twiddles(Cx<T> *tw, int n) {
    for (int m = threadIdx.x; m < n / 2; m += kBlock) {
        double s, c;
        sincospi(-2.0 * (double)m / (double)n, &s, &c);
        tw[m] = {(T)c, (T)s};
    }
}
template <typename T>
__device__ __forceinline__ Cx<T> twiddle(const Cx<T> *tw, int idx, int n) {
    idx &= n - 1;
    const int h = n >> 1;
    if (idx < h) return tw[idx];
    const Cx<T> w = tw[idx - h];
    return {-w.x, -w.y};
}

// In-place FFTs of `rows` sequences of length n (a power of two, 2 <= n <= 4096) held at
// buf[lpad(row * n + i)], rows * n <= MT * 4 * kBlock.  INV = 1: the inverse transform
// (conjugate twiddles), unnormalised.  Stockham autosort: each stage first reads the butterfly
// inputs of all of the thread's tasks into registers (statically indexed), then, after a
// barrier, writes the outputs in sorted order.
template <typename T, int INV, int MT>
__device__ void fft_lds(Cx<T> *buf, const Cx<T> *tw, int n, int logn, int rows) {
    int ns = 1;
    for (int lg = 0; lg < logn;) {
        const bool r4 = logn - lg >= 2;
        const int radix = r4 ? 4 : 2;
        const int m = n / radix;                      // tasks per row
        const int ntask = rows * m;
        const int tstep = n / (ns * radix);           // W_(ns radix)^(r kk) = W_n^(r kk tstep)
        Cx<T> v[4 * MT];
        if (r4) {
#pragma unroll
            for (int q = 0; q < MT; ++q) {
                const int t = threadIdx.x + q * kBlock;
                if (t >= ntask) break;
                const int row = t / m, j = t - row * m, kk = j & (ns - 1);
                const int base = row * n + j;
                Cx<T> a[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    a[r] = buf[lpad(base + r * m)];
                    if (r > 0 && kk > 0) {
                        Cx<T> w = twiddle(tw, r * kk * tstep, n);
                        if (INV) w.y = -w.y;
                        a[r] = cmul(a[r], w);
                    }
                }
                const Cx<T> s0 = cadd(a[0], a[2]), d0 = csub(a[0], a[2]);
                const Cx<T> s1 = cadd(a[1], a[3]), e = csub(a[1], a[3]);
                const Cx<T> d1 = INV ? Cx<T>{-e.y, e.x} : Cx<T>{e.y, -e.x};   // e * (-+i)
                v[4 * q + 0] = cadd(s0, s1);
                v[4 * q + 1] = cadd(d0, d1);
                v[4 * q + 2] = csub(s0, s1);
                v[4 * q + 3] = csub(d0, d1);
            }
        } else {
#pragma unroll
            for (int q = 0; q < 2 * MT; ++q) {
                const int t = threadIdx.x + q * kBlock;
                if (t >= ntask) break;
                const int row = t / m, j = t - row * m, kk = j & (ns - 1);
                const int base = row * n + j;
                const Cx<T> a0 = buf[lpad(base)];
                Cx<T> a1 = buf[lpad(base + m)];
                if (kk > 0) {
                    Cx<T> w = twiddle(tw, kk * tstep, n);
                    if (INV) w.y = -w.y;
                    a1 = cmul(a1, w);
                }
                v[2 * q] = cadd(a0, a1);
                v[2 * q + 1] = csub(a0, a1);
            }
        }
        __syncthreads();
        if (r4) {
#pragma unroll
            for (int q = 0; q < MT; ++q) {
                const int t = threadIdx.x + q * kBlock;
                if (t >= ntask) break;
                const int row = t / m, j = t - row * m, kk = j & (ns - 1);
                const int dst = row * n + (j - kk) * 4 + kk;
#pragma unroll
                for (int r = 0; r < 4; ++r) buf[lpad(dst + r * ns)] = v[4 * q + r];
            }
        } else {
#pragma unroll
            for (int q = 0; q < 2 * MT; ++q) {
                const int t = threadIdx.x + q * kBlock;
                if (t >= ntask) break;
                const int row = t / m, j = t - row * m, kk = j & (ns - 1);
                const int dst = row * n + (j - kk) * 2 + kk;
                buf[lpad(dst)] = v[2 * q];
                buf[lpad(dst + ns)] = v[2 * q + 1];
            }
        }
        __syncthreads();
        ns *= radix;
        lg += r4 ? 2 : 1;
    }
}

// Register budget of the transforms: complex entries per workgroup (rows x n or k x ny) at most
// 4 * kBlock * MT; MT = 4 in float64 (4096 entries, 64 KB), 8 in float32 (8192 entries).
template <typename T>
constexpr int fft_mt() { return sizeof(T) == 8 ? 4 : 8; }

// The half spectrum S[j][c][y] of an instance: complex T as (re, im) pairs (the buffer holds
// complex float64), accessed entry by entry.
template <typename T>
__device__ __forceinline__ GAS T *spectrum(const Inst &I) {
    return reinterpret_cast<GAS T *>(gp(I.fs));
}
template <typename T>
__device__ __forceinline__ Cx<T> sload(const GAS T *S, size_t i) {
    return {S[2 * i], S[2 * i + 1]};
}
template <typename T>
__device__ __forceinline__ void sstore(GAS T *S, size_t i, Cx<T> v) {
    S[2 * i] = v.x;
    S[2 * i + 1] = v.y;
}

// Pass A: forward FFT of rows y0 .. y0 + rb of component j of r, half spectrum stored
// transposed: S[j][c][y], c in [0, nx/2].
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fp_rows_fwd(const Inst *__restrict__ tab,
                                                        const int *__restrict__ fpre, int ninst,
                                                        int nb, int inner,
                                                        const T *__restrict__ rin, int use_in) {
    extern __shared__ __align__(16) unsigned char fp_lds[];
    const int L = xcd_remap(blockIdx.x, nb);
    const int ii = find_inst(fpre, ninst, L);
    const Inst &I = tab[ii];
    if (inner >= 0 && (inner ? I.st_in : I.st)->done) return;   // inner < 0: stand-alone
    const int blk = L - fpre[ii];
    const int nx = I.nx, ny = I.ny, rb = I.frb, nc = nx / 2 + 1;
    const int nrb = ny / rb;
    const int j = blk / nrb, y0 = (blk - j * nrb) * rb;
    Cx<T> *tw = reinterpret_cast<Cx<T> *>(fp_lds);
    Cx<T> *buf = tw + nx / 2;
    make_twiddles<T>(tw, nx);
    const GAS T *r = (use_in ? gp(rin) : (const GAS T *)Sel<T>::r(I)) + (size_t)j * I.n_pix;
    const uint32_t np = (uint32_t)I.n_pix;
    for (int e = threadIdx.x; e < rb * nx; e += kBlock)
        buf[lpad(e)] = {bld(r, np, (uint32_t)((y0 + e / nx) * nx + (e % nx))), (T)0};
    __syncthreads();
    fft_lds<T, 0, fft_mt<T>()>(buf, tw, nx, I.lognx, rb);
    GAS T *S = spectrum<T>(I) + (size_t)2 * j * nc * ny;
    for (int e = threadIdx.x; e < rb * nc; e += kBlock) {
        const int c = e / rb, yy = e - c * rb;
        sstore(S, (size_t)c * ny + y0 + yy, buf[lpad(yy * nx + c)]);
    }
}

// Pass B: column c of the half spectrum for every component: forward FFT along y, the per-mode
// k x k solve, the <r, z> partial (Parseval: each c in (0, nx/2) stands for itself and its
// conjugate partner), inverse FFT along y.
template <typename T, int K>
__global__ __launch_bounds__(kBlock) void k_fp_cols(const Inst *__restrict__ tab,
                                                    const int *__restrict__ fpre, int ninst,
                                                    int nb, int inner) {
    extern __shared__ __align__(16) unsigned char fp_lds[];
    const int L = xcd_remap(blockIdx.x, nb);
    const int ii = find_inst(fpre, ninst, L);
    const Inst &I = tab[ii];
    if (inner >= 0 && (inner ? I.st_in : I.st)->done) return;   // inner < 0: stand-alone
    const int c = L - fpre[ii];
    const int nx = I.nx, ny = I.ny, nc = nx / 2 + 1;
    Cx<T> *tw = reinterpret_cast<Cx<T> *>(fp_lds);
    Cx<T> *buf = tw + ny / 2;
    make_twiddles<T>(tw, ny);
    GAS T *S = spectrum<T>(I);
    for (int e = threadIdx.x; e < K * ny; e += kBlock) {
        const int j = e / ny, y = e - j * ny;
        buf[lpad(e)] = sload(S, ((size_t)j * nc + c) * ny + y);
    }
    __syncthreads();
    fft_lds<T, 0, fft_mt<T>()>(buf, tw, ny, I.logny, K);
    // per-mode blocks: diag_j tau_j (kappa_j^2 + lam)^2 + Mbar, lam = lx + 4 - 2 cos(2 pi v/ny)
    const double *fd = I.fsym;   // [kMaxK * kMaxK] Mbar, then kappa^2 [kMaxK], tau [kMaxK]
    double mb[K][K], k2[K], ta[K];
#pragma unroll
    for (int a = 0; a < K; ++a) {
        k2[a] = fd[kMaxK * kMaxK + a];
        ta[a] = fd[kMaxK * kMaxK + kMaxK + a];
#pragma unroll
        for (int b = 0; b < K; ++b) mb[a][b] = fd[a * kMaxK + b];
    }
    double cx, sxu;
    sincospi(2.0 * (double)c / (double)nx, &sxu, &cx);
    const double lx = 2.0 - 2.0 * cx;
    const double wc = (c == 0 || 2 * c == nx) ? 1.0 : 2.0;
    double rz = 0.0;
    for (int v = threadIdx.x; v < ny; v += kBlock) {
        const double lam = lx + 2.0 - 2.0 * (double)twiddle(tw, v, ny).x;
        T g[K][K];
#pragma unroll
        for (int a = 0; a < K; ++a)
#pragma unroll
            for (int b = 0; b < K; ++b) {
                double e = mb[a][b];
                if (a == b) {
                    const double s = k2[a] + lam;
                    e += ta[a] * s * s;
                }
                g[a][b] = (T)e;
            }
        // Cholesky g = l l^T (lower), then two triangular solves for the real and imaginary parts
#pragma unroll
        for (int a = 0; a < K; ++a) {
            T d = g[a][a];
#pragma unroll
            for (int q = 0; q < a; ++q) d -= g[a][q] * g[a][q];
            d = sqrt(d);
            g[a][a] = d;
#pragma unroll
            for (int b = a + 1; b < K; ++b) {
                T s = g[b][a];
#pragma unroll
                for (int q = 0; q < a; ++q) s -= g[b][q] * g[a][q];
                g[b][a] = s / d;
            }
        }
        Cx<T> rh[K], zh[K];
#pragma unroll
        for (int a = 0; a < K; ++a) rh[a] = buf[lpad(a * ny + v)];
#pragma unroll
        for (int a = 0; a < K; ++a) {
            Cx<T> s = rh[a];
#pragma unroll
            for (int q = 0; q < a; ++q) { s.x -= g[a][q] * zh[q].x; s.y -= g[a][q] * zh[q].y; }
            zh[a] = {s.x / g[a][a], s.y / g[a][a]};
        }
#pragma unroll
        for (int a = K - 1; a >= 0; --a) {
            Cx<T> s = zh[a];
#pragma unroll
            for (int q = a + 1; q < K; ++q) { s.x -= g[q][a] * zh[q].x; s.y -= g[q][a] * zh[q].y; }
            zh[a] = {s.x / g[a][a], s.y / g[a][a]};
        }
#pragma unroll
        for (int a = 0; a < K; ++a) {
            rz += wc * ((double)rh[a].x * (double)zh[a].x + (double)rh[a].y * (double)zh[a].y);
            buf[lpad(a * ny + v)] = zh[a];
        }
    }
    __syncthreads();
    fft_lds<T, 1, fft_mt<T>()>(buf, tw, ny, I.logny, K);
    for (int e = threadIdx.x; e < K * ny; e += kBlock) {
        const int j = e / ny, y = e - j * ny;
        sstore(S, ((size_t)j * nc + c) * ny + y, buf[lpad(e)]);
    }
    // <r, z> = rz / (nx ny): the partial of this column (none for the stand-alone application)
    if (I.partial) {
        double v1[1] = {rz / ((double)nx * (double)ny)};
        block_partials<1>(v1, I.partial, I.nred, SLOT_FRZ, c);
    }
}

// Pass C: rows y0 .. y0 + rb of component j: the full spectrum of each row from the half
// (X[nx - c] = conj(X[c])), inverse FFT, z = real part / (nx ny).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fp_rows_inv(const Inst *__restrict__ tab,
                                                        const int *__restrict__ fpre, int ninst,
                                                        int nb, int inner, T *__restrict__ zout,
                                                        int use_out) {
    extern __shared__ __align__(16) unsigned char fp_lds[];
    const int L = xcd_remap(blockIdx.x, nb);
    const int ii = find_inst(fpre, ninst, L);
    const Inst &I = tab[ii];
    if (inner >= 0 && (inner ? I.st_in : I.st)->done) return;   // inner < 0: stand-alone
    const int blk = L - fpre[ii];
    const int nx = I.nx, ny = I.ny, rb = I.frb, nc = nx / 2 + 1;
    const int nrb = ny / rb;
    const int j = blk / nrb, y0 = (blk - j * nrb) * rb;
    Cx<T> *tw = reinterpret_cast<Cx<T> *>(fp_lds);
    Cx<T> *buf = tw + nx / 2;
    make_twiddles<T>(tw, nx);
    const GAS T *S = spectrum<T>(I) + (size_t)2 * j * nc * ny;
    for (int e = threadIdx.x; e < rb * nc; e += kBlock) {
        const int c = e / rb, yy = e - c * rb;
        const Cx<T> v = sload(S, (size_t)c * ny + y0 + yy);
        buf[lpad(yy * nx + c)] = v;
        if (c > 0 && 2 * c < nx) buf[lpad(yy * nx + nx - c)] = {v.x, -v.y};
    }
    __syncthreads();
    fft_lds<T, 1, fft_mt<T>()>(buf, tw, nx, I.lognx, rb);
    const T scale = (T)(1.0 / ((double)nx * (double)ny));
    GAS T *z = use_out ? gp(zout) : gp(Sel<T>::z(I));
    z += (size_t)j * I.n_pix;
    const uint32_t np = (uint32_t)I.n_pix;
    for (int e = threadIdx.x; e < rb * nx; e += kBlock)
        bst(z, np, (uint32_t)((y0 + e / nx) * nx + (e % nx)), buf[lpad(e)].x * scale);
}

// Mean over pixels of every weight map, first stage: the workgroup partials of all kMaxF rows
// (zeros beyond f) in one reduction.
__global__ __launch_bounds__(kBlock) void k_wmean_part(const double *__restrict__ W, int f,
                                                       int n_pix, double *__restrict__ part) {
    const int p0 = blockIdx.x * kChunk;
    double v[kMaxF];
#pragma unroll
    for (int fi = 0; fi < kMaxF; ++fi) {
        double s = 0.0;
        if (fi < f)
            for (int e = threadIdx.x; e < kChunk; e += kBlock)
                if (p0 + e < n_pix) s += W[(size_t)fi * n_pix + p0 + e];
        v[fi] = s;
    }
    block_partials<kMaxF>(v, part, (int)gridDim.x, 0, blockIdx.x);
}

// Mbar = sum_f mean(W[f]) a_f a_f^T, kappa_j^2 and tau_j into the symbol block (one workgroup).
__global__ __launch_bounds__(kBlock) void k_fp_symbol(const double *__restrict__ part, int nblk,
                                                      const double *__restrict__ A, int f,
                                                      int k, int n_pix,
                                                      const double *__restrict__ coef,
                                                      double *__restrict__ fsym) {
    double v[kMaxF];
    consume<kMaxF>(part, nblk, 0, nblk, v);
    if (threadIdx.x < kMaxK * kMaxK) {
        const int a = threadIdx.x / kMaxK, b = threadIdx.x % kMaxK;
        double s = 0.0;
        if (a < k && b < k)
            for (int fi = 0; fi < f; ++fi)
                s += (v[fi] / (double)n_pix) * A[fi * k + a] * A[fi * k + b];
        fsym[threadIdx.x] = s;
    }
    if (threadIdx.x < kMaxK) {
        const int j = threadIdx.x;
        const double kap = j < k ? coef[j * kCoefStride + 5] : 0.0;
        fsym[kMaxK * kMaxK + j] = kap * kap;
        fsym[kMaxK * kMaxK + kMaxK + j] = j < k ? coef[j * kCoefStride + 6] : 0.0;
    }
}

template <typename T>
size_t rows_lds(int nx, int rb) {
    return sizeof(Cx<T>) * ((size_t)nx / 2 + lds_entries(rb * nx));
}
template <typename T>
size_t cols_lds(int ny, int k) {
    return sizeof(Cx<T>) * ((size_t)ny / 2 + lds_entries(k * ny));
}

}  // namespace

int fp_rows_per_block(int nx, int ny, int dtype) {
    const int budget = dtype == SYLV_F64 ? 2048 : 4096;   // complex entries per workgroup
    const int rb = nx >= budget ? 1 : budget / nx;
    return rb < ny ? rb : ny;
}

bool fp_supported(int ny, int nx, int k, int dtype, char *why, size_t why_len) {
    auto pow2 = [](int v) { return v >= 4 && v <= 4096 && (v & (v - 1)) == 0; };
    if (!pow2(nx) || !pow2(ny)) {
        snprintf(why, why_len, "the Fourier preconditioner needs grid sides that are powers of two "
                 "in [4, 4096] (grid %d x %d)", ny, nx);
        return false;
    }
    const size_t es = dtype == SYLV_F64 ? sizeof(Cx<double>) : sizeof(Cx<float>);
    const int cap = dtype == SYLV_F64 ? 4 * kBlock * fft_mt<double>() : 4 * kBlock * fft_mt<float>();
    if (k * ny > cap || es * ((size_t)ny / 2 + lds_entries(k * ny)) > 65536) {
        snprintf(why, why_len, "the Fourier preconditioner's column pass holds k x ny complex "
                 "values in 64 KB of LDS: too many in %s (k = %d, ny = %d)",
                 dtype == SYLV_F64 ? "float64" : "float32", k, ny);
        return false;
    }
    return true;
}

hipError_t launch_fp_setup(const double *W, const double *A, int f, int k, int n_pix,
                           const double *coef, double *part, double *fsym, hipStream_t s) {
    const int nblk = (int)blocks_for(n_pix, kChunk);
    hipLaunchKernelGGL(k_wmean_part, dim3(nblk), dim3(kBlock), 0, s, W, f, n_pix, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fp_symbol, dim3(1), dim3(kBlock), 0, s, part, nblk, A, f, k, n_pix,
                       coef, fsym);
    return hipGetLastError();
}

size_t fp_setup_partials(int n_pix, int f) {
    (void)f;
    return (size_t)blocks_for(n_pix, kChunk) * kMaxF;
}

// One application z = Fourier preconditioner of r for every instance of the set, in float32 (f32)
// or float64.  inner: 1 = the float32 inner runs of the mixed path (their r, z and state), 0 = the
// float64 runs, -1 = the stand-alone preconditioner (one instance, no run state): r read from
// rin, z written to zout.
size_t fp_lds_bytes(int pass, int n, int m, int dtype) {
    // pass 0: a row pass over m rows of length n; pass 1: the column pass, m components of
    // length n
    return dtype == SYLV_F64 ? (pass ? cols_lds<double>(n, m) : rows_lds<double>(n, m))
                             : (pass ? cols_lds<float>(n, m) : rows_lds<float>(n, m));
}

hipError_t launch_fp_apply(const InstSet &set, int k, int f32, int inner, const void *rin,
                           void *zout, hipStream_t s) {
    const int mixed = inner;
    return dispatch_k(k, [&](auto tag) -> hipError_t {
        constexpr int K = decltype(tag)::value;
        auto run = [&](auto tt) -> hipError_t {
            using T = decltype(tt);
            const size_t lr = set.fp_lds_rows, lc = set.fp_lds_cols;
            hipLaunchKernelGGL((k_fp_rows_fwd<T>), dim3(set.total_fa), dim3(kBlock), lr, s,
                               set.table, set.fprefa, set.ninst, set.total_fa, mixed,
                               reinterpret_cast<const T *>(rin), rin ? 1 : 0);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_fp_cols<T, K>), dim3(set.total_fb), dim3(kBlock), lc, s,
                               set.table, set.fprefb, set.ninst, set.total_fb, mixed);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL((k_fp_rows_inv<T>), dim3(set.total_fa), dim3(kBlock), lr, s,
                               set.table, set.fprefa, set.ninst, set.total_fa, mixed,
                               reinterpret_cast<T *>(zout), zout ? 1 : 0);
            return hipGetLastError();
        };
        return f32 ? run(0.0f) : run(0.0);
    });
}

}  // namespace sylv
