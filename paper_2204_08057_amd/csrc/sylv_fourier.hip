// Fourier preconditioner of the CG solver: set-up (the pixel means of the noise weights, the
// per-mode symbol, the Laplacian eigenvalue, stage-twiddle and cosine-twiddle tables) and the
// host-side queries and dispatch.  The method and the kernels of the three passes of an
// application are described and defined in sylv_fourier_impl.h.

#include "sylv_fourier_impl.h"

namespace sylv {
namespace {

// Mean over pixels of every weight map, first stage: the workgroup partials of all kMaxF rows
// (zeros beyond f) in one reduction.  A workgroup sums kWChunk pixels, four consecutive pixels
// of every map per vector load (grids here have power-of-two sides, so n_pix is a multiple of 4).
constexpr int kWChunk = 4096;
__global__ __launch_bounds__(kBlock) void k_wmean_part(const double *__restrict__ W, int f,
                                                       int n_pix, double *__restrict__ part) {
    const int p0 = blockIdx.x * kWChunk;
    double v[kMaxF];
#pragma unroll
    for (int fi = 0; fi < kMaxF; ++fi) {
        double s = 0.0;
        if (fi < f) {
            const GAS double *w = gp(W) + (size_t)fi * n_pix;
            double a[kWChunk / (4 * kBlock)][4];
#pragma unroll
            for (int u = 0; u < kWChunk / (4 * kBlock); ++u) {
                const int p = p0 + (u * kBlock + threadIdx.x) * 4;
                if (p < n_pix) ld4(w + p, a[u]);
                else a[u][0] = a[u][1] = a[u][2] = a[u][3] = 0.0;
            }
#pragma unroll
            for (int u = 0; u < kWChunk / (4 * kBlock); ++u) s += (a[u][0] + a[u][1]) + (a[u][2] + a[u][3]);
        }
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

// Entry e of the stage table of a length-n transform, in float64 and float32.
__device__ void stage_entry(int n, int e, double *t64, float *t32) {
    const int logn = __builtin_ctz((unsigned)n);
    int off = 0;
    for (int lg = 0; lg < logn;) {
        const int lr = stage_log_radix(logn, lg);
        const int cnt = ((1 << lr) - 1) << lg;
        if (e < off + cnt) {
            const int ns = 1 << lg, rm1 = (e - off) >> lg, kk = (e - off) & (ns - 1);
            // W_(ns R)^(r kk) = exp(-2 pi i r kk / (ns R))
            double s, c;
            sincospi(-2.0 * (double)((rm1 + 1) * kk) / (double)(ns << lr), &s, &c);
            t64[2 * e] = c;
            t64[2 * e + 1] = s;
            t32[2 * e] = (float)c;
            t32[2 * e + 1] = (float)s;
            return;
        }
        off += cnt;
        lg += lr;
    }
}
// The Laplacian eigenvalue tables, the stage tables of both grid sides and, on face grids, the
// cosine twiddles: thread e of the grid writes entry e of lamx | lamy | stage table of nx |
// stage table of ny | cosine twiddles of nx | of ny.
__global__ __launch_bounds__(kBlock) void k_fp_tables(int nx, int ny, int face,
                                                      double *__restrict__ base) {
    const FpTabs tb = fp_tabs(nx, ny);
    // periodic: 2 - 2 cos(2 pi u / n); face: 2 - 2 cos(pi u / n)
    const double f = face ? 1.0 : 2.0;
    int e = blockIdx.x * kBlock + threadIdx.x;
    if (e < nx) {
        base[tb.lamx + e] = 2.0 - 2.0 * cospi(f * (double)e / (double)nx);
        return;
    }
    e -= nx;
    if (e < ny) {
        base[tb.lamy + e] = 2.0 - 2.0 * cospi(f * (double)e / (double)ny);
        return;
    }
    e -= ny;
    if (e < nx - 1) {
        stage_entry(nx, e, base + tb.twx64, reinterpret_cast<float *>(base + tb.twx32));
        return;
    }
    e -= nx - 1;
    if (e < ny - 1) {
        stage_entry(ny, e, base + tb.twy64, reinterpret_cast<float *>(base + tb.twy32));
        return;
    }
    e -= ny - 1;
    if (!face) return;
    const bool x = e < nx;
    const int n = x ? nx : ny, u = x ? e : e - nx;
    if (u >= n) return;
    double sn, cs;   // exp(-i pi u / 2n)
    sincospi(-(double)u / (2.0 * n), &sn, &cs);
    double *t64 = base + (x ? tb.ctx64 : tb.cty64);
    float *t32 = reinterpret_cast<float *>(base + (x ? tb.ctx32 : tb.cty32));
    t64[2 * u] = cs;
    t64[2 * u + 1] = sn;
    t32[2 * u] = (float)cs;
    t32[2 * u + 1] = (float)sn;
}

// Diagonal scale of SYLV_PC_FOURIER_DIAG: thread e of the grid writes 1 / s for pixel p = e % n_pix
// of component j = e / n_pix, s^2 = diag(G) / diag(Q + I (x) Mbar).  diag(Q_j) at p is
// tau_j ((kappa_j^2 + d_p)^2 + d_p), the diagonal of (kappa_j^2 I + L)^2 for the grid Laplacian L
// with d_p neighbours (4 on periodic grids, whose sides here are at least 4; 2 to 4 on a face);
// diag(G) adds the pixel's mixing block entry M_p[j][j], diag(Q + I (x) Mbar) adds Mbar[j][j].
__global__ __launch_bounds__(kBlock) void k_fp_scale(const double *__restrict__ M64,
                                                     const double *__restrict__ fsym, int k,
                                                     int nx, int ny, int face,
                                                     double *__restrict__ sc64,
                                                     float *__restrict__ sc32) {
    const int n_pix = nx * ny;
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= k * n_pix) return;
    const int j = e / n_pix, p = e - j * n_pix;
    const int y = p / nx, x = p - y * nx;
    const double d = face ? (double)((x > 0) + (x < nx - 1) + (y > 0) + (y < ny - 1)) : 4.0;
    const double kap2 = fsym[kMaxK * kMaxK + j], tau = fsym[kMaxK * kMaxK + kMaxK + j];
    const double t = kap2 + d;
    const double dq = tau * (t * t + d);
    const int jj = j * k - (j * (j - 1)) / 2;   // packed index of (j, j)
    const double dg = dq + M64[(size_t)jj * n_pix + p];
    const double dm = dq + fsym[j * kMaxK + j];
    const double v = sqrt(dm / dg);
    if (sc64) sc64[e] = v;   // a solve writes the one precision its runs read
    if (sc32) sc32[e] = (float)v;
}

// Block scale of SYLV_PC_FOURIER_BLOCK: thread p of the grid forms pixel p's k x k blocks of G,
// Bp = diag(dq) + M_p, and of Q + I (x) Mbar, B0 = diag(dq) + Mbar (dq_j the prior's diagonal as
// in k_fp_scale), their Cholesky factors Lp and L0, and writes T = L0 Lp^-1 (lower triangular,
// packed at tidx(a, b)) in float64 and float32 (either pointer may be null).
template <int K>
__global__ __launch_bounds__(kBlock) void k_fp_tscale(const double *__restrict__ M64,
                                                      const double *__restrict__ fsym, int nx,
                                                      int ny, int face, double *__restrict__ sc64,
                                                      float *__restrict__ sc32) {
    const int n_pix = nx * ny;
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= n_pix) return;
    const int y = p / nx, x = p - y * nx;
    const double d = face ? (double)((x > 0) + (x < nx - 1) + (y > 0) + (y < ny - 1)) : 4.0;
    double lp[K][K], l0[K][K];
#pragma unroll
    for (int a = 0; a < K; ++a) {
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const double m = M64[(size_t)pidx<K>(a, b) * n_pix + p];
            const double mb = fsym[a * kMaxK + b];
            double dq = 0.0;
            if (a == b) {
                const double t = fsym[kMaxK * kMaxK + a] + d;
                dq = fsym[kMaxK * kMaxK + kMaxK + a] * (t * t + d);
            }
            lp[a][b] = m + dq;
            l0[a][b] = mb + dq;
        }
    }
    // Cholesky factors in place (lower triangles)
#pragma unroll
    for (int j = 0; j < K; ++j) {
#pragma unroll
        for (int m = 0; m < j; ++m) {
            lp[j][j] -= lp[j][m] * lp[j][m];
            l0[j][j] -= l0[j][m] * l0[j][m];
        }
        lp[j][j] = sqrt(lp[j][j]);
        l0[j][j] = sqrt(l0[j][j]);
#pragma unroll
        for (int i = j + 1; i < K; ++i) {
#pragma unroll
            for (int m = 0; m < j; ++m) {
                lp[i][j] -= lp[i][m] * lp[j][m];
                l0[i][j] -= l0[i][m] * l0[j][m];
            }
            lp[i][j] /= lp[j][j];
            l0[i][j] /= l0[j][j];
        }
    }
    // Lp^-1 by forward substitution, column by column (lower triangle)
    double li[K][K];
#pragma unroll
    for (int b = 0; b < K; ++b) {
#pragma unroll
        for (int a = 0; a < K; ++a) {
            if (a < b) continue;
            double v = a == b ? 1.0 : 0.0;
#pragma unroll
            for (int m = b; m < a; ++m) v -= lp[a][m] * li[m][b];
            li[a][b] = v / lp[a][a];
        }
    }
    // T = L0 Lp^-1
#pragma unroll
    for (int a = 0; a < K; ++a) {
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            double v = 0.0;
#pragma unroll
            for (int m = b; m <= a; ++m) v += l0[a][m] * li[m][b];
            const size_t o = (size_t)tidx(a, b) * n_pix + p;
            if (sc64) sc64[o] = v;   // a solve writes the one precision its runs read
            if (sc32) sc32[o] = (float)v;
        }
    }
}

}  // namespace

int fp_rows_per_block(int nx, int ny, int dtype) {
    return dtype == SYLV_F64 ? rows_per_block<double>(nx, ny) : rows_per_block<float>(nx, ny);
}

int fp_rows_per_block_blk(int nx, int ny, int k, int dtype) {
    return dtype == SYLV_F64 ? rows_per_block_blk<double>(nx, ny, k)
                             : rows_per_block_blk<float>(nx, ny, k);
}

bool fp_blk_global_twiddles(int nx, int k, int dtype) {
    return dtype == SYLV_F64 ? blk_global_twiddles<double>(nx, k) : blk_global_twiddles<float>(nx, k);
}

size_t fp_lds_bytes_blk(int nx, int k, int dtype, bool gtw) {
    return dtype == SYLV_F64 ? rows_lds_blk<double>(nx, k, !gtw) : rows_lds_blk<float>(nx, k, !gtw);
}

bool fp_supported(int ny, int nx, int k, int dtype, char *why, size_t why_len) {
    auto pow2 = [](int v) { return v >= 4 && v <= 4096 && (v & (v - 1)) == 0; };
    if (!pow2(nx) || !pow2(ny)) {
        snprintf(why, why_len, "the Fourier preconditioner needs grid sides that are powers of two "
                 "in [4, 4096] (grid %d x %d)", ny, nx);
        return false;
    }
    const bool f64 = dtype == SYLV_F64;
    const size_t cols = f64 ? cols_lds<double>(ny, k, false) : cols_lds<float>(ny, k, false);
    if (k * ny > kFftCap || cols > kMaxLds - kLdsMargin) {
        snprintf(why, why_len, "the Fourier preconditioner's column pass holds the k x ny complex "
                 "values of a column in LDS: at most %d of them, %zu bytes (k = %d, ny = %d, %s)",
                 kFftCap, (size_t)(kMaxLds - kLdsMargin), k, ny, f64 ? "float64" : "float32");
        return false;
    }
    const int rb = fp_rows_per_block(nx, ny, dtype);
    const size_t rows = f64 ? rows_lds<double>(nx, rb) : rows_lds<float>(nx, rb);
    if (rows > kMaxLds - kLdsMargin) {
        snprintf(why, why_len, "the Fourier preconditioner's row pass needs %zu bytes of LDS "
                 "(nx = %d, %s)", rows, nx, f64 ? "float64" : "float32");
        return false;
    }
    return true;
}

size_t fp_table_bytes(int nx, int ny) { return sizeof(double) * fp_tabs(nx, ny).total; }

hipError_t launch_fp_setup(const double *W, const double *A, int f, int k, int nx, int ny,
                           int face, const double *coef, double *part, double *fsym,
                           const double *M64, int scale, double *sc64, float *sc32,
                           hipStream_t s) {
    const int n_pix = nx * ny;
    const int nblk = (int)blocks_for(n_pix, kWChunk);
    hipLaunchKernelGGL(k_wmean_part, dim3(nblk), dim3(kBlock), 0, s, W, f, n_pix, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fp_symbol, dim3(1), dim3(kBlock), 0, s, part, nblk, A, f, k, n_pix,
                       coef, fsym);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int nt = nx + ny + (nx - 1) + (ny - 1) + (face ? nx + ny : 0);
    hipLaunchKernelGGL(k_fp_tables, dim3((nt + kBlock - 1) / kBlock), dim3(kBlock), 0, s, nx, ny,
                       face, fsym);
    if ((e = hipGetLastError()) != hipSuccess || !scale) return e;
    if (scale == 2)
        return dispatch_k(k, [&](auto tag) {
            constexpr int K = decltype(tag)::value;
            hipLaunchKernelGGL((k_fp_tscale<K>), dim3((n_pix + kBlock - 1) / kBlock), dim3(kBlock),
                               0, s, M64, fsym, nx, ny, face, sc64, sc32);
            return hipGetLastError();
        });
    const int ns = k * n_pix;
    hipLaunchKernelGGL(k_fp_scale, dim3((ns + kBlock - 1) / kBlock), dim3(kBlock), 0, s, M64, fsym,
                       k, nx, ny, face, sc64, sc32);
    return hipGetLastError();
}

size_t fp_setup_partials(int n_pix, int f) {
    (void)f;
    return (size_t)blocks_for(n_pix, kWChunk) * kMaxF;
}

bool fp_cols_global_twiddles(int ny, int k, int dtype) {
    const size_t b = dtype == SYLV_F64 ? cols_lds<double>(ny, k) : cols_lds<float>(ny, k);
    return b > kMaxLds - kLdsMargin;
}

size_t fp_lds_bytes(int pass, int n, int m, int dtype) {
    // pass 0: a row pass over m rows of length n; pass 1: the column pass, m components of
    // length n (without the stage table when it is read from global memory)
    if (!pass) return dtype == SYLV_F64 ? rows_lds<double>(n, m) : rows_lds<float>(n, m);
    const bool table = !fp_cols_global_twiddles(n, m, dtype);
    return dtype == SYLV_F64 ? cols_lds<double>(n, m, table) : cols_lds<float>(n, m, table);
}

hipError_t launch_fp_apply(const InstSet &set, int k, int f32, int inner, const void *rin,
                           void *zout, int upd, int it, hipStream_t s) {
    const bool face = set.bc == SYLV_BC_FACE;   // face grids: cosine transforms
    if (f32)
        return face ? fp_apply_f32_face(set, k, inner, rin, zout, upd, it, s)
                    : fp_apply_f32_periodic(set, k, inner, rin, zout, upd, it, s);
    return face ? fp_apply_f64_face(set, k, inner, rin, zout, upd, it, s)
                : fp_apply_f64_periodic(set, k, inner, rin, zout, upd, it, s);
}

int fp_radix_bit(int logn) { return cls_bit(fft_class(logn)); }

}  // namespace sylv
