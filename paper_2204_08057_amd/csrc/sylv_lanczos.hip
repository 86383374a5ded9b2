// Lanczos-Sylvester kernels (Section 3.3): the symmetric block Lanczos process for N^-1 D2 in the
// N inner product (Alg. 4) and the device side of the symmetric sparse Sylvester solver around
// it (Alg. 5).  One Lanczos step i is one pass over the grid and a two-stage reduction:
//
//   k_lz_stencil<STEP>  stages Wa_(i-1) and V_(i-1) (tile + 2-pixel periodic halo) and forms, per
//                       staged pixel, the orthogonalised block of the previous step
//                       W_(i-1) = Wa_(i-1) - V_(i-1) H_(i-1) and its Cholesky-QR normalisation
//                       V_i = W_(i-1) B_i^-1 in LDS; stores V_i (basis block i) and
//                       Wa_i = N^-1 D2 V_i - V_(i-1) B_i^T (13-point stencil of (kappa^2 - Lap)^2),
//                       with the partials of P = V_i^T N Wa_i, C = V_i^T N V_i, E = Wa_i^T N Wa_i;
//   k_lz_reduce         one workgroup per reduced quantity: the fixed-order sum of the partials;
//   k_lz_fin            H_i = sym(P) (Alg. 4), the N-Gram matrix of W_i = Wa_i - V_i H_i by the
//                       exact expansion W_i^T N W_i = E - P^T H_i - H_i P + H_i C H_i (no
//                       orthogonality assumed), its Cholesky factor B_(i+1) and inverse, and
//                       Alg. 5's residual estimate gamma, carried by a block forward elimination of
//                       T_i + rho_l I (one thread per eigenvalue rho_l of Lhat) instead of an
//                       eigendecomposition of T_i per step; the stopping test.
//
// Evaluating the Gram matrix by the expansion lets W_i live only in registers of the next pass,
// so a step moves (4k + 1) planes instead of materialising W, orthogonalising it and reading it
// again.  The blocks V_i stay in the workspace, so the approximation M = sum_i V_i G_i is one
// streaming pass over them (k_lz_assemble) once the host has solved the small projected equation
// for the G_i, instead of the paper's second Lanczos pass.  A last stencil pass recomputes the
// residual of eq. (Axb).  All reductions sum per-workgroup partials in a fixed order, so results
// are bitwise repeatable.

#include "sylv_device.h"

namespace sylv {
namespace {

using namespace dev;

enum { LZ_STEP = 0, LZ_RESID = 1 };

__device__ __forceinline__ const double *cblk(const double *base, int i) {
    return base + (size_t)i * kLzStride;
}
__device__ __forceinline__ double *wblk(double *base, int i) { return base + (size_t)i * kLzStride; }
// Workspace slot of basis block i (0-based): one slot per step when the blocks are kept, two
// alternating slots when the solution is assembled by a second Lanczos pass.
__device__ __forceinline__ size_t lz_slot(const LzArgs &a, int i) {
    return a.ring ? (size_t)(i & 1) : (size_t)i;
}

template <int K>
constexpr int lz_nv_step() { return K * K + K * (K + 1); }   // P, C, E
template <int K>
constexpr int lz_nv_start() { return K * (K + 1) / 2 + 1; }  // Gram of Yhat, invalid-n count

// Workgroup-reduce one value per thread (fixed order) into slot `e` of the LDS table.
__device__ __forceinline__ void put_wave(double v, double (*sm)[kBlock / 64], int e) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sm[e][threadIdx.x >> 6] = v;
}
template <int NV>
__device__ __forceinline__ void store_partials(double (*sm)[kBlock / 64], double *partial,
                                               int nred, int blkid) {
    __syncthreads();
    for (int i = threadIdx.x; i < NV; i += kBlock)
        gp(partial)[(size_t)i * nred + blkid] = (sm[i][0] + sm[i][1]) + (sm[i][2] + sm[i][3]);
}

// Workgroup partials of NV values per thread through LDS (red: at least CH * (kBlock + 16)
// doubles, free on entry): in chunks of CH values every thread stores its values, then 16 threads
// per value sum 16 strided entries each and one thread per value sums those 16 (fixed order).
// Partial v of the workgroup goes to partial[v * nred + blkid].
template <int NV, int CH>
__device__ __forceinline__ void lds_partials(const double (&vals)[NV], double *red,
                                             double *partial, int nred, int blkid) {
    static_assert(CH * 16 <= kBlock, "16 threads per value of a chunk");
    double *red2 = red + CH * kBlock;
    const int tid = threadIdx.x;
#pragma unroll
    for (int c0 = 0; c0 < NV; c0 += CH) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < CH; ++i)
            if (c0 + i < NV) red[i * kBlock + tid] = vals[c0 + i];
        __syncthreads();
        if (tid < CH * 16) {
            const int i = tid >> 4, g = tid & 15;
            double s = 0.0;
#pragma unroll
            for (int u = 0; u < kBlock / 16; ++u) s += red[i * kBlock + u * 16 + g];
            red2[i * 16 + g] = s;
        }
        __syncthreads();
        if (tid < CH && c0 + tid < NV) {
            double s = 0.0;
#pragma unroll
            for (int g = 0; g < 16; ++g) s += red2[tid * 16 + g];
            gp(partial)[(size_t)(c0 + tid) * nred + blkid] = s;
        }
    }
}

// Packed upper-triangle index e -> (r, q), r <= q.
template <int K>
__device__ __forceinline__ void unpack(int e, int &r, int &q) {
    r = 0;
    while (e >= K - r) { e -= K - r; ++r; }
    q = r + e;
}

// ---- small dense helpers (one thread) -------------------------------------------------------

// Upper Cholesky factor of the symmetric K x K matrix g (g = R^T R).  False if a pivot is not
// positive or not finite.
template <int K>
__device__ bool chol_upper(const double (&g)[K][K], double (&r)[K][K]) {
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j) r[i][j] = 0.0;
    for (int i = 0; i < K; ++i) {
        double d = g[i][i];
        for (int a = 0; a < i; ++a) d -= r[a][i] * r[a][i];
        if (!(d > 0.0) || !isfinite(d)) return false;
        const double rii = sqrt(d);
        r[i][i] = rii;
        for (int j = i + 1; j < K; ++j) {
            double v = g[i][j];
            for (int a = 0; a < i; ++a) v -= r[a][i] * r[a][j];
            r[i][j] = v / rii;
        }
    }
    return true;
}

// Inverse of an upper triangular K x K matrix.
template <int K>
__device__ void inv_upper(const double (&r)[K][K], double (&ri)[K][K]) {
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j) ri[i][j] = 0.0;
    for (int j = 0; j < K; ++j) {
        ri[j][j] = 1.0 / r[j][j];
        for (int i = j - 1; i >= 0; --i) {
            double v = 0.0;
            for (int a = i + 1; a <= j; ++a) v += r[i][a] * ri[a][j];
            ri[i][j] = -v / r[i][i];
        }
    }
}

// x = S^-1 b for a symmetric positive definite S given by its upper Cholesky factor r.
template <int K>
__device__ void chol_solve(const double (&r)[K][K], const double (&b)[K], double (&x)[K]) {
    double y[K];
    for (int i = 0; i < K; ++i) {        // r^T y = b
        double v = b[i];
        for (int a = 0; a < i; ++a) v -= r[a][i] * y[a];
        y[i] = v / r[i][i];
    }
    for (int i = K - 1; i >= 0; --i) {   // r x = y
        double v = y[i];
        for (int a = i + 1; a < K; ++a) v -= r[i][a] * x[a];
        x[i] = v / r[i][i];
    }
}

// ---- kernels ---------------------------------------------------------------------------------

__global__ void k_lz_init(LzArgs a, int max_iter) {
    if (threadIdx.x == 0) {
        LzState *st = a.st;
        st->nb0 = 0.0; st->thresh = 0.0; st->gamma = 0.0; st->rr = 0.0; st->bb = 0.0;
        st->iter = 0; st->done = 0; st->status = SYLV_OK; st->max_iter = max_iter;
    }
}

// Start block Yhat = Y^T T A P^-1 (eq. (Axb-Sylv)) into Yh, with the partials of its N-Gram
// matrix (packed upper triangle) and a count of invalid n_p.
template <int K>
__global__ __launch_bounds__(kBlock) void k_lz_start(LzArgs a) {
    const int chunk = xcd_remap(blockIdx.x, a.nchunks);
    const int n_pix = a.n_pix, f = a.f;
    const LzConst *c = a.c;
    const GAS double *n = gp(a.n);
    const GAS double *Y = gp(a.Y);
    double yh[4][K], wt[4];
    double bad = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int p = chunk * kChunk + e * kBlock + threadIdx.x;
        wt[e] = 0.0;
#pragma unroll
        for (int j = 0; j < K; ++j) yh[e][j] = 0.0;
        if (p < n_pix) {
            const double nv = n[p];
            if (!(nv > 0.0) || !isfinite(nv)) bad += 1.0;
            wt[e] = nv;
            for (int fi = 0; fi < f; ++fi) {
                const double y = Y[(size_t)fi * n_pix + p];
#pragma unroll
                for (int j = 0; j < K; ++j) yh[e][j] += y * c->tap[j][fi];
            }
#pragma unroll
            for (int j = 0; j < K; ++j) gp(a.Yh)[(size_t)j * n_pix + p] = yh[e][j];
        }
    }
    constexpr int NV = lz_nv_start<K>();
    __shared__ double sm[NV][kBlock / 64];
    int e = 0;
#pragma unroll
    for (int r = 0; r < K; ++r)
#pragma unroll
        for (int q = r; q < K; ++q, ++e) {
            double v = 0.0;
#pragma unroll
            for (int t = 0; t < 4; ++t) v += wt[t] * (yh[t][r] * yh[t][q]);
            put_wave(v, sm, e);
        }
    put_wave(bad, sm, NV - 1);
    store_partials<NV>(sm, a.partial, a.nred, chunk);
}

// Stencil kernels.  STEP: one Lanczos step (see the file comment).  RESID: residual of eq. (Axb)
// for X: r_j = n_p tau_j Yhat_j - (tau_j D2 X_j + n_p (A^T T A X_p)_j), with the partials of
// ||r||^2 and ||b||^2.
// replay = 1 (STEP only): step `it` of the second Lanczos pass of Alg. 5, which regenerates V_i
// from the kept H and B blocks (the same instructions as the first pass, so V_i is bitwise the
// same) and adds V_i G_(i-1) into X instead of forming Gram partials.
template <int K, int MODE, int R, int BC>
__global__ __launch_bounds__(kBlock) void k_lz_stencil(LzArgs a, int it, int replay) {
    constexpr int LH = kWavesY * R + 4;   // staged rows: tile + 2-row halo above and below
    constexpr int LW = kTileX + 4;        // staged columns
    constexpr int RPW = LH / kWavesY;     // staged rows per wavefront
    constexpr bool STEP = MODE == LZ_STEP;
    const LzState *st = a.st;
    if (STEP && !replay && st->done) return;
    const bool prev = STEP && it > 1;     // a previous block exists
    const int tile = xcd_remap(blockIdx.x, a.ntiles);
    const int nx = a.nx, ny = a.ny, n_pix = a.n_pix;
    const uint32_t np = (uint32_t)n_pix;   // plane length for buffer accesses
    const LzConst *c = a.c;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int tile_x = tile % a.tiles_x, tile_y = tile / a.tiles_x;
    const int x0 = tile_x * kTileX, y0 = tile_y * kWavesY * R;
    const int ix = x0 + tx;
    const int iy0 = y0 + ty * R;
    const bool active = (ix < nx) && (iy0 < ny);

    // ---- issue the global loads: staged fields, then per-output-pixel data -----------------
    const double *src0;                     // STEP: Wa_(i-1) (Yhat at i = 1); RESID: X
    if constexpr (STEP) src0 = (it == 1) ? a.Yh : ((it & 1) ? a.Wa1 : a.Wa0);
    else src0 = a.X;
    const GAS double *vprev = gp(a.basis) + (prev ? lz_slot(a, it - 2) : 0) * K * n_pix;
    const int cmain = wrapf(x0 + tx, nx);
    const int hitem = ty * 64 + tx;
    const int hr = hitem >> 2, hc = hitem & 3;
    const int hcol = (hc < 2) ? hc : (kTileX + hc);
    const bool hvalid = hitem < 4 * LH;
    const uint32_t hoff = hvalid ? (uint32_t)(wrapf(y0 - 2 + hr, ny) * nx + wrapf(x0 - 2 + hcol, nx)) : 0u;
    uint32_t soff[RPW];
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr)
        soff[rr] = (uint32_t)(wrapf(y0 - 2 + rr * kWavesY + ty, ny) * nx + cmain);
    // face grids: staged positions outside the face hold 0 (absent neighbours)
    bool sin[RPW];
    bool hin = hvalid;
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) sin[rr] = true;
    if constexpr (BC == BC_FACE) {
        const bool colin = x0 + tx < nx;
#pragma unroll
        for (int rr = 0; rr < RPW; ++rr) {
            const int ry = y0 - 2 + rr * kWavesY + ty;
            sin[rr] = colin && ry >= 0 && ry < ny;
        }
        const int hy = y0 - 2 + hr, hx = x0 - 2 + hcol;
        hin = hvalid && hy >= 0 && hy < ny && hx >= 0 && hx < nx;
    }
    double sa[K][RPW], ha[K], sv[K][RPW], hv[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const GAS double *s = gp(src0) + (size_t)j * n_pix;
#pragma unroll
        for (int rr = 0; rr < RPW; ++rr) sa[j][rr] = sin[rr] ? bld(s, np, soff[rr]) : 0.0;
        ha[j] = hin ? bld(s, np, hoff) : 0.0;
        if (prev) {
            const GAS double *v = vprev + (size_t)j * n_pix;
#pragma unroll
            for (int rr = 0; rr < RPW; ++rr) sv[j][rr] = sin[rr] ? bld(v, np, soff[rr]) : 0.0;
            hv[j] = hin ? bld(v, np, hoff) : 0.0;
        } else {
#pragma unroll
            for (int rr = 0; rr < RPW; ++rr) sv[j][rr] = 0.0;
            hv[j] = 0.0;
        }
    }
    const int ixc = ix < nx ? ix : 0;
    double nv[R], aux[R][K];
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const int pix = (iy0 + t < ny ? iy0 + t : 0) * nx + ixc;
        nv[t] = bld(gp(a.n), np, (uint32_t)pix);
#pragma unroll
        for (int j = 0; j < K; ++j) aux[t][j] = 0.0;
        if (prev) {          // V_(i-1) at the output pixels (just staged: served by L2)
#pragma unroll
            for (int j = 0; j < K; ++j) aux[t][j] = bld(vprev + (size_t)j * n_pix, np, (uint32_t)pix);
        } else if (MODE == LZ_RESID) {
#pragma unroll
            for (int j = 0; j < K; ++j) aux[t][j] = bld(gp(a.Yh) + (size_t)j * n_pix, np, (uint32_t)pix);
        }
    }

    // ---- stage the field in LDS (STEP: V_i = (Wa_(i-1) - V_(i-1) H_(i-1)) B_i^-1) ------------
    __shared__ double lds[K][LH][LW];
    const double *Bi = STEP ? cblk(a.B, it - 1) : nullptr;
    const double *Binv = STEP ? cblk(a.Binv, it - 1) : nullptr;
    const double *Hp = prev ? cblk(a.H, it - 2) : nullptr;
#pragma unroll
    for (int rr = 0; rr <= RPW; ++rr) {
        if (rr == RPW && !hvalid) break;
        const int row = (rr < RPW) ? rr * kWavesY + ty : hr;
        const int col = (rr < RPW) ? tx + 2 : hcol;
        if constexpr (STEP) {
            double w[K];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                double v = (rr < RPW) ? sa[j][rr] : ha[j];
                if (prev) {
#pragma unroll
                    for (int q = 0; q < K; ++q) v -= ((rr < RPW) ? sv[q][rr] : hv[q]) * Hp[q * kMaxK + j];
                }
                w[j] = v;
            }
#pragma unroll
            for (int j = 0; j < K; ++j) {
                double v = 0.0;
#pragma unroll
                for (int q = 0; q <= j; ++q) v += w[q] * Binv[q * kMaxK + j];
                lds[j][row][col] = v;
            }
        } else {
#pragma unroll
            for (int j = 0; j < K; ++j) lds[j][row][col] = (rr < RPW) ? sa[j][rr] : ha[j];
        }
    }
    __syncthreads();

    // ---- 13-point stencil of (kappa^2 - Lap)^2 from LDS --------------------------------------
    const double c0 = c->coef[0], c1 = c->coef[1], cd = c->coef[2], c2 = c->coef[3];
    const double k2 = c->kappa2;
    double uo[R][K], wo[R][K], wt[R];
    double d0 = 0.0, d1 = 0.0;
#pragma unroll
    for (int t = 0; t < R; ++t) {
        wt[t] = 0.0;
#pragma unroll
        for (int j = 0; j < K; ++j) { uo[t][j] = 0.0; wo[t][j] = 0.0; }
    }
    if (active) {
        const int lr = ty * R;
        double acc[K][R], ctr[K][R];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            double cc[R + 4], l1[R + 2], r1[R + 2], l2[R], r2[R];
#pragma unroll
            for (int t = 0; t < R + 4; ++t) cc[t] = lds[j][lr + t][tx + 2];
#pragma unroll
            for (int t = 0; t < R + 2; ++t) {
                l1[t] = lds[j][lr + t + 1][tx + 1];
                r1[t] = lds[j][lr + t + 1][tx + 3];
            }
#pragma unroll
            for (int t = 0; t < R; ++t) {
                l2[t] = lds[j][lr + t + 2][tx];
                r2[t] = lds[j][lr + t + 2][tx + 4];
            }
#pragma unroll
            for (int t = 0; t < R; ++t) {
                const double d4 = (l1[t] + r1[t]) + (l1[t + 2] + r1[t + 2]);
                const double f4 = (cc[t] + cc[t + 4]) + (l2[t] + r2[t]);
                if constexpr (BC == BC_FACE) {
                    // (kappa^2 + d_p)^2 + d_p at the centre, -(2 kappa^2 + d_p + d_q) at edge
                    // neighbour q (absent neighbours are staged as 0)
                    const int iy = iy0 + t;
                    const double dp = (double)face_deg(ix, iy, nx, ny);
                    const double e0 = k2 + dp, b0 = 2.0 * k2 + dp;
                    const double en = (b0 + face_deg(ix, iy - 1, nx, ny)) * cc[t + 1] +
                                      (b0 + face_deg(ix, iy + 1, nx, ny)) * cc[t + 3] +
                                      (b0 + face_deg(ix - 1, iy, nx, ny)) * l1[t + 1] +
                                      (b0 + face_deg(ix + 1, iy, nx, ny)) * r1[t + 1];
                    acc[j][t] = (e0 * e0 + dp) * cc[t + 2] - en + cd * d4 + c2 * f4;
                } else {
                    const double n4 = (cc[t + 1] + cc[t + 3]) + (l1[t + 1] + r1[t + 1]);
                    acc[j][t] = c0 * cc[t + 2] + c1 * n4 + cd * d4 + c2 * f4;
                }
                ctr[j][t] = cc[t + 2];
            }
        }
#pragma unroll
        for (int t = 0; t < R; ++t) {
            if (iy0 + t >= ny) continue;
            const int pix = (iy0 + t) * nx + ix;
            if constexpr (STEP) {
                GAS double *vb = gp(a.basis) + lz_slot(a, it - 1) * K * n_pix;
                GAS double *wa = gp((it & 1) ? a.Wa0 : a.Wa1);
                const double ninv = 1.0 / nv[t];
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    double w = acc[j][t] * ninv;
                    if (prev) {
#pragma unroll
                        for (int q = 0; q < K; ++q) w -= aux[t][q] * Bi[j * kMaxK + q];
                    }
                    bst(vb + (size_t)j * n_pix, np, (uint32_t)pix, ctr[j][t]);
                    bst(wa + (size_t)j * n_pix, np, (uint32_t)pix, w);
                    uo[t][j] = ctr[j][t];
                    wo[t][j] = w;
                }
                wt[t] = nv[t];
                if (replay) {   // M += V_i G_(i-1) (M = V_1 G_0 at the first step)
                    const double *Gs = cblk(a.G, it - 1);
                    GAS double *xo = gp(a.X);
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        double m = (it > 1) ? bld(xo + (size_t)j * n_pix, np, (uint32_t)pix) : 0.0;
#pragma unroll
                        for (int q = 0; q < K; ++q) m += ctr[q][t] * Gs[q * kMaxK + j];
                        bst(xo + (size_t)j * n_pix, np, (uint32_t)pix, m);
                    }
                }
            } else {
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    double mix = 0.0;
#pragma unroll
                    for (int q = 0; q < K; ++q) mix += c->ata[j][q] * ctr[q][t];
                    const double gx = c->tau[j] * acc[j][t] + nv[t] * mix;
                    const double bj = nv[t] * (c->tau[j] * aux[t][j]);
                    const double r = bj - gx;
                    d0 += r * r;
                    d1 += bj * bj;
                }
            }
        }
    }
    if constexpr (STEP) {
        if (replay) return;
        constexpr int NV = lz_nv_step<K>();
        double vals[NV];
        int e = 0;
#pragma unroll
        for (int r = 0; r < K; ++r)          // P = V^T N Wa (full)
#pragma unroll
            for (int q = 0; q < K; ++q, ++e) {
                double v = 0.0;
#pragma unroll
                for (int t = 0; t < R; ++t) v += wt[t] * (uo[t][r] * wo[t][q]);
                vals[e] = v;
            }
#pragma unroll
        for (int r = 0; r < K; ++r)          // C = V^T N V (packed)
#pragma unroll
            for (int q = r; q < K; ++q, ++e) {
                double v = 0.0;
#pragma unroll
                for (int t = 0; t < R; ++t) v += wt[t] * (uo[t][r] * uo[t][q]);
                vals[e] = v;
            }
#pragma unroll
        for (int r = 0; r < K; ++r)          // E = Wa^T N Wa (packed)
#pragma unroll
            for (int q = r; q < K; ++q, ++e) {
                double v = 0.0;
#pragma unroll
                for (int t = 0; t < R; ++t) v += wt[t] * (wo[t][r] * wo[t][q]);
                vals[e] = v;
            }
        // the staging buffer is free once every wavefront has finished its stencil reads
        // (lds_partials starts with a barrier); a chunk of CH values needs CH * (kBlock + 16)
        // doubles of it and 16 threads per value
        constexpr int CH0 = (3 * K < 16) ? 3 * K : 16;
        constexpr int CH = (CH0 < NV) ? CH0 : NV;
        static_assert(CH * (kBlock + 16) <= K * LH * LW, "reduction scratch exceeds LDS");
        static_assert(CH * 16 <= kBlock, "one workgroup sums at most kBlock / 16 values at once");
        lds_partials<NV, CH>(vals, &lds[0][0][0], a.partial, a.nred, tile);
    } else {
        __shared__ double sm[2][kBlock / 64];
        put_wave(d0, sm, 0);
        put_wave(d1, sm, 1);
        store_partials<2>(sm, a.partial, a.nred, tile);
    }
}

// Reduction of a pass's workgroup partials: workgroup i sums slot i over all blocks in a fixed
// order (every thread's loads issued before any is summed) into partial2[i].
__global__ __launch_bounds__(kBlock) void k_lz_reduce(LzArgs a, int nblocks) {
    const int i = blockIdx.x;
    const GAS double *pp = gp(a.partial) + (size_t)i * a.nred;
    double s = 0.0;
    int b = threadIdx.x;
    for (; b + 7 * kBlock < nblocks; b += 8 * kBlock) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = pp[b + u * kBlock];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; b < nblocks; b += kBlock) s += pp[b];
    __shared__ double sm[1][kBlock / 64];
    put_wave(s, sm, 0);
    __syncthreads();
    if (threadIdx.x == 0) gp(a.partial2)[i] = (sm[0][0] + sm[0][1]) + (sm[0][2] + sm[0][3]);
}

// Cholesky-QR of the running block in the N inner product, W^T N W = B^T B with B upper.
//   it == 0: the start block Yhat: B_0; ||B_0||_F sets the stopping threshold, and column l of
//            B_0 U starts the forward elimination of column l.
//   it >= 1: H_i and the Gram matrix of W_i from P, C, E (see the file comment), B_(i+1), then
//            Alg. 5's residual estimate and the stopping test.
// The estimate: Q F e_l = (T_i + rho_l I)^-1 E_1 B_0 U e_l (eq. (soln-constr)), and gamma is
// sum_l ||B_(i+1) x_l||^2 with x_l the last block of that vector.  With the Schur complements
// S_1 = H_1 + rho_l I, S_j = H_j + rho_l I - B_j S_(j-1)^-1 B_j^T and y_1 = B_0 U e_l,
// y_j = -B_j S_(j-1)^-1 y_(j-1) (block elimination of the block tridiagonal T_i + rho_l I), that
// last block is x_l = S_i^-1 y_i; each step extends the elimination by one block.
template <int K>
__global__ __launch_bounds__(kBlock) void k_lz_fin(LzArgs a, int it) {
    LzState *st = a.st;
    if (st->done) return;
    constexpr int PK = K * (K + 1) / 2;
    constexpr int kCol0 = 64;    // the column threads form the second wavefront, so that their
                                 // elimination runs beside thread 0's Cholesky-QR
    const int tid = threadIdx.x;
    __shared__ double sP[K][K], sH[K][K], sC[K][K], sE[K][K], sCH[K][K], sG[K][K], sBn[K][K];
    __shared__ double s_bad, s_gam[K];
    __shared__ int s_ok;         // 0: B valid; 1: zero block; 2: not positive definite; 3: bad
    // column threads of the residual estimate: prefetch their elimination state and B_i
    const int l = tid - kCol0;
    const bool col = it >= 1 && l >= 0 && l < K;
    double Sprev[K][K], yv[K], Bj[K][K];
    if (col) {
#pragma unroll
        for (int r = 0; r < K; ++r) {
            yv[r] = st->y[l][r];
#pragma unroll
            for (int q = 0; q < K; ++q) {
                Sprev[r][q] = (it > 1) ? st->S[l][r][q] : 0.0;
                Bj[r][q] = (it > 1) ? cblk(a.B, it - 1)[r * kMaxK + q] : 0.0;
            }
        }
    }
    const double *p2 = a.partial2;
    if (it == 0) {
        if (tid < PK) {
            int r, q;
            unpack<K>(tid, r, q);
            sG[r][q] = p2[tid];
            sG[q][r] = p2[tid];
        } else if (tid == PK) {
            s_bad = p2[PK];
        }
        __syncthreads();
    } else {
        // P (full), C and E (packed): H = sym(P); W^T N W = E - P^T H - H P + H C H
        if (tid < K * K) {
            sP[tid / K][tid % K] = p2[tid];
        } else if (tid < K * K + PK) {
            int r, q;
            unpack<K>(tid - K * K, r, q);
            sC[r][q] = p2[tid];
            sC[q][r] = p2[tid];
        } else if (tid < K * K + 2 * PK) {
            int r, q;
            unpack<K>(tid - K * K - PK, r, q);
            sE[r][q] = p2[tid];
            sE[q][r] = p2[tid];
        }
        __syncthreads();
        const int r = tid / K, q = tid % K;
        if (tid < K * K) sH[r][q] = 0.5 * (sP[r][q] + sP[q][r]);
        __syncthreads();
        if (tid < K * K) {
            double v = 0.0;
#pragma unroll
            for (int s2 = 0; s2 < K; ++s2) v += sC[r][s2] * sH[s2][q];
            sCH[r][q] = v;
        }
        __syncthreads();
        if (tid < K * K) {
            double v = sE[r][q];
#pragma unroll
            for (int s2 = 0; s2 < K; ++s2)
                v += -sP[s2][r] * sH[s2][q] - sH[r][s2] * sP[s2][q] + sH[r][s2] * sCH[s2][q];
            sG[r][q] = v;
            wblk(a.H, it - 1)[r * kMaxK + q] = sH[r][q];
        }
        __syncthreads();
    }
    // thread 0: Cholesky-QR of the block.  Column threads (meanwhile): extend the elimination
    // of T_i + rho_l I by H_i and solve for its last block x_l.
    double xl[K];
    bool xok = true;
    if (tid == 0) {
        double G[K][K], Bm[K][K], Bi[K][K];
        bool zero = true, fin = true;
        for (int r = 0; r < K; ++r)
            for (int q = 0; q < K; ++q) {
                G[r][q] = 0.5 * (sG[r][q] + sG[q][r]);
                zero = zero && G[r][q] == 0.0;
                fin = fin && isfinite(G[r][q]) && (it == 0 || isfinite(sH[r][q]));
            }
        const double bad = (it == 0) ? s_bad : 0.0;
        int ok = 0;
        if (it == 0 && bad > 0.0) ok = 3;
        else if (!fin) ok = 3;
        else if (zero) ok = 1;
        else if (!chol_upper<K>(G, Bm)) ok = 2;
        double *Bo = wblk(a.B, it), *Bio = wblk(a.Binv, it);
        if (ok == 0) {
            inv_upper<K>(Bm, Bi);
        } else {
            for (int r = 0; r < K; ++r)
                for (int q = 0; q < K; ++q) { Bm[r][q] = 0.0; Bi[r][q] = 0.0; }
        }
        for (int r = 0; r < K; ++r)
            for (int q = 0; q < K; ++q) {
                Bo[r * kMaxK + q] = Bm[r][q];
                Bio[r * kMaxK + q] = Bi[r][q];
                sBn[r][q] = Bm[r][q];
            }
        if (it == 0) {
            double nb = 0.0;
            for (int r = 0; r < K; ++r)
                for (int q = 0; q < K; ++q) nb += Bm[r][q] * Bm[r][q];
            st->nb0 = sqrt(nb);
            st->thresh = a.c->tol * sqrt(nb);
            for (int c = 0; c < K; ++c)          // y_1 for column c: B_0 U e_c
                for (int r = 0; r < K; ++r) {
                    double v = 0.0;
                    for (int q = 0; q < K; ++q) v += Bm[r][q] * a.c->U[q][c];
                    st->y[c][r] = v;
                }
            if (ok != 0) {                        // zero start block: X = 0; invalid n_p / values
                st->status = (ok == 1) ? SYLV_OK : (bad > 0.0 ? SYLV_BAD_INPUT : SYLV_NONFINITE);
                st->iter = 0;
                st->gamma = 0.0;
                st->done = 1;
            }
        }
        s_ok = ok;
    } else if (col) {
        const double rho = a.c->rho[l];
        double S[K][K], y[K];
#pragma unroll
        for (int r = 0; r < K; ++r) y[r] = yv[r];
        if (it == 1) {
            for (int r = 0; r < K; ++r)
                for (int q = 0; q < K; ++q) S[r][q] = sH[r][q] + (r == q ? rho : 0.0);
        } else {
            double Ro[K][K];
            chol_upper<K>(Sprev, Ro);              // S_(i-1) is positive definite
            // X = S_(i-1)^-1 B_i^T column by column; S_i = H_i + rho I - B_i X
            double X[K][K];
            for (int q = 0; q < K; ++q) {
                double bcol[K], xcol[K];
                for (int r = 0; r < K; ++r) bcol[r] = Bj[q][r];   // column q of B_i^T
                chol_solve<K>(Ro, bcol, xcol);
                for (int r = 0; r < K; ++r) X[r][q] = xcol[r];
            }
            for (int r = 0; r < K; ++r)
                for (int q = 0; q < K; ++q) {
                    double v = sH[r][q] + (r == q ? rho : 0.0);
                    for (int s2 = 0; s2 < K; ++s2) v -= Bj[r][s2] * X[s2][q];
                    S[r][q] = v;
                }
            for (int r = 0; r < K; ++r)           // symmetrise against rounding
                for (int q = r + 1; q < K; ++q) {
                    const double m = 0.5 * (S[r][q] + S[q][r]);
                    S[r][q] = m;
                    S[q][r] = m;
                }
            double z[K];
            chol_solve<K>(Ro, yv, z);
            for (int r = 0; r < K; ++r) {
                double v = 0.0;
                for (int q = 0; q < K; ++q) v -= Bj[r][q] * z[q];
                y[r] = v;
            }
        }
        double Rs[K][K];
        if (chol_upper<K>(S, Rs)) chol_solve<K>(Rs, y, xl);
        else xok = false;
        for (int r = 0; r < K; ++r) {
            st->y[l][r] = y[r];
            for (int q = 0; q < K; ++q) st->S[l][r][q] = S[r][q];
        }
    }
    __syncthreads();
    if (it == 0) return;
    const int ok = s_ok;
    if (ok == 2 || ok == 3) {
        if (tid == 0) {
            st->status = (ok == 2) ? SYLV_BREAKDOWN : SYLV_NONFINITE;
            st->iter = (ok == 2) ? it : it - 1;
            st->gamma = -1.0;
            a.hist[it - 1] = -1.0;
            st->done = 1;
        }
        return;
    }
    if (col) {                                    // gamma_l = ||B_(i+1) x_l||^2
        double gl = 0.0;
        if (xok) {
            for (int r = 0; r < K; ++r) {
                double v = 0.0;
                for (int q = r; q < K; ++q) v += sBn[r][q] * xl[q];
                gl += v * v;
            }
        } else {
            gl = __builtin_nan("");
        }
        s_gam[l] = gl;
    }
    __syncthreads();
    if (tid == 0) {
        double gam = 0.0;
        for (int c = 0; c < K; ++c) gam += s_gam[c];
        st->gamma = gam;
        st->iter = it;
        a.hist[it - 1] = sqrt(gam) / st->nb0;
        if (!isfinite(gam)) {
            st->status = SYLV_NONFINITE;
            st->done = 1;
        } else if (ok == 1 || sqrt(gam) <= st->thresh) {
            st->status = SYLV_OK;
            st->done = 1;
        } else if (it >= st->max_iter) {
            st->status = SYLV_NOT_CONVERGED;
            st->done = 1;
        }
    }
}

// Running flag for the host: 1 while the solve has not finished (written to pinned memory).
__global__ void k_lz_flag(const LzState *st, int *host) {
    if (threadIdx.x == 0) host[0] = st->done ? 0 : 1;
}

// M = sum_s V_(s+1) G_s over the kept blocks, written to X.
template <int K>
__global__ __launch_bounds__(kBlock) void k_lz_assemble(LzArgs a, int iters) {
    const int chunk = xcd_remap(blockIdx.x, a.nchunks);
    const int n_pix = a.n_pix;
    double acc[4][K];
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int j = 0; j < K; ++j) acc[e][j] = 0.0;
    const int pb = chunk * kChunk + threadIdx.x;
    for (int s = 0; s < iters; ++s) {
        const double *Gs = cblk(a.G, s);
        const GAS double *Vs = gp(a.basis) + (size_t)s * K * n_pix;
        double v[4][K];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int p = pb + e * kBlock;
#pragma unroll
            for (int q = 0; q < K; ++q) v[e][q] = (p < n_pix) ? Vs[(size_t)q * n_pix + p] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int j = 0; j < K; ++j) {
                double sum = acc[e][j];
#pragma unroll
                for (int q = 0; q < K; ++q) sum += v[e][q] * Gs[q * kMaxK + j];
                acc[e][j] = sum;
            }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int p = pb + e * kBlock;
        if (p >= n_pix) continue;
#pragma unroll
        for (int j = 0; j < K; ++j) gp(a.X)[(size_t)j * n_pix + p] = acc[e][j];
    }
}

// ||b - G x||^2 and ||b||^2 from the residual pass (after the first reduction stage).
__global__ void k_lz_rfin(LzArgs a) {
    if (threadIdx.x == 0) {
        a.st->rr = a.partial2[0];
        a.st->bb = a.partial2[1];
    }
}

// Final sums of the NV slots of a pass with `nblocks` workgroup partials, into partial2[0, NV).
hipError_t launch_reduce(const LzArgs &a, int nv, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_lz_reduce, dim3(nv), dim3(kBlock), 0, s, a, nblocks);
    return hipGetLastError();
}

}  // namespace

int lz_tiles(int ny, int nx, int rows) {
    const int tx = (nx + kTileX - 1) / kTileX;
    const int ty = (ny + kWavesY * rows - 1) / (kWavesY * rows);
    return tx * ty;
}

int lz_rows_valid(int k, int rows) { return rows == 2 || (rows == 4 && k <= 4); }

hipError_t lz_launch_init(const LzArgs &a, int max_iter, hipStream_t s) {
    hipLaunchKernelGGL(k_lz_init, dim3(1), dim3(64), 0, s, a, max_iter);
    return hipGetLastError();
}

hipError_t lz_launch_start(const LzArgs &a, hipStream_t s) {
    return dispatch_k(a.k, [&](auto kt) -> hipError_t {
        constexpr int K = decltype(kt)::value;
        hipLaunchKernelGGL((k_lz_start<K>), dim3(a.nchunks), dim3(kBlock), 0, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if ((e = launch_reduce(a, lz_nv_start<K>(), a.nchunks, s)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_lz_fin<K>), dim3(1), dim3(kBlock), 0, s, a, 0);
        return hipGetLastError();
    });
}

// The step kernel of the first (replay = 0) or second (replay = 1) Lanczos pass.
static hipError_t launch_step_kernel(const LzArgs &a, int it, int replay, hipStream_t s) {
    return dispatch_k(a.k, [&](auto kt) -> hipError_t {
        constexpr int K = decltype(kt)::value;
        if (a.bc == SYLV_BC_FACE)
            hipLaunchKernelGGL((k_lz_stencil<K, LZ_STEP, 2, BC_FACE>), dim3(a.ntiles),
                               dim3(kBlock), 0, s, a, it, replay);
        else if (K <= 4 && a.rows == 4)
            hipLaunchKernelGGL((k_lz_stencil<K, LZ_STEP, (K <= 4 ? 4 : 2), BC_PERIODIC>),
                               dim3(a.ntiles), dim3(kBlock), 0, s, a, it, replay);
        else
            hipLaunchKernelGGL((k_lz_stencil<K, LZ_STEP, 2, BC_PERIODIC>), dim3(a.ntiles),
                               dim3(kBlock), 0, s, a, it, replay);
        return hipGetLastError();
    });
}

hipError_t lz_launch_step(const LzArgs &a, int it, hipStream_t s) {
    hipError_t e = launch_step_kernel(a, it, 0, s);
    if (e != hipSuccess) return e;
    return dispatch_k(a.k, [&](auto kt) -> hipError_t {
        constexpr int K = decltype(kt)::value;
        hipError_t e2 = launch_reduce(a, lz_nv_step<K>(), a.ntiles, s);
        if (e2 != hipSuccess) return e2;
        hipLaunchKernelGGL((k_lz_fin<K>), dim3(1), dim3(kBlock), 0, s, a, it);
        return hipGetLastError();
    });
}

hipError_t lz_launch_replay(const LzArgs &a, int it, hipStream_t s) {
    return launch_step_kernel(a, it, 1, s);
}

hipError_t lz_launch_flag(const LzArgs &a, int *host_running, hipStream_t s) {
    hipLaunchKernelGGL(k_lz_flag, dim3(1), dim3(64), 0, s, a.st, host_running);
    return hipGetLastError();
}

hipError_t lz_launch_finish(const LzArgs &a, int iters, hipStream_t s) {
    hipError_t e = dispatch_k(a.k, [&](auto kt) -> hipError_t {
        constexpr int K = decltype(kt)::value;
        hipLaunchKernelGGL((k_lz_assemble<K>), dim3(a.nchunks), dim3(kBlock), 0, s, a, iters);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    return lz_launch_resid(a, s);
}

hipError_t lz_launch_resid(const LzArgs &a, hipStream_t s) {
    return dispatch_k(a.k, [&](auto kt) -> hipError_t {
        constexpr int K = decltype(kt)::value;
        hipError_t e;
        if (a.bc == SYLV_BC_FACE)
            hipLaunchKernelGGL((k_lz_stencil<K, LZ_RESID, 2, BC_FACE>), dim3(a.ntiles),
                               dim3(kBlock), 0, s, a, 0, 0);
        else if (K <= 4 && a.rows == 4)
            hipLaunchKernelGGL((k_lz_stencil<K, LZ_RESID, (K <= 4 ? 4 : 2), BC_PERIODIC>),
                               dim3(a.ntiles), dim3(kBlock), 0, s, a, 0, 0);
        else
            hipLaunchKernelGGL((k_lz_stencil<K, LZ_RESID, 2, BC_PERIODIC>), dim3(a.ntiles),
                               dim3(kBlock), 0, s, a, 0, 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = launch_reduce(a, 2, a.ntiles, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_lz_rfin, dim3(1), dim3(64), 0, s, a);
        return hipGetLastError();
    });
}

}  // namespace sylv
