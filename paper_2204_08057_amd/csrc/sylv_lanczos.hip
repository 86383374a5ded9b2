// Lanczos-Sylvester kernels (Section 3.3): the symmetric block Lanczos process for N^-1 D2 in the
// N inner product (Alg. 4) and the device side of the symmetric sparse Sylvester solver around
// it (Alg. 5).  One Lanczos step i is four launches:
//
//   k_lz_stencil<STEP>  V_i = W_(i-1) B_i^-1 formed while the tile and its 2-pixel halo are staged
//                       in LDS (the Cholesky-QR normalisation of the previous block, fused), V_i
//                       stored as basis block i, W = N^-1 D2 V_i - V_(i-1) B_i^T (13-point stencil
//                       of (kappa^2 - Lap)^2), partials of H_i = V_i^T N W;
//   k_lz_hfin           H_i (symmetric part) from the partials, fixed order;
//   k_lz_orth           W <- W - V_i H_i, partials of the N-Gram matrix W^T N W;
//   k_lz_qr             W^T N W = B_(i+1)^T B_(i+1) (Cholesky), B_(i+1)^-1, and Alg. 5's residual
//                       estimate gamma, carried by a block forward elimination of T_i + rho_l I
//                       (one thread per eigenvalue rho_l of Lhat) instead of an eigendecomposition
//                       of T_i at every step; the stopping test.
//
// The blocks V_i stay in the workspace, so the approximation M = sum_i V_i G_i is one streaming
// pass over them (k_lz_assemble) once the host has solved the small projected equation for the
// G_i, instead of the paper's second Lanczos pass.  A last stencil pass recomputes the residual
// of eq. (Axb) for the statistics.  All reductions are per-workgroup partials summed in a fixed
// order by a one-workgroup kernel, so results are bitwise repeatable.

#include "sylv_device.h"

namespace sylv {
namespace {

using namespace dev;

constexpr int kLzRows = 2;           // output rows per lane in the stencil kernels
enum { LZ_STEP = 0, LZ_RESID = 1 };

__device__ __forceinline__ const double *cblk(const double *base, int i) {
    return base + (size_t)i * kLzStride;
}
__device__ __forceinline__ double *wblk(double *base, int i) { return base + (size_t)i * kLzStride; }

// Workgroup partial of the packed symmetric matrix sum_t wt_t sym(u_t w_t^T) (upper triangle row
// by row, K (K + 1) / 2 values) and, if EXTRA, one more scalar; stored at partial[slot * nred +
// blkid].  Each value is reduced in turn, so only one is live at a time.
template <int K, int NP, bool EXTRA>
__device__ __forceinline__ void sym_partials(const double (&u)[NP][K], const double (&w)[NP][K],
                                             const double (&wt)[NP], double extra,
                                             double *partial, int nred, int blkid) {
    constexpr int PK = K * (K + 1) / 2;
    constexpr int NV = PK + (EXTRA ? 1 : 0);
    __shared__ double sm[NV][kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int e = 0;
#pragma unroll
    for (int a = 0; a < K; ++a) {
#pragma unroll
        for (int b = a; b < K; ++b, ++e) {
            double v = 0.0;
#pragma unroll
            for (int t = 0; t < NP; ++t) v += wt[t] * (0.5 * (u[t][a] * w[t][b] + u[t][b] * w[t][a]));
            v = wave_sum(v);
            if (lane == 0) sm[e][wid] = v;
        }
    }
    if constexpr (EXTRA) {
        const double v = wave_sum(extra);
        if (lane == 0) sm[PK][wid] = v;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const int i = threadIdx.x;
        gp(partial)[(size_t)i * nred + blkid] = (sm[i][0] + sm[i][1]) + (sm[i][2] + sm[i][3]);
    }
}

// ---- small dense helpers (one thread) -------------------------------------------------------

// Upper Cholesky factor of the symmetric K x K matrix g (g = R^T R).  False if a pivot is not
// positive or not finite.
template <int K>
__device__ bool chol_upper(const double (&g)[K][K], double (&r)[K][K]) {
#pragma unroll
    for (int i = 0; i < K; ++i) {
#pragma unroll
        for (int j = 0; j < K; ++j) r[i][j] = 0.0;
    }
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

// Start block Yhat = Y^T T A P^-1 (eq. (Axb-Sylv)), written to Yh and to the running block W,
// with the partials of its N-Gram matrix and a count of invalid n_p.
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
            for (int j = 0; j < K; ++j) {
                gp(a.Yh)[(size_t)j * n_pix + p] = yh[e][j];
                gp(a.Wn)[(size_t)j * n_pix + p] = yh[e][j];
            }
        }
    }
    sym_partials<K, 4, true>(yh, yh, wt, bad, a.partial, a.nred, chunk);
}

// Stencil kernels.  STEP: one Lanczos step's product (see the file comment).  RESID: residual of
// eq. (Axb) for X: r_j = n_p tau_j Yhat_j - (tau_j D2 X_j + n_p (A^T T A X_p)_j), with the
// partials of ||r||^2 and ||b||^2.
template <int K, int MODE>
__global__ __launch_bounds__(kBlock) void k_lz_stencil(LzArgs a, int it) {
    constexpr int R = kLzRows;
    constexpr int LH = kWavesY * R + 4;   // staged rows: tile + 2-row halo above and below
    constexpr int LW = kTileX + 4;        // staged columns
    constexpr int RPW = LH / kWavesY;     // staged rows per wavefront
    LzState *st = a.st;
    if (MODE == LZ_STEP && st->done) return;
    const int tile = xcd_remap(blockIdx.x, a.ntiles);
    const int nx = a.nx, ny = a.ny, n_pix = a.n_pix;
    const LzConst *c = a.c;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int tile_x = tile % a.tiles_x, tile_y = tile / a.tiles_x;
    const int x0 = tile_x * kTileX, y0 = tile_y * kWavesY * R;
    const int ix = x0 + tx;
    const int iy0 = y0 + ty * R;
    const bool active = (ix < nx) && (iy0 < ny);

    // ---- issue the global loads: staged field, then per-output-pixel data ------------------
    const GAS double *src = gp(MODE == LZ_STEP ? (const double *)a.Wn : (const double *)a.X);
    const int cmain = wrapi(x0 + tx, nx);
    const int hitem = ty * 64 + tx;
    const int hr = hitem >> 2, hc = hitem & 3;
    const int hcol = (hc < 2) ? hc : (kTileX + hc);
    const bool hvalid = hitem < 4 * LH;
    const int hoff = hvalid ? wrapi(y0 - 2 + hr, ny) * nx + wrapi(x0 - 2 + hcol, nx) : 0;
    int soff[RPW];
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) soff[rr] = wrapi(y0 - 2 + rr * kWavesY + ty, ny) * nx + cmain;
    double sa[K][RPW], ha[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const GAS double *s = src + (size_t)j * n_pix;
#pragma unroll
        for (int rr = 0; rr < RPW; ++rr) sa[j][rr] = s[soff[rr]];
        ha[j] = hvalid ? s[hoff] : 0.0;
    }
    const int ixc = ix < nx ? ix : 0;
    double nv[R], aux[R][K];
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const int pix = (iy0 + t < ny ? iy0 + t : 0) * nx + ixc;
        nv[t] = gp(a.n)[pix];
#pragma unroll
        for (int j = 0; j < K; ++j) aux[t][j] = 0.0;
        if (MODE == LZ_STEP && it > 1) {
            const GAS double *vo = gp(a.basis) + (size_t)(it - 2) * K * n_pix;
#pragma unroll
            for (int j = 0; j < K; ++j) aux[t][j] = vo[(size_t)j * n_pix + pix];
        } else if (MODE == LZ_RESID) {
#pragma unroll
            for (int j = 0; j < K; ++j) aux[t][j] = gp(a.Yh)[(size_t)j * n_pix + pix];
        }
    }

    // ---- stage the field in LDS (STEP: normalised, V_i = W B_i^-1) ---------------------------
    __shared__ double lds[K][LH][LW];
    const double *Bi = (MODE == LZ_STEP) ? cblk(a.B, it - 1) : nullptr;
    const double *Binv = (MODE == LZ_STEP) ? cblk(a.Binv, it - 1) : nullptr;
#pragma unroll
    for (int rr = 0; rr <= RPW; ++rr) {
        if (rr == RPW && !hvalid) break;
        double w[K];
#pragma unroll
        for (int j = 0; j < K; ++j) w[j] = (rr < RPW) ? sa[j][rr] : ha[j];
        const int row = (rr < RPW) ? rr * kWavesY + ty : hr;
        const int col = (rr < RPW) ? tx + 2 : hcol;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            double v;
            if constexpr (MODE == LZ_STEP) {
                v = 0.0;
#pragma unroll
                for (int q = 0; q <= j; ++q) v += w[q] * Binv[q * kMaxK + j];
            } else {
                v = w[j];
            }
            lds[j][row][col] = v;
        }
    }
    __syncthreads();

    // ---- 13-point stencil of (kappa^2 - Lap)^2 from LDS --------------------------------------
    const double c0 = c->coef[0], c1 = c->coef[1], cd = c->coef[2], c2 = c->coef[3];
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
                const double n4 = (cc[t + 1] + cc[t + 3]) + (l1[t + 1] + r1[t + 1]);
                const double d4 = (l1[t] + r1[t]) + (l1[t + 2] + r1[t + 2]);
                const double f4 = (cc[t] + cc[t + 4]) + (l2[t] + r2[t]);
                acc[j][t] = c0 * cc[t + 2] + c1 * n4 + cd * d4 + c2 * f4;
                ctr[j][t] = cc[t + 2];
            }
        }
#pragma unroll
        for (int t = 0; t < R; ++t) {
            if (iy0 + t >= ny) continue;
            const int pix = (iy0 + t) * nx + ix;
            if constexpr (MODE == LZ_STEP) {
                GAS double *vb = gp(a.basis) + (size_t)(it - 1) * K * n_pix;
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    double w = acc[j][t] / nv[t];
                    if (it > 1) {
#pragma unroll
                        for (int q = 0; q < K; ++q) w -= aux[t][q] * Bi[j * kMaxK + q];
                    }
                    vb[(size_t)j * n_pix + pix] = ctr[j][t];
                    gp(a.Wa)[(size_t)j * n_pix + pix] = w;
                    uo[t][j] = ctr[j][t];
                    wo[t][j] = w;
                }
                wt[t] = nv[t];
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
    if constexpr (MODE == LZ_STEP) {
        sym_partials<K, R, false>(uo, wo, wt, 0.0, a.partial, a.nred, tile);
    } else {
        double v[2] = {d0, d1};
        block_partials<2>(v, a.partial, a.nred, 0, tile);
    }
}

// H_i from the stencil kernel's partials (its symmetric part, stored as a full block).
template <int K>
__global__ __launch_bounds__(kBlock) void k_lz_hfin(LzArgs a, int it) {
    LzState *st = a.st;
    if (st->done) return;
    constexpr int PK = K * (K + 1) / 2;
    double h[PK];
    consume<PK>(a.partial, a.nred, 0, a.ntiles, h);
    if (threadIdx.x == 0) {
        double *H = wblk(a.H, it - 1);
        bool fin = true;
        int e = 0;
        for (int r = 0; r < K; ++r)
            for (int q = r; q < K; ++q, ++e) {
                H[r * kMaxK + q] = h[e];
                H[q * kMaxK + r] = h[e];
                fin = fin && isfinite(h[e]);
            }
        if (!fin) {
            st->status = SYLV_NONFINITE;
            st->iter = it - 1;
            st->done = 1;
        }
    }
}

// W <- W - V_i H_i and the partials of W^T N W.
template <int K>
__global__ __launch_bounds__(kBlock) void k_lz_orth(LzArgs a, int it) {
    if (a.st->done) return;
    const int chunk = xcd_remap(blockIdx.x, a.nchunks);
    const int n_pix = a.n_pix;
    const double *H = cblk(a.H, it - 1);
    const GAS double *V = gp(a.basis) + (size_t)(it - 1) * K * n_pix;
    const GAS double *Wa = gp(a.Wa);
    double w[4][K], v[4][K], wt[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int p = chunk * kChunk + e * kBlock + threadIdx.x;
        const bool in = p < n_pix;
        wt[e] = in ? gp(a.n)[p] : 0.0;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            w[e][j] = in ? Wa[(size_t)j * n_pix + p] : 0.0;
            v[e][j] = in ? V[(size_t)j * n_pix + p] : 0.0;
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int p = chunk * kChunk + e * kBlock + threadIdx.x;
        double o[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            double s = w[e][j];
#pragma unroll
            for (int q = 0; q < K; ++q) s -= v[e][q] * H[q * kMaxK + j];
            o[j] = s;
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
            w[e][j] = o[j];
            if (p < n_pix) gp(a.Wn)[(size_t)j * n_pix + p] = o[j];
        }
    }
    sym_partials<K, 4, false>(w, w, wt, 0.0, a.partial, a.nred, chunk);
}

// Cholesky-QR of the running block in the N inner product: W^T N W = B^T B, B upper.
//   it == 0: the start block, B_0; ||B_0||_F sets the stopping threshold, and column l of
//            B_0 U starts the forward elimination of column l.
//   it >= 1: B_(i+1) after step i, then Alg. 5's residual estimate and the stopping test.
// The estimate: Q F e_l = (T_i + rho_l I)^-1 E_1 B_0 U e_l (eq. (soln-constr)), and gamma is
// sum_l ||B_(i+1) x_l||^2 with x_l the last block of that vector.  With the Schur complements
// S_1 = H_1 + rho_l I, S_j = H_j + rho_l I - B_j S_(j-1)^-1 B_j^T and y_1 = B_0 U e_l,
// y_j = -B_j S_(j-1)^-1 y_(j-1) (block elimination of the block tridiagonal T_i + rho_l I), that
// last block is x_l = S_i^-1 y_i; each step extends the elimination by one block.
template <int K>
__global__ __launch_bounds__(kBlock) void k_lz_qr(LzArgs a, int it, int nblocks) {
    LzState *st = a.st;
    if (st->done) return;
    constexpr int PK = K * (K + 1) / 2;
    double g[PK + 1];
    if (it == 0) {   // start block: one more slot, the count of invalid n_p
        consume<PK + 1>(a.partial, a.nred, 0, nblocks, g);
    } else {
        double gg[PK];
        consume<PK>(a.partial, a.nred, 0, nblocks, gg);
#pragma unroll
        for (int e = 0; e < PK; ++e) g[e] = gg[e];
        g[PK] = 0.0;
    }
    __shared__ int s_ok;         // 0: B valid; 1: zero block; 2: not positive definite; 3: bad
    __shared__ double s_gam[K];
    if (threadIdx.x == 0) {
        double G[K][K], Bm[K][K], Bi[K][K];
        int e = 0;
        bool zero = true, fin = true;
        for (int r = 0; r < K; ++r)
            for (int q = r; q < K; ++q, ++e) {
                G[r][q] = g[e];
                G[q][r] = g[e];
                zero = zero && g[e] == 0.0;
                fin = fin && isfinite(g[e]);
            }
        int ok = 0;
        if (it == 0 && g[PK] > 0.0) ok = 3;
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
            }
        if (it == 0) {
            double nb = 0.0;
            for (int r = 0; r < K; ++r)
                for (int q = 0; q < K; ++q) nb += Bm[r][q] * Bm[r][q];
            st->nb0 = sqrt(nb);
            st->thresh = a.c->tol * sqrt(nb);
            for (int l = 0; l < K; ++l)          // y_1 for column l: B_0 U e_l
                for (int r = 0; r < K; ++r) {
                    double v = 0.0;
                    for (int q = 0; q < K; ++q) v += Bm[r][q] * a.c->U[q][l];
                    st->y[l][r] = v;
                }
            if (ok != 0) {                        // zero start block: X = 0; invalid n_p / values
                st->status = (ok == 1) ? SYLV_OK : (g[PK] > 0.0 ? SYLV_BAD_INPUT : SYLV_NONFINITE);
                st->iter = 0;
                st->gamma = 0.0;
                st->done = 1;
            }
        }
        s_ok = ok;
    }
    __syncthreads();
    if (it == 0) return;
    const int ok = s_ok;
    if (ok == 2 || ok == 3) {
        if (threadIdx.x == 0) {
            st->status = (ok == 2) ? SYLV_BREAKDOWN : SYLV_NONFINITE;
            st->iter = (ok == 2) ? it : it - 1;
            st->gamma = -1.0;
            a.hist[it - 1] = -1.0;
            st->done = 1;
        }
        return;
    }
    // residual estimate: thread l carries column l
    if (threadIdx.x < K) {
        const int l = threadIdx.x;
        const double rho = a.c->rho[l];
        const double *H = cblk(a.H, it - 1);
        const double *Bn = cblk(a.B, it);          // B_(i+1)
        double S[K][K], y[K];
        for (int r = 0; r < K; ++r) y[r] = st->y[l][r];
        if (it == 1) {
            for (int r = 0; r < K; ++r)
                for (int q = 0; q < K; ++q) S[r][q] = H[r * kMaxK + q] + (r == q ? rho : 0.0);
        } else {
            const double *Bj = cblk(a.B, it - 1);  // B_i
            double So[K][K], Ro[K][K];
            for (int r = 0; r < K; ++r)
                for (int q = 0; q < K; ++q) So[r][q] = st->S[l][r][q];
            chol_upper<K>(So, Ro);                 // S_(i-1) is positive definite
            // X = S_(i-1)^-1 B_i^T column by column; S_i = H_i + rho I - B_i X
            double X[K][K];
            for (int q = 0; q < K; ++q) {
                double bcol[K], xcol[K];
                for (int r = 0; r < K; ++r) bcol[r] = Bj[q * kMaxK + r];   // column q of B_i^T
                chol_solve<K>(Ro, bcol, xcol);
                for (int r = 0; r < K; ++r) X[r][q] = xcol[r];
            }
            for (int r = 0; r < K; ++r)
                for (int q = 0; q < K; ++q) {
                    double v = H[r * kMaxK + q] + (r == q ? rho : 0.0);
                    for (int s2 = 0; s2 < K; ++s2) v -= Bj[r * kMaxK + s2] * X[s2][q];
                    S[r][q] = v;
                }
            for (int r = 0; r < K; ++r)           // symmetrise against rounding
                for (int q = r + 1; q < K; ++q) {
                    const double m = 0.5 * (S[r][q] + S[q][r]);
                    S[r][q] = m;
                    S[q][r] = m;
                }
            double z[K];
            chol_solve<K>(Ro, y, z);
            for (int r = 0; r < K; ++r) {
                double v = 0.0;
                for (int q = 0; q < K; ++q) v -= Bj[r * kMaxK + q] * z[q];
                y[r] = v;
            }
        }
        double Rs[K][K], x[K];
        double gl;
        if (chol_upper<K>(S, Rs)) {
            chol_solve<K>(Rs, y, x);
            gl = 0.0;
            for (int r = 0; r < K; ++r) {
                double v = 0.0;
                for (int q = r; q < K; ++q) v += Bn[r * kMaxK + q] * x[q];
                gl += v * v;
            }
        } else {
            gl = __builtin_nan("");
        }
        for (int r = 0; r < K; ++r) {
            st->y[l][r] = y[r];
            for (int q = 0; q < K; ++q) st->S[l][r][q] = S[r][q];
        }
        s_gam[l] = gl;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double gam = 0.0;
        for (int l = 0; l < K; ++l) gam += s_gam[l];
        st->gamma = gam;
        st->iter = it;
        const double nb0 = st->nb0;
        a.hist[it - 1] = sqrt(gam) / nb0;
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

// ||b - G x||^2 and ||b||^2 from the residual pass.
__global__ __launch_bounds__(kBlock) void k_lz_rfin(LzArgs a) {
    double s[2];
    consume<2>(a.partial, a.nred, 0, a.ntiles, s);
    if (threadIdx.x == 0) {
        a.st->rr = s[0];
        a.st->bb = s[1];
    }
}

}  // namespace

int lz_tiles(int ny, int nx) {
    const int tx = (nx + kTileX - 1) / kTileX;
    const int ty = (ny + kWavesY * kLzRows - 1) / (kWavesY * kLzRows);
    return tx * ty;
}

hipError_t lz_launch_start(const LzArgs &a, hipStream_t s) {
    return dispatch_k(a.k, [&](auto kt) -> hipError_t {
        constexpr int K = decltype(kt)::value;
        hipLaunchKernelGGL((k_lz_start<K>), dim3(a.nchunks), dim3(kBlock), 0, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_lz_qr<K>), dim3(1), dim3(kBlock), 0, s, a, 0, a.nchunks);
        return hipGetLastError();
    });
}

hipError_t lz_launch_init(const LzArgs &a, int max_iter, hipStream_t s) {
    hipLaunchKernelGGL(k_lz_init, dim3(1), dim3(64), 0, s, a, max_iter);
    return hipGetLastError();
}

hipError_t lz_launch_step(const LzArgs &a, int it, hipStream_t s) {
    return dispatch_k(a.k, [&](auto kt) -> hipError_t {
        constexpr int K = decltype(kt)::value;
        hipLaunchKernelGGL((k_lz_stencil<K, LZ_STEP>), dim3(a.ntiles), dim3(kBlock), 0, s, a, it);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_lz_hfin<K>), dim3(1), dim3(kBlock), 0, s, a, it);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL((k_lz_orth<K>), dim3(a.nchunks), dim3(kBlock), 0, s, a, it);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL((k_lz_qr<K>), dim3(1), dim3(kBlock), 0, s, a, it, a.nchunks);
        return hipGetLastError();
    });
}

hipError_t lz_launch_flag(const LzArgs &a, int *host_running, hipStream_t s) {
    hipLaunchKernelGGL(k_lz_flag, dim3(1), dim3(64), 0, s, a.st, host_running);
    return hipGetLastError();
}

hipError_t lz_launch_finish(const LzArgs &a, int iters, hipStream_t s) {
    return dispatch_k(a.k, [&](auto kt) -> hipError_t {
        constexpr int K = decltype(kt)::value;
        hipLaunchKernelGGL((k_lz_assemble<K>), dim3(a.nchunks), dim3(kBlock), 0, s, a, iters);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_lz_stencil<K, LZ_RESID>), dim3(a.ntiles), dim3(kBlock), 0, s, a, 0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_lz_rfin, dim3(1), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    });
}

}  // namespace sylv
