// Block conjugate gradients over the s right-hand sides of one grid (O'Leary's block CG, the
// block analogue of Alg. 2 with the same per-pixel block-Jacobi preconditioner), for batches of
// perturbation-optimisation right-hand sides.  Per iteration:
//   P = Z + P beta                 (k_bdir; P = Z at the start)
//   Q = G P,  P^T Q                (k_bapply: the s applies share every read of the per-pixel
//                                   mixing block; Gram partials in float64)
//   alpha = (P^T Q)^-1 (R^T Z)     (k_bgram, phase 1)
//   X += P alpha, R -= Q alpha, Z = Minv R, R^T Z, ||r_c||^2   (k_bupdate)
//   beta = (R^T Z)_old^-1 (R^T Z)_new, per-column stopping test (k_bgram, phase 2)
// s x s systems are solved by Cholesky in float64 on the active columns only: a column that has
// converged leaves the block (deflation).  If a Gram matrix is not numerically positive
// definite the group switches to independent CG for every column (diagonal alpha and beta,
// after one restart with beta = 0).
//
// Reductions follow the same fence-free scheme as the single-vector kernels: every workgroup
// writes fixed-order partials and the one-workgroup Gram kernel reduces them in fixed order.

//
// This header holds the kernels and the launchers of one right-hand-side count S in one
// precision (BlockLaunch<S, T>); each pair is instantiated in a translation unit of its own
// (sylv_block_s{2,4,8}_{f32,f64}.hip) so that they compile in parallel.  sylv_block.hip
// dispatches on s and the precision and launches the Gram kernels.
#pragma once

#include "sylv_device.h"

namespace sylv {
namespace {
using namespace dev;

template <int S>
constexpr int gram_n() { return S * (S + 1) / 2; }

// Accumulate one quantity into the workgroup's per-wavefront slot (lane 0 of each wavefront
// owns its slot, so no two threads write the same LDS word).
__device__ __forceinline__ void wave_accum(double v, double *slot) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) *slot += v;
}

// Write NQ per-workgroup partials from the [4 wavefronts][NQ] LDS accumulators.
template <int NQ>
__device__ __forceinline__ void flush_partials(const double (&acc)[kBlock / 64][NQ],
                                               double *partial, int nred, int blk) {
    __syncthreads();
    GAS double *pp = gp(partial);
    for (int i = threadIdx.x; i < NQ; i += kBlock)
        pp[(size_t)i * nred + blk] = (acc[0][i] + acc[1][i]) + (acc[2][i] + acc[3][i]);
}

template <int NQ>
__device__ __forceinline__ void zero_acc(double (&acc)[kBlock / 64][NQ]) {
    for (int i = threadIdx.x; i < (kBlock / 64) * NQ; i += kBlock) (&acc[0][0])[i] = 0.0;
    __syncthreads();
}

// ---- the streaming block kernels: V = block_vec pixels per thread ---------------------------
// V consecutive pixels of one plane move as one buffer access per lane (8 bytes) when every lane
// of the wavefront holds V pixels of the grid and the group's planes allow it (F = true), else
// element by element with bounds checks.  Kernels decide F once per wavefront.
template <typename T, int V, bool F>
__device__ __forceinline__ void ldv(const GAS T *plane, uint32_t n, uint32_t i, T (&v)[V]) {
    if constexpr (V == 2 && sizeof(T) == 4 && F) {
        {
            const u32x2 a = __builtin_amdgcn_raw_buffer_load_b64(plane_rsrc(plane, n), i * 4u, 0, 0);
            v[0] = __uint_as_float(a.x);
            v[1] = __uint_as_float(a.y);
            return;
        }
    }
#pragma unroll
    for (int e = 0; e < V; ++e) v[e] = (i + e < n) ? bld(plane, n, i + e) : (T)0;
}
template <typename T, int V, bool F, int AUX = 0>
__device__ __forceinline__ void stv(GAS T *plane, uint32_t n, uint32_t i, const T (&v)[V]) {
    if constexpr (V == 2 && sizeof(T) == 4 && F) {
        {
            const u32x2 a = {__float_as_uint(v[0]), __float_as_uint(v[1])};
            __builtin_amdgcn_raw_buffer_store_b64(a, plane_rsrc((const GAS float *)plane, n),
                                                  i * 4u, 0, AUX);
            return;
        }
    }
#pragma unroll
    for (int e = 0; e < V; ++e)
        if (i + e < n) bst<AUX>(plane, n, i + e, v[e]);
}

// Preconditioner of one pixel from the bfloat16 factor planes (block kind: G = L^-1 with
// G[a][c], a >= c, at plane pidx(c, a); Jacobi kind: 1 / diagonal per component), loaded once
// and applied to every column of the group: z = G^T (G r).  Same arithmetic as
// precond_cg_pixel.
template <typename T, int K>
struct PcPix {
    T g[K * (K + 1) / 2];
};
template <typename T, int K>
__device__ __forceinline__ void pc_load(int pc, const GAS unsigned short *F, int n_pix, int pix,
                                        bool valid, PcPix<T, K> &c) {
    constexpr int MK = K * (K + 1) / 2;
    const int ne = (pc == SYLV_PC_BLOCK) ? MK : (pc == SYLV_PC_JACOBI) ? K : 0;
#pragma unroll
    for (int e = 0; e < MK; ++e)
        c.g[e] = (valid && e < ne) ? (T)bf16_value(F[(size_t)e * n_pix + pix]) : (T)0;
}
template <typename T, int K>
__device__ __forceinline__ void pc_apply(int pc, const PcPix<T, K> &c, const T (&r)[K],
                                         T (&z)[K]) {
    if (pc == SYLV_PC_BLOCK) {
        T t[K];
#pragma unroll
        for (int a = 0; a < K; ++a) {
            T s = 0;
#pragma unroll
            for (int q = 0; q <= a; ++q) s += c.g[pidx<K>(q, a)] * r[q];
            t[a] = s;
        }
#pragma unroll
        for (int q = 0; q < K; ++q) {
            T s = 0;
#pragma unroll
            for (int a = q; a < K; ++a) s += c.g[pidx<K>(q, a)] * t[a];
            z[q] = s;
        }
    } else if (pc == SYLV_PC_JACOBI) {
#pragma unroll
        for (int j = 0; j < K; ++j) z[j] = c.g[j] * r[j];
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j) z[j] = r[j];
    }
}

// The s x s coefficients (alpha or beta) of the current step, rounded to T, staged in LDS by the
// workgroup: read once from the group state, before any plane is written (the state could
// otherwise alias those stores and be re-read from memory at every use).
template <typename T, int S>
__device__ __forceinline__ void stage_coef(const double (&src)[kMaxS][kMaxS], T (&dst)[S][S]) {
    for (int i = threadIdx.x; i < S * S; i += kBlock) dst[i / S][i % S] = (T)src[i / S][i % S];
    __syncthreads();
}

template <bool B>
struct BTag {
    static constexpr bool value = B;
};

// 1 when every lane of the calling wavefront holds V whole pixels of the grid and the group's
// planes allow wide accesses; the same value in every lane.
__device__ __forceinline__ bool wave_full(int chunk, int v, int n_pix, int vec) {
    const int plast = (chunk * kBlock + (int)(threadIdx.x | 63u)) * v;
    return __builtin_amdgcn_readfirstlane((vec && plast + v <= n_pix) ? 1 : 0) != 0;
}

// Z = Minv R column by column (handed to `dst` for the columns in `use`), with the R^T Z and
// ||r_c||^2 sums of the thread's pixels added to its wavefront's slots of `acc` (the kernel
// zeroes and flushes acc, one array for every wavefront of the workgroup whichever code path it
// took).  rv holds the residuals of the thread's V pixels (zero for pixels outside the grid and
// for unused columns, whose terms are then exact zeros).
template <typename T, int K, int S, int V, typename Dst>
__device__ __forceinline__ void precond_and_gram(const Inst *__restrict__ tab, const Group &G,
                                                 const T (&rv)[S][K][V], const bool (&use)[S],
                                                 int p0, bool valid,
                                                 double (&acc)[kBlock / 64][gram_n<S>() + S],
                                                 Dst &&dst) {
    constexpr int NG = gram_n<S>();
    const Inst &I0 = tab[G.inst0];
    const int n_pix = I0.n_pix;
    PcPix<T, K> pcv[V];
#pragma unroll
    for (int e = 0; e < V; ++e)
        pc_load<T, K>(I0.pc, Pcg(I0), n_pix, p0 + e, valid && p0 + e < n_pix, pcv[e]);
    const int wid = threadIdx.x >> 6;
#pragma unroll
    for (int b = 0; b < S; ++b) {
        T zb[K][V];
#pragma unroll
        for (int e = 0; e < V; ++e) {
            T r1[K], z1[K];
#pragma unroll
            for (int j = 0; j < K; ++j) r1[j] = rv[b][j][e];
            pc_apply<T, K>(I0.pc, pcv[e], r1, z1);
#pragma unroll
            for (int j = 0; j < K; ++j) zb[j][e] = z1[j];
        }
        if (valid && use[b]) dst(b, zb);
#pragma unroll
        for (int a = 0; a <= b; ++a) {
            double v = 0.0;
#pragma unroll
            for (int j = 0; j < K; ++j)
#pragma unroll
                for (int e = 0; e < V; ++e) v += (double)rv[a][j][e] * (double)zb[j][e];
            wave_accum(v, &acc[wid][pidx<S>(a, b)]);
        }
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < K; ++j)
#pragma unroll
            for (int e = 0; e < V; ++e) v += (double)rv[b][j][e] * (double)rv[b][j][e];
        wave_accum(v, &acc[wid][NG + b]);
    }
}

// Start of a block run: per column r, r_r = rounded residual (float32 inner run) or the float64
// residual, z_r = Minv r_r, P_0 = Z_0, and the partials of R^T Z and ||r_r||^2.
template <typename T, int K, int S>
__global__ __launch_bounds__(kBlock) void k_bpinit(const Inst *__restrict__ tab,
                                                   const Group *__restrict__ groups,
                                                   const int *__restrict__ gcprefix, int ngroup,
                                                   int nb) {
    constexpr int V = block_vec(sizeof(T) == 8);
    const int L = xcd_remap(blockIdx.x, nb);
    const int g = find_inst(gcprefix, ngroup, L);
    const Group &G = groups[g];
    const int chunk = L - gcprefix[g];
    const Inst &I0 = tab[G.inst0];
    const int n_pix = I0.n_pix;
    const uint32_t np = (uint32_t)n_pix;
    const int p0 = (chunk * kBlock + threadIdx.x) * V;
    const bool valid = p0 < n_pix;
    constexpr int NQ = gram_n<S>() + S;
    __shared__ double acc[kBlock / 64][NQ];
    zero_acc<NQ>(acc);
    auto body = [&](auto ftag) {
        constexpr bool F = decltype(ftag)::value;
        T rv[S][K][V];
        bool use[S];
#pragma unroll
        for (int r = 0; r < S; ++r) {
            const Inst &I = tab[G.inst0 + r];
            use[r] = !I.st->done;   // outer run finished / initial residual zero
#pragma unroll
            for (int j = 0; j < K; ++j) {
#pragma unroll
                for (int e = 0; e < V; ++e) rv[r][j][e] = 0;
                if (valid && use[r]) {
                    double r64[V];
                    ldv<double, V, false>(gp(I.r) + (size_t)j * n_pix, np, (uint32_t)p0, r64);
#pragma unroll
                    for (int e = 0; e < V; ++e) rv[r][j][e] = (T)r64[e];
                    if constexpr (sizeof(T) == 4) {
                        float zero[V];
#pragma unroll
                        for (int e = 0; e < V; ++e) zero[e] = 0.0f;
                        stv<float, V, F>(gp(I.r32) + (size_t)j * n_pix, np, (uint32_t)p0, rv[r][j]);
                        stv<float, V, F>(gp(I.d32) + (size_t)j * n_pix, np, (uint32_t)p0, zero);
                    }
                }
            }
        }
        precond_and_gram<T, K, S, V>(tab, G, rv, use, p0, valid, acc,
                                     [&](int r, const T (&zb)[K][V]) {
            const Inst &I = tab[G.inst0 + r];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                stv<T, V, F>(Sel<T>::z(I) + (size_t)j * n_pix, np, (uint32_t)p0, zb[j]);
                stv<T, V, F>(Sel<T>::p(I, 0) + (size_t)j * n_pix, np, (uint32_t)p0, zb[j]);
            }
        });
    };
    if (wave_full(chunk, V, n_pix, G.vec)) body(BTag<true>{});
    else body(BTag<false>{});
    flush_partials<NQ>(acc, G.partial, G.nred, chunk);
}

// P_it = Z + P_(it-1) beta on the active columns (it >= 1).  SA: cache policy of the stores
// (non-temporal when the batch exceeds the last-level cache, float32 only).
template <typename T, int K, int S, int SA>
__global__ __launch_bounds__(kBlock) void k_bdir(const Inst *__restrict__ tab,
                                                 const Group *__restrict__ groups,
                                                 const int *__restrict__ gcprefix, int ngroup,
                                                 int nb, int it) {
    constexpr int V = block_vec(sizeof(T) == 8);
    const int L = xcd_remap(blockIdx.x, nb);
    const int g = find_inst(gcprefix, ngroup, L);
    const Group &G = groups[g];
    const GroupState *gs = G.gs;
    if (gs->done) return;
    const int chunk = L - gcprefix[g];
    const Inst &I0 = tab[G.inst0];
    const int n_pix = I0.n_pix;
    const uint32_t np = (uint32_t)n_pix;
    const int p0 = (chunk * kBlock + threadIdx.x) * V;
    const bool full = wave_full(chunk, V, n_pix, G.vec);
    bool act[S];
#pragma unroll
    for (int r = 0; r < S; ++r) act[r] = __builtin_amdgcn_readfirstlane(gs->active[r]) != 0;
    __shared__ T beta[S][S];
    stage_coef<T, S>(gs->beta, beta);
    if (p0 >= n_pix) return;
    auto body = [&](auto ftag) {
        constexpr bool F = decltype(ftag)::value;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            T po[S][V], zz[S][V];
#pragma unroll
            for (int c = 0; c < S; ++c) {
#pragma unroll
                for (int e = 0; e < V; ++e) po[c][e] = zz[c][e] = 0;
                if (act[c]) {
                    const Inst &I = tab[G.inst0 + c];
                    ldv<T, V, F>(Sel<T>::p(I, it - 1) + (size_t)j * n_pix, np, (uint32_t)p0, po[c]);
                    ldv<T, V, F>(Sel<T>::z(I) + (size_t)j * n_pix, np, (uint32_t)p0, zz[c]);
                }
            }
#pragma unroll
            for (int r = 0; r < S; ++r) {
                if (!act[r]) continue;
                T v[V];
#pragma unroll
                for (int e = 0; e < V; ++e) v[e] = zz[r][e];
#pragma unroll
                for (int c = 0; c < S; ++c) {
                    if (!act[c]) continue;
                    const T b = beta[c][r];
#pragma unroll
                    for (int e = 0; e < V; ++e) v[e] += b * po[c][e];
                }
                stv<T, V, F, SA>(Sel<T>::p(tab[G.inst0 + r], it) + (size_t)j * n_pix, np,
                             (uint32_t)p0, v);
            }
        }
    };
    if (full) body(BTag<true>{});
    else body(BTag<false>{});
}

// Q = G P for the active columns of a group, sharing the per-pixel mixing blocks, and the
// partials of P^T Q.  Same tiling and LDS staging as the single-vector apply.
template <typename T, int K, int R, int S, int BC, int SA>
__global__ __launch_bounds__(kBlock) void k_bapply(const Inst *__restrict__ tab,
                                                   const Group *__restrict__ groups,
                                                   const int *__restrict__ gtprefix, int ngroup,
                                                   int nb, int it) {
    constexpr int MK = K * (K + 1) / 2;
    constexpr int LH = kWavesY * R + 4;
    constexpr int LW = kTileX + 4;
    constexpr int RPW = LH / kWavesY;
    constexpr int NQ = gram_n<S>();
    const int L = xcd_remap(blockIdx.x, nb);
    const int g = find_inst(gtprefix, ngroup, L);
    const Group &G = groups[g];
    const GroupState *gs = G.gs;
    if (gs->done) return;
    const int tile = L - gtprefix[g];
    const Inst &I0 = tab[G.inst0];
    const int nx = I0.nx, ny = I0.ny, n_pix = I0.n_pix;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int tile_x = tile % I0.tiles_x, tile_y = tile / I0.tiles_x;
    const int x0 = tile_x * kTileX, y0 = tile_y * kWavesY * R;
    const int ix = x0 + tx;
    const int iy0 = y0 + ty * R;
    const bool active = (ix < nx) && (iy0 < ny);

    __shared__ double acc[kBlock / 64][NQ];
    __shared__ T lds[K][LH][LW];
    zero_acc<NQ>(acc);

    const uint32_t np = (uint32_t)n_pix;   // plane length for buffer accesses
    const int cmain = wrapf(x0 + tx, nx);
    const int hitem = ty * 64 + tx;
    const int hr = hitem >> 2, hc = hitem & 3;
    const int hcol = (hc < 2) ? hc : (kTileX + hc);
    const bool hvalid = hitem < 4 * LH;
    const uint32_t hoff =
        hvalid ? (uint32_t)(wrapf(y0 - 2 + hr, ny) * nx + wrapf(x0 - 2 + hcol, nx)) : 0u;
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

    T m[R][MK];
    {
        const GAS T *M = Sel<T>::M(I0);
        const int ixc = ix < nx ? ix : 0;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const uint32_t pix = (uint32_t)((iy0 + t < ny ? iy0 + t : 0) * nx + ixc);
#pragma unroll
            for (int e = 0; e < MK; ++e) m[t][e] = bld(M + (size_t)e * n_pix, np, pix);
        }
    }
    // every value read from memory that a store below could alias is read first: the active
    // columns and the stencil coefficients
    bool act[S];
#pragma unroll
    for (int r = 0; r < S; ++r) act[r] = __builtin_amdgcn_readfirstlane(gs->active[r]) != 0;
    T cf[K][6];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const double *cj = I0.coef + j * kCoefStride;
        cf[j][0] = (T)cj[0]; cf[j][1] = (T)cj[1]; cf[j][2] = (T)cj[2]; cf[j][3] = (T)cj[3];
        cf[j][4] = (T)cj[6]; cf[j][5] = (T)(cj[5] * cj[5]);
    }
    T pc[S][K][R];   // centres of every column's direction at this lane's output pixels
    const int wid = ty;
    // staged values of one column, loaded one column ahead of its stencil
    T sa[K][RPW], ha[K];
    auto load_col = [&](int c) {
        const GAS T *u = Sel<T>::p(tab[G.inst0 + c], it);
#pragma unroll
        for (int j = 0; j < K; ++j) {
#pragma unroll
            for (int rr = 0; rr < RPW; ++rr)
                sa[j][rr] = sin[rr] ? bld(u + (size_t)j * n_pix, np, soff[rr]) : (T)0;
            ha[j] = hin ? bld(u + (size_t)j * n_pix, np, hoff) : (T)0;
        }
    };
    {
        int c0 = 0;
        while (c0 < S && !act[c0]) ++c0;
        if (c0 < S) load_col(c0);
    }
#pragma unroll
    for (int b = 0; b < S; ++b) {
        if (!act[b]) continue;
        const Inst &Ib = tab[G.inst0 + b];
        __syncthreads();   // previous column's stencil reads are done
#pragma unroll
        for (int j = 0; j < K; ++j) {
#pragma unroll
            for (int rr = 0; rr < RPW; ++rr) lds[j][rr * kWavesY + ty][tx + 2] = sa[j][rr];
            if (hvalid) lds[j][hr][hcol] = ha[j];   // 0 outside a face (hin)
        }
        __syncthreads();
        {   // the next active column's loads fly during this column's stencil
            int nc = b + 1;
            while (nc < S && !act[nc]) ++nc;
            if (nc < S) load_col(nc);
        }
        T q[K][R];
#pragma unroll
        for (int j = 0; j < K; ++j)
#pragma unroll
            for (int t = 0; t < R; ++t) q[j][t] = 0;
        if (active) {
            const int lr = ty * R;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const T c0 = cf[j][0], c1 = cf[j][1], cd = cf[j][2], c2 = cf[j][3];
                const T tj = cf[j][4], k2 = cf[j][5];
                T cc[R + 4], l1[R + 2], r1[R + 2], l2[R], r2[R];
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
                    const T d4 = (l1[t] + r1[t]) + (l1[t + 2] + r1[t + 2]);
                    const T f4 = (cc[t] + cc[t + 4]) + (l2[t] + r2[t]);
                    if constexpr (BC == BC_FACE) {
                        const int iy = iy0 + t;
                        const T dp = (T)face_deg(ix, iy, nx, ny);
                        const T e0 = k2 + dp, b0 = (T)2 * k2 + dp;
                        const T en = (b0 + (T)face_deg(ix, iy - 1, nx, ny)) * cc[t + 1] +
                                     (b0 + (T)face_deg(ix, iy + 1, nx, ny)) * cc[t + 3] +
                                     (b0 + (T)face_deg(ix - 1, iy, nx, ny)) * l1[t + 1] +
                                     (b0 + (T)face_deg(ix + 1, iy, nx, ny)) * r1[t + 1];
                        q[j][t] = tj * (e0 * e0 + dp) * cc[t + 2] - tj * en + cd * d4 + c2 * f4;
                    } else {
                        const T n4 = (cc[t + 1] + cc[t + 3]) + (l1[t + 1] + r1[t + 1]);
                        q[j][t] = c0 * cc[t + 2] + c1 * n4 + cd * d4 + c2 * f4;
                    }
                    pc[b][j][t] = (iy0 + t < ny) ? cc[t + 2] : (T)0;
                }
            }
            GAS T *qq = Sel<T>::q(Ib);
#pragma unroll
            for (int t = 0; t < R; ++t) {
                if (iy0 + t < ny) {
                    const int pix = (iy0 + t) * nx + ix;
                    T tmp[K];
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        T sum = q[j][t];
#pragma unroll
                        for (int i = 0; i < K; ++i) sum += m[t][pidx<K>(j, i)] * pc[b][i][t];
                        tmp[j] = sum;
                    }
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        q[j][t] = tmp[j];
                        bst<SA>(qq + (size_t)j * n_pix, np, (uint32_t)pix, tmp[j]);
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < K; ++j) q[j][t] = 0;
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < K; ++j)
#pragma unroll
                for (int t = 0; t < R; ++t) pc[b][j][t] = 0;
        }
        // Gram entries (a, b), a <= b, with this column's q
#pragma unroll
        for (int a = 0; a <= b; ++a) {
            if (!act[a]) continue;
            double v = 0.0;
#pragma unroll
            for (int j = 0; j < K; ++j)
#pragma unroll
                for (int t = 0; t < R; ++t) v += (double)pc[a][j][t] * (double)q[j][t];
            wave_accum(v, &acc[wid][pidx<S>(a, b)]);
        }
    }
    flush_partials<NQ>(acc, G.partial, G.nred, tile);
}

// X += P alpha, R -= Q alpha, Z = Minv R on the active columns; partials of R^T Z, ||r_c||^2.
template <typename T, int K, int S, int SA>
__global__ __launch_bounds__(kBlock) void k_bupdate(const Inst *__restrict__ tab,
                                                    const Group *__restrict__ groups,
                                                    const int *__restrict__ gcprefix, int ngroup,
                                                    int nb, int it) {
    constexpr int V = block_vec(sizeof(T) == 8);
    const int L = xcd_remap(blockIdx.x, nb);
    const int g = find_inst(gcprefix, ngroup, L);
    const Group &G = groups[g];
    const GroupState *gs = G.gs;
    if (gs->done) return;
    const int chunk = L - gcprefix[g];
    const Inst &I0 = tab[G.inst0];
    const int n_pix = I0.n_pix;
    const uint32_t np = (uint32_t)n_pix;
    const int p0 = (chunk * kBlock + threadIdx.x) * V;
    const bool valid = p0 < n_pix;
    bool act[S];
#pragma unroll
    for (int r = 0; r < S; ++r) act[r] = __builtin_amdgcn_readfirstlane(gs->active[r]) != 0;
    __shared__ T alpha[S][S];
    stage_coef<T, S>(gs->alpha, alpha);
    constexpr int NQ = gram_n<S>() + S;
    __shared__ double acc[kBlock / 64][NQ];
    zero_acc<NQ>(acc);
    auto body = [&](auto ftag) {
        constexpr bool F = decltype(ftag)::value;
        T rv[S][K][V];
#pragma unroll
        for (int r = 0; r < S; ++r)
#pragma unroll
            for (int j = 0; j < K; ++j)
#pragma unroll
                for (int e = 0; e < V; ++e) rv[r][j][e] = 0;
        if (valid) {
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const size_t o = (size_t)j * n_pix;
                T pj[S][V], qj[S][V];
#pragma unroll
                for (int c = 0; c < S; ++c) {
#pragma unroll
                    for (int e = 0; e < V; ++e) pj[c][e] = qj[c][e] = 0;
                    if (act[c]) {
                        const Inst &I = tab[G.inst0 + c];
                        ldv<T, V, F>(Sel<T>::p(I, it) + o, np, (uint32_t)p0, pj[c]);
                        ldv<T, V, F>(Sel<T>::q(I) + o, np, (uint32_t)p0, qj[c]);
                    }
                }
#pragma unroll
                for (int r = 0; r < S; ++r) {
                    if (!act[r]) continue;
                    const Inst &I = tab[G.inst0 + r];
                    T xv[V], rr[V];
                    ldv<T, V, F>(Sel<T>::x(I) + o, np, (uint32_t)p0, xv);
                    ldv<T, V, F>(Sel<T>::r(I) + o, np, (uint32_t)p0, rr);
#pragma unroll
                    for (int c = 0; c < S; ++c) {
                        if (!act[c]) continue;
                        const T a = alpha[c][r];
#pragma unroll
                        for (int e = 0; e < V; ++e) {
                            xv[e] += a * pj[c][e];
                            rr[e] -= a * qj[c][e];
                        }
                    }
                    stv<T, V, F, SA>(Sel<T>::x(I) + o, np, (uint32_t)p0, xv);
                    stv<T, V, F, SA>(Sel<T>::r(I) + o, np, (uint32_t)p0, rr);
#pragma unroll
                    for (int e = 0; e < V; ++e) rv[r][j][e] = rr[e];
                }
            }
        }
        precond_and_gram<T, K, S, V>(tab, G, rv, act, p0, valid, acc,
                                     [&](int r, const T (&zb)[K][V]) {
            const Inst &I = tab[G.inst0 + r];
#pragma unroll
            for (int j = 0; j < K; ++j)
                stv<T, V, F, SA>(Sel<T>::z(I) + (size_t)j * n_pix, np, (uint32_t)p0, zb[j]);
        });
    };
    if (wave_full(chunk, V, n_pix, G.vec)) body(BTag<true>{});
    else body(BTag<false>{});
    flush_partials<NQ>(acc, G.partial, G.nred, chunk);
}

// ---- small dense float64 algebra (one thread) -----------------------------------------------
// Cholesky in place (lower triangle); fails when an active pivot is not positive or falls below
// 1e-13 of the largest active diagonal entry.
// The same factorisation and solve on the full S x S system with the inactive rows and columns
// set to the identity (and zero right-hand sides): the loops are static, so the matrices stay in
// registers, and every term an inactive index adds is an exact zero, so the active entries are
// bitwise those of the compacted system.  The breakdown test scales by the active diagonal only.
template <int S>
__device__ __forceinline__ bool chol_masked(double (&a)[S][S], const bool (&act)[S]) {
    double dmax = 0.0;
#pragma unroll
    for (int i = 0; i < S; ++i)
        if (act[i]) dmax = fmax(dmax, fabs(a[i][i]));
    bool ok = true;
#pragma unroll
    for (int c = 0; c < S; ++c) {
        double s = a[c][c];
#pragma unroll
        for (int t = 0; t < c; ++t) s -= a[c][t] * a[c][t];
        if (act[c] && (!(s > 1e-13 * dmax) || !isfinite(s))) ok = false;
        const double d = sqrt(s > 0.0 ? s : 1.0);
        a[c][c] = d;
#pragma unroll
        for (int r = c + 1; r < S; ++r) {
            double v = a[r][c];
#pragma unroll
            for (int t = 0; t < c; ++t) v -= a[r][t] * a[c][t];
            a[r][c] = v / d;
        }
    }
    return ok;
}
template <int S>
__device__ __forceinline__ void chol_solve_masked(const double (&l)[S][S], double (&b)[S][S]) {
#pragma unroll
    for (int col = 0; col < S; ++col) {
#pragma unroll
        for (int r = 0; r < S; ++r) {
            double v = b[r][col];
#pragma unroll
            for (int t = 0; t < r; ++t) v -= l[r][t] * b[t][col];
            b[r][col] = v / l[r][r];
        }
#pragma unroll
        for (int r = S - 1; r >= 0; --r) {
            double v = b[r][col];
#pragma unroll
            for (int t = r + 1; t < S; ++t) v -= l[t][r] * b[t][col];
            b[r][col] = v / l[r][r];
        }
    }
}

// Group-level reductions and the s x s recurrences (one workgroup per group).
//  phase 0: start of a run (after k_bpinit): R^T Z, per-column thresholds and active set
//  phase 1: alpha = (P^T Q)^-1 R^T Z on the active set (after k_bapply)
//  phase 2: per-column stopping test, beta = (R^T Z)_old^-1 (R^T Z)_new (after k_bupdate)
// Column states are mirrored into each instance's DevState (float64 run, or the inner run of
// the mixed path), which the completion count and the statistics read.
// Fold the per-workgroup partials of one Gram quantity of one group (fixed order, four loads in
// flight per thread) into entry 0: grid (groups, quantities).  Phase 1 sums the P^T Q partials
// of the apply tiles, phases 0 and 2 the R^T Z and ||r||^2 partials of the streaming chunks.
template <int S>
__global__ __launch_bounds__(kBlock) void k_bgram_fold(const Group *__restrict__ groups,
                                                       int phase, int mixed) {
    constexpr int NG = gram_n<S>();
    constexpr int NQ = NG + S;
    const Group &G = groups[blockIdx.x];
    const int i = blockIdx.y;
    if (i >= ((phase == 1) ? NG : NQ)) return;
    if (phase != 0 && G.gs->done) return;
    const int nsum = (phase == 1) ? (mixed ? G.ntiles32 : G.ntiles) : G.nchunks;
    double v[1];
    consume<1>(G.partial, G.nred, i, nsum, v);   // every read precedes its final barrier
    if (threadIdx.x == 0) gp(G.partial)[(size_t)i * G.nred] = v[0];
}

template <int S>
__global__ __launch_bounds__(kBlock) void k_bgram(const Inst *__restrict__ tab,
                                                  const Group *__restrict__ groups, int phase,
                                                  int mixed, double inner_tol, double safety,
                                                  int max_iter) {
    constexpr int NG = gram_n<S>();
    constexpr int NQ = NG + S;
    const Group &G = groups[blockIdx.x];
    GroupState *gs = G.gs;
    if (phase != 0 && gs->done) return;
    const int nq = (phase == 1) ? NG : NQ;
    // k_bgram_fold has summed every quantity's partials into entry 0
    __shared__ double q[NQ];
    const GAS double *pp = gp(G.partial);
    for (int i = threadIdx.x; i < nq; i += kBlock) q[i] = pp[(size_t)i * G.nred];
    __syncthreads();
    if (threadIdx.x != 0) return;

    auto state = [&](int r) -> DevState * {
        const Inst &I = tab[G.inst0 + r];
        return mixed ? I.st_in : I.st;
    };
    auto finish = [&](int r, int status) {
        DevState *st = state(r);
        st->status = status;
        st->done = 1;
        st->iter = gs->iter;
        st->total_iter += gs->iter;
        gs->active[r] = 0;
    };

    if (phase == 0) {
        int nact = 0;
        for (int r = 0; r < S; ++r) {
            const Inst &I = tab[G.inst0 + r];
            DevState *st = state(r);
            const double rz = q[pidx<S>(r, r)], rr = q[NG + r];
            double tol = st->tol;
            bool act;
            if (mixed) {
                act = !I.st->done;
                if (act) {
                    const double need = safety * sqrt(I.st->thresh / fmax(I.st->rr, 1e-300));
                    tol = fmin(0.1, fmax(inner_tol, need));
                }
                st->tol = tol;
                st->max_iter = max_iter;
            } else {
                act = !st->done;
            }
            // float64 runs stop against ||b - G x0|| (threshold of the initial residual pass,
            // kept across restarts); inner runs against their own starting residual
            const double thresh = mixed ? tol * tol * rr : st->thresh;
            gs->rr0[r] = rr;
            gs->rr[r] = rr;
            gs->thresh[r] = thresh;
            if (mixed) {
                st->rr0 = rr;
                st->thresh = thresh;
            }
            st->rr = rr;
            st->iter = 0;
            st->status = SYLV_OK;
            st->done = act ? 0 : 1;
            gs->active[r] = act ? 1 : 0;
            if (act) {
                if (!isfinite(rr) || !isfinite(rz)) { st->status = SYLV_NONFINITE; st->done = 1; gs->active[r] = 0; }
                else if (rr <= thresh) { st->done = 1; gs->active[r] = 0; }
                else if (!(rz > 0.0)) { st->status = SYLV_BREAKDOWN; st->done = 1; gs->active[r] = 0; }
            }
            nact += gs->active[r];
        }
        for (int a = 0; a < S; ++a)
            for (int b = 0; b < S; ++b) {
                gs->rz[a][b] = q[pidx<S>(a, b)];
                gs->alpha[a][b] = 0.0;
                gs->beta[a][b] = 0.0;
            }
        gs->mode = BM_BLOCK;
        gs->restart = 0;
        gs->iter = 0;
        gs->done = nact == 0;
        return;
    }

    bool act0[S];   // columns active at entry (static loops keep the small arrays in registers)
#pragma unroll
    for (int r = 0; r < S; ++r) act0[r] = gs->active[r] != 0;

    if (phase == 1) {
        double alpha[S][S];
#pragma unroll
        for (int a = 0; a < S; ++a)
#pragma unroll
            for (int b = 0; b < S; ++b) alpha[a][b] = 0.0;
        bool ok = false;
        if (gs->mode == BM_BLOCK) {
            bool act[S];
#pragma unroll
            for (int r = 0; r < S; ++r) act[r] = gs->active[r] != 0;
            double l[S][S], x[S][S];
#pragma unroll
            for (int a = 0; a < S; ++a)
#pragma unroll
                for (int b = 0; b < S; ++b) {
                    const bool on = act[a] && act[b];
                    l[a][b] = on ? q[pidx<S>(a, b)] : (a == b ? 1.0 : 0.0);
                    x[a][b] = on ? gs->rz[a][b] : 0.0;
                }
            ok = chol_masked<S>(l, act);
            if (ok) {
                chol_solve_masked<S>(l, x);
#pragma unroll
                for (int a = 0; a < S; ++a)
#pragma unroll
                    for (int b = 0; b < S; ++b) {
                        if (!isfinite(x[a][b])) ok = false;
                        alpha[a][b] = x[a][b];
                    }
            }
            if (!ok) {
                gs->mode = BM_DIAG;
                gs->restart = 1;
#pragma unroll
                for (int a = 0; a < S; ++a)
#pragma unroll
                    for (int b = 0; b < S; ++b) alpha[a][b] = 0.0;
            }
        }
        if (gs->mode == BM_DIAG) {
#pragma unroll
            for (int r = 0; r < S; ++r) {
                if (!act0[r]) continue;
                const double pq = q[pidx<S>(r, r)];
                if (!isfinite(pq)) finish(r, SYLV_NONFINITE);
                else if (!(pq > 0.0)) finish(r, SYLV_BREAKDOWN);
                else alpha[r][r] = gs->rz[r][r] / pq;
            }
        }
#pragma unroll
        for (int a = 0; a < S; ++a)
#pragma unroll
            for (int b = 0; b < S; ++b) gs->alpha[a][b] = alpha[a][b];
        int left = 0;
        for (int r = 0; r < S; ++r) left += gs->active[r];
        gs->done = left == 0;
        return;
    }

    // phase 2
    gs->iter += 1;
#pragma unroll
    for (int r = 0; r < S; ++r) {
        if (!act0[r]) continue;
        const double rr = q[NG + r];
        gs->rr[r] = rr;
        DevState *st = state(r);
        st->rr = rr;
        st->iter = gs->iter;
        if (!isfinite(rr) || !isfinite(q[pidx<S>(r, r)])) finish(r, SYLV_NONFINITE);
        else if (rr <= gs->thresh[r]) finish(r, SYLV_OK);
        else if (gs->iter >= max_iter) finish(r, SYLV_NOT_CONVERGED);
    }
    bool act1[S];   // columns still active after this step's stopping tests
    int m = 0;
#pragma unroll
    for (int r = 0; r < S; ++r) {
        act1[r] = gs->active[r] != 0;
        m += act1[r] ? 1 : 0;
    }
    double beta[S][S];
#pragma unroll
    for (int a = 0; a < S; ++a)
#pragma unroll
        for (int b = 0; b < S; ++b) beta[a][b] = 0.0;
    if (gs->restart) {
        gs->restart = 0;
    } else if (gs->mode == BM_BLOCK && m > 0) {
        const bool (&act)[S] = act1;
        double l[S][S], x[S][S];
#pragma unroll
        for (int a = 0; a < S; ++a)
#pragma unroll
            for (int b = 0; b < S; ++b) {
                const bool on = act[a] && act[b];
                l[a][b] = on ? gs->rz[a][b] : (a == b ? 1.0 : 0.0);
                x[a][b] = on ? q[pidx<S>(a, b)] : 0.0;
            }
        bool ok = chol_masked<S>(l, act);
        if (ok) {
            chol_solve_masked<S>(l, x);
#pragma unroll
            for (int a = 0; a < S; ++a)
#pragma unroll
                for (int b = 0; b < S; ++b) {
                    if (!isfinite(x[a][b])) ok = false;
                    beta[a][b] = x[a][b];
                }
        }
        if (!ok) {   // restart as independent CG
            gs->mode = BM_DIAG;
#pragma unroll
            for (int a = 0; a < S; ++a)
#pragma unroll
                for (int b = 0; b < S; ++b) beta[a][b] = 0.0;
        }
    } else if (gs->mode == BM_DIAG) {
#pragma unroll
        for (int r = 0; r < S; ++r) {
            if (!act1[r]) continue;
            const double rzn = q[pidx<S>(r, r)], rzo = gs->rz[r][r];
            if (!(rzn > 0.0)) finish(r, SYLV_BREAKDOWN);
            else beta[r][r] = rzn / rzo;
        }
    }
#pragma unroll
    for (int a = 0; a < S; ++a)
#pragma unroll
        for (int b = 0; b < S; ++b) {
            gs->rz[a][b] = q[pidx<S>(a, b)];
            gs->beta[a][b] = beta[a][b];
        }
    int left = 0;
    for (int r = 0; r < S; ++r) left += gs->active[r];
    gs->done = left == 0;
}

// The block apply keeps every column's direction at its output pixels in registers: 2 rows per
// lane on every grid.
template <typename T, int K, int S, int SA>
hipError_t launch_bapply_sa(const GroupSet &gset, int total, const int *prefix, int it,
                            hipStream_t st) {
    const dim3 grid(total);
    if (gset.bc == SYLV_BC_FACE) {
        hipLaunchKernelGGL((k_bapply<T, K, kBlockRows, S, BC_FACE, SA>), grid, dim3(kBlock), 0, st,
                           gset.table, gset.groups, prefix, gset.ngroup, (int)grid.x, it);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_bapply<T, K, kBlockRows, S, BC_PERIODIC, SA>), grid, dim3(kBlock), 0, st,
                       gset.table, gset.groups, prefix, gset.ngroup, (int)grid.x, it);
    return hipGetLastError();
}

// Batches beyond the last-level cache stream the float32 stores (as the single-vector kernels).
template <typename T, int K, int S>
hipError_t launch_bapply_t(const GroupSet &gset, int total, const int *prefix, int it,
                           hipStream_t st) {
    if constexpr (sizeof(T) == 4)
        if (gset.stream) return launch_bapply_sa<T, K, S, kNT>(gset, total, prefix, it, st);
    return launch_bapply_sa<T, K, S, 0>(gset, total, prefix, it, st);
}

}  // namespace

// The launches of one right-hand-side count S in precision T (float: the inner runs of the mixed
// path, with streaming stores for batches beyond the last-level cache; double: float64 runs).
template <int S, typename T>
struct BlockLaunch {
    static hipError_t pinit(const GroupSet &g, int k, hipStream_t st);
    static hipError_t dir(const GroupSet &g, int k, int it, hipStream_t st);
    static hipError_t apply(const GroupSet &g, int k, int it, hipStream_t st);
    static hipError_t update(const GroupSet &g, int k, int it, hipStream_t st);
};

template <int S, typename T>
hipError_t BlockLaunch<S, T>::pinit(const GroupSet &g, int k, hipStream_t st) {
    return dispatch_k(k, [&](auto tag) {
        constexpr int K = decltype(tag)::value;
        const dim3 grid(g.total_chunks);
        hipLaunchKernelGGL((k_bpinit<T, K, S>), grid, dim3(kBlock), 0, st, g.table, g.groups,
                           g.gcprefix, g.ngroup, (int)grid.x);
        return hipGetLastError();
    });
}

template <int S, typename T>
hipError_t BlockLaunch<S, T>::dir(const GroupSet &g, int k, int it, hipStream_t st) {
    return dispatch_k(k, [&](auto tag) {
        constexpr int K = decltype(tag)::value;
        const dim3 grid(g.total_chunks);
        bool streamed = false;
        if constexpr (sizeof(T) == 4) {
            if (g.stream) {
                hipLaunchKernelGGL((k_bdir<T, K, S, kNT>), grid, dim3(kBlock), 0, st, g.table,
                                   g.groups, g.gcprefix, g.ngroup, (int)grid.x, it);
                streamed = true;
            }
        }
        if (!streamed)
            hipLaunchKernelGGL((k_bdir<T, K, S, 0>), grid, dim3(kBlock), 0, st, g.table, g.groups,
                               g.gcprefix, g.ngroup, (int)grid.x, it);
        return hipGetLastError();
    });
}

template <int S, typename T>
hipError_t BlockLaunch<S, T>::apply(const GroupSet &g, int k, int it, hipStream_t st) {
    return dispatch_k(k, [&](auto tag) {
        constexpr int K = decltype(tag)::value;
        if constexpr (sizeof(T) == 4)
            return launch_bapply_t<T, K, S>(g, g.total_tiles32, g.gtprefix32, it, st);
        else
            return launch_bapply_t<T, K, S>(g, g.total_tiles, g.gtprefix, it, st);
    });
}

template <int S, typename T>
hipError_t BlockLaunch<S, T>::update(const GroupSet &g, int k, int it, hipStream_t st) {
    return dispatch_k(k, [&](auto tag) {
        constexpr int K = decltype(tag)::value;
        const dim3 grid(g.total_chunks);
        bool streamed = false;
        if constexpr (sizeof(T) == 4) {
            if (g.stream) {
                hipLaunchKernelGGL((k_bupdate<T, K, S, kNT>), grid, dim3(kBlock), 0, st, g.table,
                                   g.groups, g.gcprefix, g.ngroup, (int)grid.x, it);
                streamed = true;
            }
        }
        if (!streamed)
            hipLaunchKernelGGL((k_bupdate<T, K, S, 0>), grid, dim3(kBlock), 0, st, g.table,
                               g.groups, g.gcprefix, g.ngroup, (int)grid.x, it);
        return hipGetLastError();
    });
}

// Instantiated in sylv_block_s<S>_<f32|f64>.hip only.
extern template struct BlockLaunch<2, float>;
extern template struct BlockLaunch<2, double>;
extern template struct BlockLaunch<4, float>;
extern template struct BlockLaunch<4, double>;
extern template struct BlockLaunch<8, float>;
extern template struct BlockLaunch<8, double>;

}  // namespace sylv
