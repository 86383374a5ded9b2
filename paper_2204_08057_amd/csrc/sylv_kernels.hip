// HIP kernels (gfx950) of the matrix-free preconditioned CG solve for the posterior mean of the
// CMB source-separation model (Section 3: eq. (Axb); Section 3.1 matrix-free products;
// Alg. 2 conjugate gradients).
//
// Data layout: every map is a plane of n_pix = ny * nx values, pixel p = iy * nx + ix, and a
// k-component field is k consecutive planes (component-major, the paper's stacking by map).
// Per-pixel k x k symmetric blocks (mixing M_p, preconditioner) are stored as k(k+1)/2 planes,
// upper triangle row by row.
//
// Work decomposition:
//  * operator apply: a workgroup owns a 64 x (4R) tile; each wavefront covers 64 consecutive
//    pixels of a row (coalesced accesses) and each lane walks R rows of one column, keeping a
//    register window of the 13-point stencil, so an interior value is fetched about 7 times per
//    R=4 outputs instead of 13 (the x-neighbours hit in L1).  The k x k mixing runs on VALU from
//    the packed block.
//  * streaming kernels: 4 consecutive pixels per lane, 16-byte vector accesses.
//  * reductions: shuffle tree in the wavefront, fixed-order sum of the 4 wavefronts, one
//    partial per workgroup.  No device-scope fence or atomic is used (on this multi-XCD part an
//    agent-scope release/acquire writes back and invalidates the XCD's L2): the kernel that
//    needs the reduced value re-reduces the partials in a fixed order at its start, after the
//    kernel boundary has made them visible.  Results are bitwise reproducible run to run.
//  * workgroup -> tile mapping is XCD-aware: consecutive workgroup ids are dealt round-robin to
//    the 8 XCDs, so ids are remapped to give every XCD a contiguous band of tiles, which keeps
//    stencil halos and shared per-pixel blocks in that XCD's L2.
//  * pointers read from the instance table are cast to the global address space so that
//    memory accesses compile to global_* rather than flat_* instructions.

#include <string.h>

#include <algorithm>

#include "sylv_device.h"

namespace sylv {
namespace {
using namespace dev;
// ---------------------------------------------------------------------------------------------
// Stencil coefficients of Q_j = tau (kappa^2 - Lap)^2 on the periodic 5-point Laplacian.
// Expanding the square with N4 = sum of the 4 edge neighbours (Lap = N4 - 4):
//   (kappa^2 + 4 - N4)^2 = (kappa^2+4)^2 - 2 (kappa^2+4) N4 + N4^2,
//   N4^2 = 4 (centre) + 2 (each of the 4 diagonal neighbours) + 1 (each of the 4 pixels at
//   distance 2 along an axis),
// so c0 = tau((kappa^2+4)^2 + 4), c1 = -2 tau (kappa^2+4), cd = 2 tau, c2 = tau.  Since the
// shift operators commute, the expansion is exact on every periodic grid; on grids with a side
// <= 2 several offsets land on the same pixel and their coefficients simply add, which is what
// the apply does with wrapped indices.  `diag` is the true diagonal of Q_j including those
// coincidences (used by the preconditioner).
__global__ void k_coef(const double *__restrict__ kappa, const double *__restrict__ tau, int k,
                       int ny, int nx, double *__restrict__ coef) {
    const int j = threadIdx.x;
    if (j >= k) return;
    const double kp = kappa[j], t = tau[j];
    const double s = kp * kp + 4.0;
    const double c0 = t * (s * s + 4.0), c1 = -2.0 * t * s, cd = 2.0 * t, c2 = t;
    double dg = c0;
    dg += 2.0 * c1 * ((nx == 1 ? 1.0 : 0.0) + (ny == 1 ? 1.0 : 0.0));
    dg += 4.0 * cd * ((nx == 1 && ny == 1) ? 1.0 : 0.0);
    dg += 2.0 * c2 * ((nx <= 2 ? 1.0 : 0.0) + (ny <= 2 ? 1.0 : 0.0));
    double *c = coef + j * kCoefStride;
    c[0] = c0; c[1] = c1; c[2] = cd; c[3] = c2; c[4] = dg; c[5] = kp; c[6] = t; c[7] = 0.0;
}

// Per-pixel mixing block M_p = sum_f W[f,p] a_f a_f^T (the block map N (M A^T) T A of
// Section 3.1 done pixel by pixel) and the preconditioner: block-Jacobi inverts
// diag_j(Q_j diagonal) + M_p by a k x k Cholesky factorisation in float64.  A block that is not
// positive definite (negative tau, say) gets NaN entries so the solve reports it.
template <int K>
__global__ __launch_bounds__(kBlock) void k_setup(const double *__restrict__ W,
                                                  const double *__restrict__ A, int f, int ny,
                                                  int nx, int bc,
                                                  const double *__restrict__ coef, int pc,
                                                  double *__restrict__ M64, float *__restrict__ M32,
                                                  double *__restrict__ P64, float *__restrict__ P32,
                                                  unsigned short *__restrict__ P16, int exact) {
    constexpr int MK = K * (K + 1) / 2;
    const int n_pix = ny * nx;
    const int pix = blockIdx.x * kBlock + threadIdx.x;
    if (pix >= n_pix) return;
    // diagonal of Q_j at this pixel: periodic grids share one value (with the wrap coincidences
    // of tiny grids); on a face it is tau ((kappa^2 + d)^2 + d), d = in-face neighbours
    double qd[K];
    {
        const int iy = pix / nx, ix = pix - iy * nx;
        const double d = (double)face_deg(ix, iy, nx, ny);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const double *cj = coef + j * kCoefStride;
            const double e = cj[5] * cj[5] + d;
            qd[j] = (bc == SYLV_BC_FACE) ? cj[6] * (e * e + d) : cj[4];
        }
    }
    double m[MK];
#pragma unroll
    for (int e = 0; e < MK; ++e) m[e] = 0.0;
    for (int fi = 0; fi < f; ++fi) {
        const double w = W[(size_t)fi * n_pix + pix];
        double a[K];
#pragma unroll
        for (int j = 0; j < K; ++j) a[j] = A[fi * K + j];
#pragma unroll
        for (int i = 0; i < K; ++i)
#pragma unroll
            for (int j = i; j < K; ++j) m[pidx<K>(i, j)] += w * a[i] * a[j];
    }
#pragma unroll
    for (int e = 0; e < MK; ++e) {
        M64[(size_t)e * n_pix + pix] = m[e];
        M32[(size_t)e * n_pix + pix] = (float)m[e];
    }
    if (pc == SYLV_PC_JACOBI) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const double d = 1.0 / (qd[j] + m[pidx<K>(j, j)]);
            if (exact) {
                P64[(size_t)j * n_pix + pix] = d;
                P32[(size_t)j * n_pix + pix] = (float)d;
            }
            P16[(size_t)j * n_pix + pix] = bf16_round((float)d);
        }
    } else if (pc == SYLV_PC_BLOCK) {
        double a[K][K], l[K][K];
#pragma unroll
        for (int i = 0; i < K; ++i)
#pragma unroll
            for (int j = 0; j < K; ++j) {
                a[i][j] = m[pidx<K>(i, j)] + (i == j ? qd[i] : 0.0);
                l[i][j] = 0.0;
            }
        bool ok = true;
#pragma unroll
        for (int c = 0; c < K; ++c) {
            double s = a[c][c];
#pragma unroll
            for (int t = 0; t < c; ++t) s -= l[c][t] * l[c][t];
            ok = ok && (s > 0.0);
            const double d = sqrt(s > 0.0 ? s : 1.0);
            l[c][c] = d;
            const double inv = 1.0 / d;
#pragma unroll
            for (int r = c + 1; r < K; ++r) {
                double v = a[r][c];
#pragma unroll
                for (int t = 0; t < c; ++t) v -= l[r][t] * l[c][t];
                l[r][c] = v * inv;
            }
        }
        // inverse = L^-T L^-1, column by column; y = L^-1 e_col is column col of G = L^-1
        const double bad = ok ? 0.0 : __builtin_nan("");
        double inv[K][K];
#pragma unroll
        for (int col = 0; col < K; ++col) {
            double y[K];
#pragma unroll
            for (int r = 0; r < K; ++r) {
                double v = (r == col) ? 1.0 : 0.0;
#pragma unroll
                for (int t = 0; t < r; ++t) v -= l[r][t] * y[t];
                y[r] = v / l[r][r];
            }
#pragma unroll
            for (int r = col; r < K; ++r)
                P16[(size_t)pidx<K>(col, r) * n_pix + pix] = bf16_round((float)(y[r] + bad));
#pragma unroll
            for (int r = K - 1; r >= 0; --r) {
                double v = y[r];
#pragma unroll
                for (int t = r + 1; t < K; ++t) v -= l[t][r] * inv[t][col];
                inv[r][col] = v / l[r][r];
            }
        }
        if (exact) {
#pragma unroll
            for (int i = 0; i < K; ++i)
#pragma unroll
                for (int j = i; j < K; ++j) {
                    const double v = 0.5 * (inv[i][j] + inv[j][i]) + bad;
                    P64[(size_t)pidx<K>(i, j) * n_pix + pix] = v;
                    P32[(size_t)pidx<K>(i, j) * n_pix + pix] = (float)v;
                }
        }
    }
}

// Right-hand side b = B^T C Y (+ extra): b[j,p] = sum_f W[f,p] Y[f,p] A[f,j] (eq. (mu*)).
template <int K>
__global__ __launch_bounds__(kBlock) void k_rhs(const double *__restrict__ W,
                                                const double *__restrict__ Y,
                                                const double *__restrict__ A, int f, int n_pix,
                                                const double *__restrict__ bext,
                                                double *__restrict__ b) {
    const int pix = blockIdx.x * kBlock + threadIdx.x;
    if (pix >= n_pix) return;
    double acc[K];
#pragma unroll
    for (int j = 0; j < K; ++j) acc[j] = bext ? bext[(size_t)j * n_pix + pix] : 0.0;
    if (Y) {
        for (int fi = 0; fi < f; ++fi) {
            const double wy = W[(size_t)fi * n_pix + pix] * Y[(size_t)fi * n_pix + pix];
#pragma unroll
            for (int j = 0; j < K; ++j) acc[j] += wy * A[fi * K + j];
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) b[(size_t)j * n_pix + pix] = acc[j];
}

// ---------------------------------------------------------------------------------------------
// Operator apply G(u) = sum_j Q_j u_j + M_p u_p, fused variants:
//   AM_PLAIN : out = G(in)                                       (stand-alone apply)
//   AM_CG    : iteration `it` of Alg. 2 with preconditioner.  First the stopping test on the
//              residual left by the previous update (its <r,z> and ||r||^2 partials), then
//              beta = rho_it / rho_(it-1), u = z + beta p_old (u = z at it = 0), p_new <- u,
//              q = G(u) and the <p, q> partials.
//   AM_RESID : r = b - G(x) and the ||r||^2, ||b||^2 partials   (initial / true residual)
enum ApplyMode { AM_PLAIN = 0, AM_CG = 1, AM_RESID = 2 };

// CP: cache policy of the data this kernel touches once (bit 0: the per-pixel mixing blocks, b
// and the interior x / p_(it-2) loads; bit 1: every store) -- non-temporal when the solve's
// working set exceeds the last-level cache (the staged fields keep the default: their halos are
// re-read by neighbouring tiles through the cache).
template <typename T, int K, int R, int MODE, int BC, int CP>
__global__ __launch_bounds__(kBlock) void k_apply(const Inst *__restrict__ tab,
                                                  const int *__restrict__ tprefix, int ninst,
                                                  int nb, int it,
                                                  const T *__restrict__ ext_in,
                                                  T *__restrict__ ext_out) {
    constexpr int MK = K * (K + 1) / 2;
    constexpr int LH = kWavesY * R + 4;   // staged rows: tile + 2-row halo above and below
    constexpr int LW = kTileX + 4;        // staged columns: tile + 2-column halo left and right
    constexpr int RPW = LH / kWavesY;     // staged rows per wavefront
    constexpr int LA = (CP & 1) ? kNT : 0, SA = (CP & 2) ? kNT : 0;
    const int L = xcd_remap(blockIdx.x, nb);
    const int ii = (MODE == AM_PLAIN) ? 0 : find_inst(tprefix, ninst, L);
    const Inst &I = tab[ii];
    const int tile = (MODE == AM_PLAIN) ? L : L - tprefix[ii];
    const int nx = I.nx, ny = I.ny, n_pix = I.n_pix;
    const uint32_t np = (uint32_t)n_pix;   // plane length for buffer accesses
    DevState *st = (MODE == AM_CG) ? Sel<T>::st(I) : nullptr;
    if constexpr (MODE == AM_CG) {
        if (st->done) return;
    } else if constexpr (MODE == AM_RESID) {
        // `it` is the residual phase; a refinement step (2) of a finished run is a no-op, as is
        // the reduction that would read these partials
        if (it == 2 && I.st->done) return;
    }

    // u = field to apply: the input (plain), x (residual), or z + beta p_old (CG; z alone at
    // it = 0, where p_old is aliased to z so that no uninitialised value is ever read).
    const GAS T *u0;
    const GAS T *u1 = nullptr;
    if constexpr (MODE == AM_PLAIN) {
        u0 = gp(ext_in) + (size_t)blockIdx.y * K * n_pix;
    } else if constexpr (MODE == AM_CG) {
        u1 = Sel<T>::z(I);
        u0 = (it == 0) ? u1 : (const GAS T *)Sel<T>::p(I, it);
    } else {
        u0 = (const GAS T *)gp(I.x);
    }

    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int tile_x = tile % I.tiles_x, tile_y = tile / I.tiles_x;
    const int x0 = tile_x * kTileX, y0 = tile_y * kWavesY * R;
    const int ix = x0 + tx;
    const int iy0 = y0 + ty * R;
    const bool active = (ix < nx) && (iy0 < ny);

    // ---- issue every global load of the tile before any barrier ---------------------------
    // Staging: rows by whole wavefronts (coalesced), the 4 halo columns of all rows by one lane
    // each.  Every staged column is the periodic wrap of x0 - 2 + c, so ragged tiles see true
    // neighbours.
    const int cmain = wrapf(x0 + tx, nx);
    const int hitem = ty * 64 + tx;                     // halo item: (row, one of 4 columns)
    const int hr = hitem >> 2, hc = hitem & 3;
    const int hcol = (hc < 2) ? hc : (kTileX + hc);     // staged columns 0, 1, 66, 67
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
    T sa[K][RPW], sb[K][RPW], ha[K], hb[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const GAS T *a = u0 + (size_t)j * n_pix;
#pragma unroll
        for (int rr = 0; rr < RPW; ++rr) sa[j][rr] = sin[rr] ? bld(a, np, soff[rr]) : (T)0;
        ha[j] = hin ? bld(a, np, hoff) : (T)0;
        if constexpr (MODE == AM_CG) {
            const GAS T *zz = u1 + (size_t)j * n_pix;
#pragma unroll
            for (int rr = 0; rr < RPW; ++rr) sb[j][rr] = sin[rr] ? bld(zz, np, soff[rr]) : (T)0;
            hb[j] = hin ? bld(zz, np, hoff) : (T)0;
        }
    }
    // CG: x += alpha_(it-1) p_(it-1) on the staged interior values (each pixel of the grid is
    // interior to exactly one tile).  Float64 runs advance x every second iteration instead: even
    // it >= 2 adds alpha_(it-2) p_(it-2) and then alpha_(it-1) p_(it-1) (the rounding of two single
    // steps), odd it touches x only when the run stops there; p_(it-2) is read at this
    // workgroup's own interior pixels from the buffer that receives p_it at the same pixels below,
    // so no other workgroup overwrites it first.  That saves half of the x traffic; the float32
    // apply is latency-bound at these sizes and runs faster with one step per iteration.
    constexpr bool kPairX = sizeof(T) == 8;
    const bool pair = kPairX && it >= 2 && (it & 1) == 0;   // this apply adds two steps
    const bool xnow = it > 0 && (!kPairX || pair);           // x advances here in any case
    T xs[K][RPW], po[K][RPW];
    bool xin[RPW];
    if constexpr (MODE == AM_CG) {
#pragma unroll
        for (int rr = 0; rr < RPW; ++rr) {
            const int r = rr * kWavesY + ty;
            xin[rr] = it > 0 && r >= 2 && r < LH - 2 && (y0 + r - 2) < ny && (x0 + tx) < nx;
        }
        if (xnow) {
            const GAS T *xx = Sel<T>::x(I);
            const GAS T *p2 = Sel<T>::p(I, it + 1);
#pragma unroll
            for (int j = 0; j < K; ++j)
#pragma unroll
                for (int rr = 0; rr < RPW; ++rr) {
                    xs[j][rr] = xin[rr] ? bld<LA>(xx + (size_t)j * n_pix, np, soff[rr]) : (T)0;
                    if (pair) po[j][rr] = xin[rr] ? bld<LA>(p2 + (size_t)j * n_pix, np, soff[rr]) : (T)0;
                }
        }
    }
    // per-pixel mixing blocks (and, for the residual, b) of this lane's R output pixels
    T m[R][MK];
    double bpre[R][K];
    {
        const GAS T *M = Sel<T>::M(I);
        const int ixc = ix < nx ? ix : 0;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int pix = (iy0 + t < ny ? iy0 + t : 0) * nx + ixc;
#pragma unroll
            for (int e = 0; e < MK; ++e) m[t][e] = bld<LA>(M + (size_t)e * n_pix, np, (uint32_t)pix);
            if constexpr (MODE == AM_RESID) {
                const GAS double *bb = gp(I.b);
#pragma unroll
                for (int j = 0; j < K; ++j) bpre[t][j] = bld<LA>(bb + (size_t)j * n_pix, np, (uint32_t)pix);
            }
        }
    }

    // ---- CG: stopping test on the last update's residual, then beta -----------------------
    T beta = 0;
    if constexpr (MODE == AM_CG) {
        double s[2];
        if (I.pc == SYLV_PC_FOURIER && !I.pre) {
            // <r, z> from the Fourier preconditioner's column pass, ||r||^2 from its row pass
            consume_pair(I.partial, I.nred, SLOT_FRZ, I.nfft, SLOT_RR, I.nrr, s);
        } else {
            consume<2>(I.partial, I.nred, SLOT_RZ, I.pre ? 1 : I.nchunks, s);
        }
        const double rz = s[0], rr = s[1];
        // float64 runs stop against ||b - G x0|| (threshold set by the initial residual pass,
        // also across restarts); a float32 inner run against its own starting residual
        const double thresh = (it == 0 && sizeof(T) == 4) ? st->tol * st->tol * rr : st->thresh;
        int status = -1;
        if (!finite_d(rz) || !finite_d(rr)) status = SYLV_NONFINITE;
        else if (rr <= thresh) status = SYLV_OK;
        else if (!(rz > 0.0)) status = SYLV_BREAKDOWN;
        else if (it >= st->max_iter) status = SYLV_NOT_CONVERGED;
        if (tile == 0 && threadIdx.x == 0) {
            st->iter = it;
            st->rr = rr;
            st->rho[it & 1] = rz;
            st->pend = status;
            if (it == 0 && sizeof(T) == 4) { st->rr0 = rr; st->thresh = thresh; }
        }
        if (it > 0 && (xnow || status >= 0)) {   // x_it, also when the run stops here
            const T a1 = (T)st->alpha[(it - 1) & 1];
            GAS T *xx = Sel<T>::x(I);
            if (pair) {
                const T a2 = (T)st->alpha[it & 1];   // alpha_(it-2): update(it) has not run yet
#pragma unroll
                for (int j = 0; j < K; ++j)
#pragma unroll
                    for (int rr2 = 0; rr2 < RPW; ++rr2)
                        if (xin[rr2]) {
                            const T x1 = xs[j][rr2] + a2 * po[j][rr2];
                            bst<SA>(xx + (size_t)j * n_pix, np, soff[rr2], x1 + a1 * sa[j][rr2]);
                        }
            } else if (xnow) {
#pragma unroll
                for (int j = 0; j < K; ++j)
#pragma unroll
                    for (int rr2 = 0; rr2 < RPW; ++rr2)
                        if (xin[rr2]) bst<SA>(xx + (size_t)j * n_pix, np, soff[rr2], xs[j][rr2] + a1 * sa[j][rr2]);
            } else {   // float64, odd it: the run stops here; alpha_(it-2) p_(it-2) is in x
#pragma unroll
                for (int j = 0; j < K; ++j)
#pragma unroll
                    for (int rr2 = 0; rr2 < RPW; ++rr2)
                        if (xin[rr2]) {
                            const T x0v = bld<LA>(xx + (size_t)j * n_pix, np, soff[rr2]);
                            bst<SA>(xx + (size_t)j * n_pix, np, soff[rr2], x0v + a1 * sa[j][rr2]);
                        }
            }
        }
        if (status >= 0) return;
        if (it > 0) beta = (T)(rz / st->rho[(it - 1) & 1]);
    }

    // ---- stage u in LDS ---------------------------------------------------------------------
    __shared__ T lds[K][LH][LW];
#pragma unroll
    for (int j = 0; j < K; ++j) {
#pragma unroll
        for (int rr = 0; rr < RPW; ++rr) {
            T v = sa[j][rr];
            if constexpr (MODE == AM_CG) v = sb[j][rr] + beta * v;
            lds[j][rr * kWavesY + ty][tx + 2] = v;
        }
        if (hvalid) {
            T v = ha[j];
            if constexpr (MODE == AM_CG) v = hb[j] + beta * v;
            lds[j][hr][hcol] = v;
        }
    }
    __syncthreads();

    // ---- 13-point stencil from LDS, k x k mixing, stores and dot partials --------------------
    double d0 = 0.0, d1 = 0.0;
    if (active) {
        const int lr = ty * R;   // first staged row of this wavefront's window
        T acc[K][R];
        T ctr[K][R];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const double *cj = I.coef + j * kCoefStride;
            const T c0 = (T)cj[0], c1 = (T)cj[1], cd = (T)cj[2], c2 = (T)cj[3];
            const T tj = (T)cj[6], k2 = (T)(cj[5] * cj[5]);
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
                    // tau ((kappa^2 + d_p)^2 + d_p) at the centre, -tau (2 kappa^2 + d_p + d_q)
                    // at edge neighbour q (absent neighbours are staged as 0)
                    const int iy = iy0 + t;
                    const T dp = (T)face_deg(ix, iy, nx, ny);
                    const T e0 = k2 + dp, b0 = (T)2 * k2 + dp;
                    const T en = (b0 + (T)face_deg(ix, iy - 1, nx, ny)) * cc[t + 1] +
                                 (b0 + (T)face_deg(ix, iy + 1, nx, ny)) * cc[t + 3] +
                                 (b0 + (T)face_deg(ix - 1, iy, nx, ny)) * l1[t + 1] +
                                 (b0 + (T)face_deg(ix + 1, iy, nx, ny)) * r1[t + 1];
                    acc[j][t] = tj * (e0 * e0 + dp) * cc[t + 2] - tj * en + cd * d4 + c2 * f4;
                } else {
                    const T n4 = (cc[t + 1] + cc[t + 3]) + (l1[t + 1] + r1[t + 1]);
                    acc[j][t] = c0 * cc[t + 2] + c1 * n4 + cd * d4 + c2 * f4;
                }
                ctr[j][t] = cc[t + 2];
            }
        }
#pragma unroll
        for (int t = 0; t < R; ++t) {
            if (iy0 + t < ny) {
                const int pix = (iy0 + t) * nx + ix;
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    T sum = acc[j][t];
#pragma unroll
                    for (int i = 0; i < K; ++i) sum += m[t][pidx<K>(j, i)] * ctr[i][t];
                    acc[j][t] = sum;
                }
                if constexpr (MODE == AM_PLAIN) {
                    GAS T *o = gp(ext_out) + (size_t)blockIdx.y * K * n_pix;
#pragma unroll
                    for (int j = 0; j < K; ++j) bst<SA>(o + (size_t)j * n_pix, np, (uint32_t)pix, acc[j][t]);
                } else if constexpr (MODE == AM_CG) {
                    GAS T *pp = Sel<T>::p(I, it + 1);
                    GAS T *qq = Sel<T>::q(I);
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        bst<SA>(pp + (size_t)j * n_pix, np, (uint32_t)pix, ctr[j][t]);
                        bst<SA>(qq + (size_t)j * n_pix, np, (uint32_t)pix, acc[j][t]);
                        d0 += (double)ctr[j][t] * (double)acc[j][t];
                    }
                } else {
                    GAS double *rv = gp(I.r);
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        const double bv = bpre[t][j];
                        const double res = bv - (double)acc[j][t];
                        bst<SA>(rv + (size_t)j * n_pix, np, (uint32_t)pix, res);
                        d0 += res * res;
                        d1 += bv * bv;
                    }
                }
            }
        }
    }
    if constexpr (MODE == AM_CG) {
        double v[1] = {d0};
        block_partials<1>(v, I.partial, I.nred, SLOT_PQ, tile);
    } else if constexpr (MODE == AM_RESID) {
        double v[2] = {d0, d1};
        block_partials<2>(v, I.partial, I.nred, SLOT_RES_RR, tile);
    }
}

// Reduction of the residual pass (one workgroup per instance).
//   phase 0: initial residual: ||b||^2, ||r0||^2, threshold tol^2 ||r0||^2
//   phase 1: true residual of the result (relres_true only)
//   phase 2: refinement step of the mixed path: converged / stagnated / failed inner run
__global__ __launch_bounds__(kBlock) void k_resid_fin(const Inst *__restrict__ tab, int phase) {
    const Inst &I = tab[blockIdx.x];
    DevState *st = I.st;
    if (phase == 2 && st->done) return;
    double s[2];
    consume<2>(I.partial, I.nred, SLOT_RES_RR, I.ntiles, s);
    if (threadIdx.x != 0) return;
    const double rr = s[0];
    if (phase == 0) {
        st->bb = s[1];
        st->rr0 = rr;
        st->rr = rr;
        st->rr_prev = rr;
        // Alg. 2's test is relative to the initial residual; warm starts over a parameter
        // sweep may ask for ||b|| instead
        st->thresh = st->tol * st->tol * (st->ref == SYLV_STOP_B ? s[1] : rr);
        if (!finite_d(rr) || !finite_d(s[1])) { st->status = SYLV_NONFINITE; st->done = 1; }
        else if (rr == 0.0) { st->status = SYLV_OK; st->done = 1; }
    } else if (phase == 2) {
        const int inner = I.st_in->status;
        st->rr = rr;
        st->outer += 1;
        if (!finite_d(rr)) {
            st->status = SYLV_NONFINITE; st->done = 1;
        } else if (rr <= st->thresh) {
            st->status = SYLV_OK; st->done = 1;
        } else if (inner == SYLV_NONFINITE || inner == SYLV_BREAKDOWN) {
            st->status = inner; st->done = 1;
        } else if (rr > 0.25 * st->rr_prev) {
            st->status = SYLV_STAGNATED; st->done = 1;
        }
        st->rr_prev = rr;
    }
    if (phase == 1) {
        // residual replacement: a float64 run whose recursive residual met the threshold but
        // whose recomputed residual did not (rounding drift of the recurrence) is reopened and
        // restarted from its current x by the host
        st->outer += 1;
        if (st->status == SYLV_OK && st->done && finite_d(rr) && rr > st->thresh &&
            st->outer <= kMaxRestarts)
            st->done = 0;
    }
    const double bb = st->bb;
    st->rel_true = (bb > 0.0) ? sqrt(rr / bb) : sqrt(rr);
}

// ---------------------------------------------------------------------------------------------
// CG vector update of Alg. 2 (iteration `it`) with the preconditioner fused in:
//   alpha = rho / <p, q> (from the apply's partials), r -= alpha q, z = Pinv r, and the
//   <r, z>, ||r||^2 partials for the next stopping test and beta.  The matching x += alpha p is
//   done by the next iteration's apply, which reads p anyway (alpha is kept in the state).
// T = double: the float64 run.  T = float: an inner run of the mixed path.
// CP as for k_apply (bit 0: the loads of r, q and the preconditioner factor; bit 1: the stores).
template <typename T, int K, int CP>
__global__ __launch_bounds__(kBlock) void k_update(const Inst *__restrict__ tab,
                                                   const int *__restrict__ cprefix, int ninst,
                                                   int nb, int it) {
    constexpr int LA = (CP & 1) ? kNT : 0, SA = (CP & 2) ? kNT : 0;
    const int L = xcd_remap(blockIdx.x, nb);
    const int ii = find_inst(cprefix, ninst, L);
    const Inst &I = tab[ii];
    const int chunk = L - cprefix[ii];
    DevState *st = Sel<T>::st(I);
    if (st->done) return;
    const int pend = st->pend;
    if (pend >= 0) {   // this iteration's apply stopped the run
        if (chunk == 0 && threadIdx.x == 0) {
            st->status = pend;
            st->done = 1;
            st->total_iter += it;
        }
        return;
    }
    const int n_pix = I.n_pix;
    const uint32_t np = (uint32_t)n_pix;   // plane length for buffer accesses
    GAS T *r = Sel<T>::r(I);
    GAS T *z = Sel<T>::z(I);
    const GAS T *q = Sel<T>::q(I);
    const GAS unsigned short *P = Pcg(I);
    const int pc = I.pc;
    const int p0 = chunk * kChunk + threadIdx.x * 4;
    const bool vec = I.vec4 && p0 + 4 <= n_pix;
    // issue the vector loads before the reduction of the apply's partials
    T rv[K][4], qv[K][4];
    if (vec) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            bld4<LA>(r + (size_t)j * n_pix, np, (uint32_t)p0, rv[j]);
            bld4<LA>(q + (size_t)j * n_pix, np, (uint32_t)p0, qv[j]);
        }
    }
    double s[1];
    consume<1>(I.partial, I.nred, SLOT_PQ, I.pre ? 1 : (sizeof(T) == 4 ? I.ntiles32 : I.ntiles), s);
    const double pq = s[0];
    int status = -1;
    if (!finite_d(pq)) status = SYLV_NONFINITE;
    else if (!(pq > 0.0)) status = SYLV_BREAKDOWN;
    const double alpha_d = st->rho[it & 1] / pq;
    if (chunk == 0 && threadIdx.x == 0) {
        if (status >= 0) {
            st->status = status;
            st->done = 1;
            st->total_iter += it;
        } else {
            st->alpha[it & 1] = alpha_d;
        }
    }
    if (status >= 0) return;
    const T alpha = (T)alpha_d;
    double rz = 0.0, rr = 0.0;
    if (p0 < n_pix) {
        if (vec) {
            T zv[K][4];
#pragma unroll
            for (int j = 0; j < K; ++j) {
#pragma unroll
                for (int e = 0; e < 4; ++e) rv[j][e] -= alpha * qv[j][e];
                bst4<SA>(r + (size_t)j * n_pix, np, (uint32_t)p0, rv[j]);
            }
            if (pc == SYLV_PC_FOURIER) {   // z and <r, z> come from the Fourier passes
#pragma unroll
                for (int j = 0; j < K; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) rr += (double)rv[j][e] * (double)rv[j][e];
            } else {
                precond_cg_vec4<T, K, LA>(pc, P, n_pix, p0, rv, zv);
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    bst4<SA>(z + (size_t)j * n_pix, np, (uint32_t)p0, zv[j]);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        rz += (double)rv[j][e] * (double)zv[j][e];
                        rr += (double)rv[j][e] * (double)rv[j][e];
                    }
                }
            }
        } else {
            for (int e = 0; e < 4 && p0 + e < n_pix; ++e) {
                const int pix = p0 + e;
                T rs[K], zs[K];
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    const size_t o = (size_t)j * n_pix + pix;
                    rs[j] = r[o] - alpha * q[o];
                    r[o] = rs[j];
                }
                if (pc == SYLV_PC_FOURIER) {
#pragma unroll
                    for (int j = 0; j < K; ++j) rr += (double)rs[j] * (double)rs[j];
                    continue;
                }
                precond_cg_pixel<T, K>(pc, P, n_pix, pix, rs, zs);
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    z[(size_t)j * n_pix + pix] = zs[j];
                    rz += (double)rs[j] * (double)zs[j];
                    rr += (double)rs[j] * (double)rs[j];
                }
            }
        }
    }
    double v[2] = {rz, rr};
    block_partials<2>(v, I.partial, I.nred, SLOT_RZ, chunk);
}

// Start of a CG run: z0 = Pinv r0 and the <r0, z0>, ||r0||^2 partials (the stopping test and
// threshold are taken by the first apply).
// T = double: r is the float64 residual of the float64 run.
// T = float : start of an inner run of the mixed path: the float64 outer residual I.r is
//             rounded to float32 (r32), the correction d32 is zeroed, and the inner tolerance
//             asks for the reduction that brings the outer residual to tolerance (times the
//             `safety` factor), but never less than `inner_tol` nor more than 0.1.
template <typename T, int K>
__global__ __launch_bounds__(kBlock) void k_pinit(const Inst *__restrict__ tab,
                                                  const int *__restrict__ cprefix, int ninst,
                                                  int nb, double inner_tol, double safety,
                                                  int max_iter) {
    const int L = xcd_remap(blockIdx.x, nb);
    const int ii = find_inst(cprefix, ninst, L);
    const Inst &I = tab[ii];
    const int chunk = L - cprefix[ii];
    DevState *st = Sel<T>::st(I);
    const DevState *outer = I.st;
    if (outer->done) {
        if constexpr (sizeof(T) == 4) {
            if (chunk == 0 && threadIdx.x == 0) { st->done = 1; st->status = SYLV_OK; }
        }
        return;
    }
    if (chunk == 0 && threadIdx.x == 0) {
        st->iter = 0;
        st->pend = -1;
        st->max_iter = max_iter;
        if constexpr (sizeof(T) == 4) {
            st->done = 0;
            st->status = SYLV_OK;
            const double need = safety * sqrt(outer->thresh / fmax(outer->rr, 1e-300));
            st->tol = fmin(0.1, fmax(inner_tol, need));
        }
    }
    const int n_pix = I.n_pix;
    const uint32_t np = (uint32_t)n_pix;   // plane length for buffer accesses
    const GAS double *r64 = gp(I.r);
    GAS T *rr_out = Sel<T>::r(I);
    GAS T *z = Sel<T>::z(I);
    const GAS unsigned short *P = Pcg(I);
    const int pc = I.pc;
    const int p0 = chunk * kChunk + threadIdx.x * 4;
    double rz = 0.0, rr = 0.0;
    if (I.vec4 && p0 + 4 <= n_pix) {
        T rv[K][4], zv[K][4];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const size_t o = (size_t)j * n_pix;
            double r4[4];
            bld4(r64 + o, np, (uint32_t)p0, r4);
#pragma unroll
            for (int e = 0; e < 4; ++e) rv[j][e] = (T)r4[e];
            if constexpr (sizeof(T) == 4) {
                bst4(rr_out + o, np, (uint32_t)p0, rv[j]);
                const float zero4[4] = {0.f, 0.f, 0.f, 0.f};
                bst4(gp(I.d32) + o, np, (uint32_t)p0, zero4);
            }
        }
        if (pc == SYLV_PC_FOURIER) {   // z and <r, z> come from the Fourier passes
#pragma unroll
            for (int j = 0; j < K; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) rr += (double)rv[j][e] * (double)rv[j][e];
        } else {
            precond_cg_vec4<T, K>(pc, P, n_pix, p0, rv, zv);
#pragma unroll
            for (int j = 0; j < K; ++j) {
                bst4(z + (size_t)j * n_pix, np, (uint32_t)p0, zv[j]);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    rz += (double)rv[j][e] * (double)zv[j][e];
                    rr += (double)rv[j][e] * (double)rv[j][e];
                }
            }
        }
    } else {
        for (int e = 0; e < 4 && p0 + e < n_pix; ++e) {
            const int pix = p0 + e;
            T rv[K], zv[K];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const size_t o = (size_t)j * n_pix + pix;
                rv[j] = (T)r64[o];
                if constexpr (sizeof(T) == 4) {
                    rr_out[o] = rv[j];
                    gp(I.d32)[o] = 0.0f;
                }
            }
            if (pc == SYLV_PC_FOURIER) {
#pragma unroll
                for (int j = 0; j < K; ++j) rr += (double)rv[j] * (double)rv[j];
                continue;
            }
            precond_cg_pixel<T, K>(pc, P, n_pix, pix, rv, zv);
#pragma unroll
            for (int j = 0; j < K; ++j) {
                z[(size_t)j * n_pix + pix] = zv[j];
                rz += (double)rv[j] * (double)zv[j];
                rr += (double)rv[j] * (double)rv[j];
            }
        }
    }
    double v[2] = {rz, rr};
    block_partials<2>(v, I.partial, I.nred, SLOT_RZ, chunk);
}

// Mixed path: x += d (float32 correction promoted to float64), for instances still refining.
template <int K>
__global__ __launch_bounds__(kBlock) void k_refine_axpy(const Inst *__restrict__ tab,
                                                        const int *__restrict__ cprefix,
                                                        int ninst, int nb) {
    const int L = xcd_remap(blockIdx.x, nb);
    const int ii = find_inst(cprefix, ninst, L);
    const Inst &I = tab[ii];
    if (I.st->done) return;
    const int st_in = I.st_in->status;
    if (st_in == SYLV_NONFINITE || st_in == SYLV_BREAKDOWN) return;
    const int chunk = L - cprefix[ii];
    const int n_pix = I.n_pix;
    const uint32_t np = (uint32_t)n_pix;   // plane length for buffer accesses
    const int p0 = chunk * kChunk + threadIdx.x * 4;
    GAS double *x = gp(I.x);
    const GAS float *d = gp(I.d32);
    if (I.vec4 && p0 + 4 <= n_pix) {
        double xv[K][4];
        float dv[K][4];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            bld4(x + (size_t)j * n_pix, np, (uint32_t)p0, xv[j]);
            bld4(d + (size_t)j * n_pix, np, (uint32_t)p0, dv[j]);
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
#pragma unroll
            for (int e = 0; e < 4; ++e) xv[j][e] += (double)dv[j][e];
            bst4(x + (size_t)j * n_pix, np, (uint32_t)p0, xv[j]);
        }
        return;
    }
    for (int e = 0; e < 4 && p0 + e < n_pix; ++e) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const size_t o = (size_t)j * n_pix + p0 + e;
            x[o] += (double)d[o];
        }
    }
}

// Stand-alone preconditioner apply: out = Pinv in.
template <typename T, int K>
__global__ __launch_bounds__(kBlock) void k_precond_plain(const Inst *__restrict__ tab,
                                                          const T *__restrict__ in,
                                                          T *__restrict__ out) {
    const Inst &I = tab[0];
    const int n_pix = I.n_pix;
    const int pix = blockIdx.x * kBlock + threadIdx.x;
    if (pix >= n_pix) return;
    const T *src = in + (size_t)blockIdx.y * K * n_pix;
    T *dst = out + (size_t)blockIdx.y * K * n_pix;
    T rv[K], zv[K];
#pragma unroll
    for (int j = 0; j < K; ++j) rv[j] = src[(size_t)j * n_pix + pix];
    precond_pixel<T, K>(I.pc, Sel<T>::P(I), n_pix, pix, rv, zv);
#pragma unroll
    for (int j = 0; j < K; ++j) dst[(size_t)j * n_pix + pix] = zv[j];
}

// Reset the run states of every instance before a solve.
__global__ void k_state_init(const Inst *__restrict__ tab, int ninst, double tol, int max_iter,
                             int ref) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst) return;
    DevState *ss[2] = {tab[i].st, tab[i].st_in};
    for (int s = 0; s < 2; ++s) {
        DevState *st = ss[s];
        st->rho[0] = 0.0; st->rho[1] = 0.0; st->rr = 0.0; st->rr0 = 0.0; st->bb = 0.0;
        st->thresh = 0.0; st->tol = tol; st->rel_true = 0.0; st->rr_prev = 0.0;
        st->iter = 0; st->max_iter = max_iter; st->status = SYLV_OK; st->done = 0;
        st->total_iter = 0; st->outer = 0; st->pend = -1; st->ref = ref;
    }
}

// Number of instances whose run (outer or inner) has not finished.
// Fold the nblocks partials of quantities slot0..slot0+NV-1 of one instance (one workgroup per
// instance, same fixed order as consume) into entry 0, for instances with Inst::pre set.
// count: 0 = float64 apply tiles, 1 = float32 apply tiles, 2 = streaming chunks.
template <int NV>
__global__ __launch_bounds__(kBlock) void k_prereduce(const Inst *__restrict__ tab, int slot0,
                                                      int count) {
    const Inst &I = tab[blockIdx.x];
    if (!I.pre) return;
    const int nb = count == 0 ? I.ntiles : count == 1 ? I.ntiles32 : I.nchunks;
    double v[NV];
    if (NV == 2 && slot0 == SLOT_RZ && I.pc == SYLV_PC_FOURIER) {
        // <r, z> from the Fourier column pass, ||r||^2 from its row pass
        double w[2];
        consume_pair(I.partial, I.nred, SLOT_FRZ, I.nfft, SLOT_RR, I.nrr, w);
        v[0] = w[0];
        v[NV - 1] = w[1];
    } else {
        consume<NV>(I.partial, I.nred, slot0, nb, v);   // every read precedes its final barrier
    }
    if (threadIdx.x == 0) {
        GAS double *pp = gp(I.partial);
#pragma unroll
        for (int i = 0; i < NV; ++i) pp[(size_t)(slot0 + i) * I.nred] = v[i];
    }
}

// Completion report for the host: out[0] = runs not finished; out[1] = the latest iteration
// tested among them; out[2] = max over them of log2(rr / thresh) in 1/256 units (how far the
// slowest run still is from its threshold, rounded up, 0 when unknown); out[3] the same for
// their starting residuals rr0, so that one report already gives a rate.  The host sizes the
// next batch of iterations from them.
__global__ void k_count_running(const Inst *__restrict__ tab, int ninst, int inner,
                                int *__restrict__ out) {
    __shared__ int cnt, last, gap, gap0;
    if (threadIdx.x == 0) { cnt = 0; last = 0; gap = 0; gap0 = 0; }
    __syncthreads();
    for (int i = threadIdx.x; i < ninst; i += blockDim.x) {
        const DevState *st = inner ? tab[i].st_in : tab[i].st;
        if (st->done) continue;
        atomicAdd(&cnt, 1);
        atomicMax(&last, st->iter);
        const double q = st->rr / st->thresh, q0 = st->rr0 / st->thresh;
        if (st->thresh > 0.0 && q > 1.0 && q < 1e300)
            atomicMax(&gap, (int)fmin(ceil(256.0 * log2(q)), 1e9));
        if (st->thresh > 0.0 && q0 > 1.0 && q0 < 1e300)
            atomicMax(&gap0, (int)fmin(ceil(256.0 * log2(q0)), 1e9));
    }
    __syncthreads();
    if (threadIdx.x == 0) { out[0] = cnt; out[1] = last; out[2] = gap; out[3] = gap0; }
}

// Host-to-device copy of a small table through the kernel arguments: the bytes travel with the
// launch itself, so the copy needs neither a host-side staging buffer that must outlive the call
// nor a synchronisation, and a captured graph keeps its own copy of them.
struct UploadChunk {
    uint32_t w[kUploadWords];
};
__global__ void k_upload(uint32_t *__restrict__ dst, int nwords, UploadChunk c) {
    for (int i = threadIdx.x; i < nwords; i += blockDim.x) dst[i] = c.w[i];
}

__global__ void k_stats(const Inst *__restrict__ tab, int ninst, sylv_pcg_stats *__restrict__ out,
                        int mixed) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst) return;
    const DevState *st = tab[i].st;
    const DevState *si = tab[i].st_in;
    sylv_pcg_stats s;
    s.status = st->status;
    if (st->status == SYLV_OK && !st->done) s.status = SYLV_NOT_CONVERGED;
    if (mixed) {
        s.iters = si->total_iter;
        s.outer = st->outer;
    } else {
        s.iters = st->total_iter;
        s.outer = st->outer;
    }
    s.relres_rec = (st->rr0 > 0.0) ? sqrt(st->rr / st->rr0) : 0.0;
    s.reserved = 0;
    s.relres_true = st->rel_true;
    out[i] = s;
}

// Perturbation for posterior sampling:
// eta_j = sqrt(tau_j) L_j xi_j + sum_f A[f,j] sqrt(W[f]) zeta_f, L_j = (kappa_j^2 + 4) - N4
// (L_j is symmetric, so L_j^T xi = L_j xi).
template <int K>
__global__ __launch_bounds__(kBlock) void k_po(const double *__restrict__ kappa,
                                               const double *__restrict__ tau,
                                               const double *__restrict__ A,
                                               const double *__restrict__ W,
                                               const double *__restrict__ xi,
                                               const double *__restrict__ zeta,
                                               double *__restrict__ eta, int f, int ny, int nx,
                                               int bc) {
    const int n_pix = ny * nx;
    const int pix = blockIdx.x * kBlock + threadIdx.x;
    if (pix >= n_pix) return;
    const int rhs = blockIdx.y;
    const double *xr = xi + (size_t)rhs * K * n_pix;
    const double *zr = zeta + (size_t)rhs * f * n_pix;
    double *er = eta + (size_t)rhs * K * n_pix;
    const int iy = pix / nx, ix = pix - iy * nx;
    const int n = wrapi(iy - 1, ny) * nx + ix, s = wrapi(iy + 1, ny) * nx + ix;
    const int w = iy * nx + wrapi(ix - 1, nx), e = iy * nx + wrapi(ix + 1, nx);
    // face grids: neighbours outside the face are absent and the diagonal counts the others
    const bool face = bc == SYLV_BC_FACE;
    const double hn = (!face || iy > 0) ? 1.0 : 0.0, hs = (!face || iy < ny - 1) ? 1.0 : 0.0;
    const double hw = (!face || ix > 0) ? 1.0 : 0.0, he = (!face || ix < nx - 1) ? 1.0 : 0.0;
    const double dg = face ? (hn + hs) + (hw + he) : 4.0;
    double acc[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const double *u = xr + (size_t)j * n_pix;
        const double kp = kappa[j], t = tau[j];
        const double lu = (kp * kp + dg) * u[pix] - ((hn * u[n] + hs * u[s]) + (hw * u[w] + he * u[e]));
        acc[j] = sqrt(t) * lu;
    }
    for (int fi = 0; fi < f; ++fi) {
        const double v = sqrt(W[(size_t)fi * n_pix + pix]) * zr[(size_t)fi * n_pix + pix];
#pragma unroll
        for (int j = 0; j < K; ++j) acc[j] += A[fi * K + j] * v;
    }
#pragma unroll
    for (int j = 0; j < K; ++j) er[(size_t)j * n_pix + pix] = acc[j];
}

// Gradient reductions of the adjoint (backward) pass: per-workgroup partials of
//   dtau_j = -<L lambda_j, L x*_j>, dkappa_j = -4 kappa_j tau_j <lambda_j, L x*_j>,
//   dA[f,j] = sum_p W[f,p] (r_f(p) lambda_j(p) - (a_f . lambda_p) x*_j(p)),
// and the pointwise dW = (a_f . lambda) r_f, dY = W (a_f . lambda), r_f = Y_f - a_f . x*.
// One pixel per thread; L x*_j and L lambda_j come from 5-point stencils on the fly.
template <int K>
__global__ __launch_bounds__(kBlock) void k_grad(const double *__restrict__ coef,
                                                 const double *__restrict__ A,
                                                 const double *__restrict__ W,
                                                 const double *__restrict__ Y,
                                                 const double *__restrict__ X,
                                                 const double *__restrict__ Lm, int f, int ny,
                                                 int nx, int bc, double *__restrict__ dW,
                                                 double *__restrict__ dY,
                                                 double *__restrict__ partial) {
    const int n_pix = ny * nx;
    const int nblk = gridDim.x;
    const int nv = 2 * K + f * K;
    __shared__ double sm[2 * kMaxK + kMaxF * kMaxK][kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int pix = blockIdx.x * kBlock + threadIdx.x;
    const bool active = pix < n_pix;
    double xs[K], lm[K], tx[K], tl[K];
#pragma unroll
    for (int j = 0; j < K; ++j) { xs[j] = lm[j] = tx[j] = tl[j] = 0.0; }
    if (active) {
        const int iy = pix / nx, ix = pix - iy * nx;
        const int n = wrapi(iy - 1, ny) * nx + ix, s = wrapi(iy + 1, ny) * nx + ix;
        const int w = iy * nx + wrapi(ix - 1, nx), e = iy * nx + wrapi(ix + 1, nx);
        // face grids: neighbours outside the face are absent and the diagonal counts the others
        const bool face = bc == SYLV_BC_FACE;
        const double hn = (!face || iy > 0) ? 1.0 : 0.0, hs = (!face || iy < ny - 1) ? 1.0 : 0.0;
        const double hw = (!face || ix > 0) ? 1.0 : 0.0, he = (!face || ix < nx - 1) ? 1.0 : 0.0;
        const double dg = face ? (hn + hs) + (hw + he) : 4.0;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const double kp = coef[j * kCoefStride + 5];
            const double d = kp * kp + dg;
            const double *u = X + (size_t)j * n_pix;
            const double *v = Lm + (size_t)j * n_pix;
            xs[j] = u[pix];
            lm[j] = v[pix];
            tx[j] = d * xs[j] - ((hn * u[n] + hs * u[s]) + (hw * u[w] + he * u[e]));
            tl[j] = d * lm[j] - ((hn * v[n] + hs * v[s]) + (hw * v[w] + he * v[e]));
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const double kp = coef[j * kCoefStride + 5], t = coef[j * kCoefStride + 6];
        const double a = wave_sum(-tl[j] * tx[j]);
        const double b = wave_sum(-4.0 * kp * t * lm[j] * tx[j]);
        if (lane == 0) { sm[j][wid] = a; sm[K + j][wid] = b; }
    }
    for (int fi = 0; fi < f; ++fi) {
        double a[K];
#pragma unroll
        for (int j = 0; j < K; ++j) a[j] = A[fi * K + j];
        double al = 0.0, ax = 0.0;
#pragma unroll
        for (int j = 0; j < K; ++j) { al += a[j] * lm[j]; ax += a[j] * xs[j]; }
        double wv = 0.0, yv = 0.0;
        if (active) {
            wv = W[(size_t)fi * n_pix + pix];
            yv = Y[(size_t)fi * n_pix + pix];
        }
        const double rf = yv - ax;
        if (active) {
            if (dW) dW[(size_t)fi * n_pix + pix] = al * rf;
            if (dY) dY[(size_t)fi * n_pix + pix] = wv * al;
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const double g = wave_sum(wv * (rf * lm[j] - al * xs[j]));
            if (lane == 0) sm[2 * K + fi * K + j][wid] = g;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nv; i += kBlock)
        partial[(size_t)i * nblk + blockIdx.x] = (sm[i][0] + sm[i][1]) + (sm[i][2] + sm[i][3]);
}

// Sum the gradient partials (one thread per quantity, fixed order over workgroups).
__global__ void k_grad_fin(const double *__restrict__ partial, int nv, int nblk, int k,
                           double *__restrict__ dkappa, double *__restrict__ dtau,
                           double *__restrict__ dA) {
    for (int i = threadIdx.x; i < nv; i += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += partial[(size_t)i * nblk + b];
        if (i < k) {
            if (dtau) dtau[i] = s;
        } else if (i < 2 * k) {
            if (dkappa) dkappa[i - k] = s;
        } else {
            if (dA) dA[i - 2 * k] = s;
        }
    }
}

// Face grids always run with 2 rows per lane (the host sizes their tiles accordingly).  Only the
// row counts that apply_rows_for can return for (T, K) are instantiated.
template <typename T, int K, int MODE, int CP>
hipError_t launch_apply_rows_cp(int rows, int bc, dim3 grid, hipStream_t s, const Inst *table,
                                const int *tprefix, int ninst, int it, const void *in, void *out) {
    constexpr int cap = apply_rows_cap(sizeof(T) == 8, K);
    const T *i = reinterpret_cast<const T *>(in);
    T *o = reinterpret_cast<T *>(out);
    const int nb = (int)grid.x;
    if (bc == SYLV_BC_FACE) {
        hipLaunchKernelGGL((k_apply<T, K, 2, MODE, BC_FACE, CP>), grid, dim3(kBlock), 0, s, table,
                           tprefix, ninst, nb, it, i, o);
        return hipGetLastError();
    }
    if constexpr (cap >= 8) {
        if (rows == 8) {
            hipLaunchKernelGGL((k_apply<T, K, 8, MODE, BC_PERIODIC, CP>), grid, dim3(kBlock), 0, s,
                               table, tprefix, ninst, nb, it, i, o);
            return hipGetLastError();
        }
    }
    if constexpr (cap >= 4) {
        if (rows == 4) {
            hipLaunchKernelGGL((k_apply<T, K, 4, MODE, BC_PERIODIC, CP>), grid, dim3(kBlock), 0, s,
                               table, tprefix, ninst, nb, it, i, o);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_apply<T, K, 2, MODE, BC_PERIODIC, CP>), grid, dim3(kBlock), 0, s, table,
                       tprefix, ninst, nb, it, i, o);
    return hipGetLastError();
}

// Streaming policy of each precision (measured on 2048^2 grids): float64 applies gain most from
// non-temporal loads of the once-read planes, float32 applies and updates from non-temporal
// stores; both at once, or either inside the last-level cache, is slower.  The float64 update
// keeps the default policy: it reads q right after the apply wrote it, and streaming its loads
// slowed whole float64 solves (batched grids +6 %).
template <typename T>
constexpr int stream_cp() { return sizeof(T) == 8 ? 1 : 2; }

template <typename T, int K, int MODE>
hipError_t launch_apply_rows(int rows, int bc, int stream, dim3 grid, hipStream_t s,
                             const Inst *table, const int *tprefix, int ninst, int it,
                             const void *in, void *out) {
    if (stream)
        return launch_apply_rows_cp<T, K, MODE, stream_cp<T>()>(rows, bc, grid, s, table, tprefix,
                                                                ninst, it, in, out);
    return launch_apply_rows_cp<T, K, MODE, 0>(rows, bc, grid, s, table, tprefix, ninst, it, in,
                                               out);
}

}  // namespace

// ---- launchers -------------------------------------------------------------------------------

int apply_rows_valid(int rows) { return rows == 2 || rows == 4 || rows == 8; }

int apply_rows_for(int k, int dtype, int request) {
    // default: 4 rows where the register window leaves >= 2 waves per SIMD, else 2
    int rows = request;
    if (!apply_rows_valid(rows)) rows = (dtype == SYLV_F64) ? (k <= 3 ? 4 : 2) : (k <= 4 ? 4 : 2);
    const int cap = apply_rows_cap(dtype == SYLV_F64, k);
    return rows < cap ? rows : cap;
}

int grad_blocks(int n_pix) { return (int)blocks_for(n_pix, kBlock); }
int grad_nv(int k, int f) { return 2 * k + f * k; }

hipError_t launch_coef(const double *kappa, const double *tau, int k, int ny, int nx,
                       double *coef, hipStream_t s) {
    hipLaunchKernelGGL(k_coef, dim3(1), dim3(64), 0, s, kappa, tau, k, ny, nx, coef);
    return hipGetLastError();
}

hipError_t launch_setup(const double *W, const double *A, int f, int ny, int nx, int bc,
                        const double *coef, int pc, double *M64, float *M32, double *P64,
                        float *P32, unsigned short *P16, int exact, int k, hipStream_t s) {
    const long n_pix = (long)ny * nx;
    return dispatch_k(k, [&](auto tag) {
        constexpr int K = decltype(tag)::value;
        hipLaunchKernelGGL((k_setup<K>), dim3(blocks_for(n_pix, kBlock)), dim3(kBlock), 0, s, W,
                           A, f, ny, nx, bc, coef, pc, M64, M32, P64, P32, P16, exact);
        return hipGetLastError();
    });
}

hipError_t launch_rhs(const double *W, const double *Y, const double *A, int f, int n_pix,
                      const double *bext, double *b, int k, hipStream_t s) {
    return dispatch_k(k, [&](auto tag) {
        constexpr int K = decltype(tag)::value;
        hipLaunchKernelGGL((k_rhs<K>), dim3(blocks_for(n_pix, kBlock)), dim3(kBlock), 0, s, W,
                           Y, A, f, n_pix, bext, b);
        return hipGetLastError();
    });
}

hipError_t launch_apply_plain(const Inst *table0, int k, int dtype, int rows, int bc, int stream,
                              int ny, int nx, int nrhs, const void *in, void *out, hipStream_t s) {
    if (bc == SYLV_BC_FACE) rows = 2;
    const unsigned tx = blocks_for(nx, kTileX);
    const unsigned ty = blocks_for(ny, kWavesY * rows);
    const dim3 grid(tx * ty, nrhs);
    return dispatch_k(k, [&](auto tag) {
        constexpr int K = decltype(tag)::value;
        if (dtype == SYLV_F64)
            return launch_apply_rows<double, K, AM_PLAIN>(rows, bc, stream, grid, s, table0,
                                                          nullptr, 1, 0, in, out);
        return launch_apply_rows<float, K, AM_PLAIN>(rows, bc, stream, grid, s, table0, nullptr,
                                                     1, 0, in, out);
    });
}

hipError_t launch_precond_plain(const Inst *table0, int k, int dtype, int n_pix, int nrhs,
                                const void *in, void *out, hipStream_t s) {
    const dim3 grid(blocks_for(n_pix, kBlock), nrhs);
    return dispatch_k(k, [&](auto tag) {
        constexpr int K = decltype(tag)::value;
        if (dtype == SYLV_F64)
            hipLaunchKernelGGL((k_precond_plain<double, K>), grid, dim3(kBlock), 0, s, table0,
                               reinterpret_cast<const double *>(in),
                               reinterpret_cast<double *>(out));
        else
            hipLaunchKernelGGL((k_precond_plain<float, K>), grid, dim3(kBlock), 0, s, table0,
                               reinterpret_cast<const float *>(in),
                               reinterpret_cast<float *>(out));
        return hipGetLastError();
    });
}

hipError_t launch_resid(const InstSet &set, int k, int phase, hipStream_t s) {
    return dispatch_k(k, [&](auto tag) {
        constexpr int K = decltype(tag)::value;
        return launch_apply_rows<double, K, AM_RESID>(set.rows64, set.bc, set.stream,
                                                      dim3(set.total_tiles), s, set.table,
                                                      set.tprefix, set.ninst, phase, nullptr,
                                                      nullptr);
    });
}

hipError_t launch_resid_fin(const InstSet &set, int phase, hipStream_t s) {
    hipLaunchKernelGGL(k_resid_fin, dim3(set.ninst), dim3(kBlock), 0, s, set.table, phase);
    return hipGetLastError();
}

hipError_t launch_cg_apply(const InstSet &set, int k, int mixed, int it, hipStream_t s) {
    return dispatch_k(k, [&](auto tag) {
        constexpr int K = decltype(tag)::value;
        if (mixed)
            return launch_apply_rows<float, K, AM_CG>(set.rows32, set.bc, set.stream,
                                                      dim3(set.total_tiles32), s, set.table,
                                                      set.tprefix32, set.ninst, it, nullptr,
                                                      nullptr);
        return launch_apply_rows<double, K, AM_CG>(set.rows64, set.bc, set.stream,
                                                   dim3(set.total_tiles), s, set.table,
                                                   set.tprefix, set.ninst, it, nullptr, nullptr);
    });
}

hipError_t launch_cg_update(const InstSet &set, int k, int mixed, int it, hipStream_t s) {
    return dispatch_k(k, [&](auto tag) {
        constexpr int K = decltype(tag)::value;
        const dim3 grid(set.total_chunks);
        if (mixed && set.stream)
            hipLaunchKernelGGL((k_update<float, K, stream_cp<float>()>), grid, dim3(kBlock), 0, s,
                               set.table, set.cprefix, set.ninst, (int)grid.x, it);
        else if (mixed)
            hipLaunchKernelGGL((k_update<float, K, 0>), grid, dim3(kBlock), 0, s, set.table,
                               set.cprefix, set.ninst, (int)grid.x, it);
        else
            hipLaunchKernelGGL((k_update<double, K, 0>), grid, dim3(kBlock), 0, s, set.table,
                               set.cprefix, set.ninst, (int)grid.x, it);
        return hipGetLastError();
    });
}

hipError_t launch_pinit(const InstSet &set, int k, int mixed, double inner_tol, double safety,
                        int max_iter, hipStream_t s) {
    return dispatch_k(k, [&](auto tag) {
        constexpr int K = decltype(tag)::value;
        const dim3 grid(set.total_chunks);
        if (mixed)
            hipLaunchKernelGGL((k_pinit<float, K>), grid, dim3(kBlock), 0, s, set.table,
                               set.cprefix, set.ninst, (int)grid.x, inner_tol, safety, max_iter);
        else
            hipLaunchKernelGGL((k_pinit<double, K>), grid, dim3(kBlock), 0, s, set.table,
                               set.cprefix, set.ninst, (int)grid.x, inner_tol, safety, max_iter);
        return hipGetLastError();
    });
}

hipError_t launch_refine_axpy(const InstSet &set, int k, hipStream_t s) {
    return dispatch_k(k, [&](auto tag) {
        constexpr int K = decltype(tag)::value;
        const dim3 grid(set.total_chunks);
        hipLaunchKernelGGL((k_refine_axpy<K>), grid, dim3(kBlock), 0, s, set.table, set.cprefix,
                           set.ninst, (int)grid.x);
        return hipGetLastError();
    });
}

hipError_t launch_state_init(const InstSet &set, double tol, int max_iter, int ref,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_state_init, dim3(blocks_for(set.ninst, 64)), dim3(64), 0, s, set.table,
                       set.ninst, tol, max_iter, ref);
    return hipGetLastError();
}

hipError_t launch_upload(void *dst, const void *src, size_t bytes, hipStream_t s) {
    if (bytes % 4 != 0 || ((uintptr_t)dst & 3u) != 0) return hipErrorInvalidValue;
    const size_t words = bytes / 4;
    const uint32_t *w = static_cast<const uint32_t *>(src);
    for (size_t off = 0; off < words; off += kUploadWords) {
        const int n = (int)std::min<size_t>(kUploadWords, words - off);
        UploadChunk c;
        memcpy(c.w, w + off, sizeof(uint32_t) * n);
        for (int i = n; i < kUploadWords; ++i) c.w[i] = 0u;
        hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, s,
                           static_cast<uint32_t *>(dst) + off, n, c);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_count_running(const InstSet &set, int inner, int *out, hipStream_t s) {
    hipLaunchKernelGGL(k_count_running, dim3(1), dim3(256), 0, s, set.table, set.ninst, inner,
                       out);
    return hipGetLastError();
}

hipError_t launch_prereduce_pq(const InstSet &set, int mixed, hipStream_t s) {
    if (!set.any_pre) return hipSuccess;
    hipLaunchKernelGGL(k_prereduce<1>, dim3(set.ninst), dim3(kBlock), 0, s, set.table,
                       (int)SLOT_PQ, mixed ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_prereduce_rz(const InstSet &set, hipStream_t s) {
    if (!set.any_pre) return hipSuccess;
    hipLaunchKernelGGL(k_prereduce<2>, dim3(set.ninst), dim3(kBlock), 0, s, set.table,
                       (int)SLOT_RZ, 2);
    return hipGetLastError();
}

hipError_t launch_stats(const InstSet &set, void *stats, int mixed, hipStream_t s) {
    hipLaunchKernelGGL(k_stats, dim3(blocks_for(set.ninst, 64)), dim3(64), 0, s, set.table,
                       set.ninst, reinterpret_cast<sylv_pcg_stats *>(stats), mixed);
    return hipGetLastError();
}

hipError_t launch_po(const double *kappa, const double *tau, const double *A, const double *W,
                     const double *xi, const double *zeta, double *eta, int k, int f, int ny,
                     int nx, int bc, int nrhs, hipStream_t s) {
    return dispatch_k(k, [&](auto tag) {
        constexpr int K = decltype(tag)::value;
        const dim3 grid(blocks_for((long)ny * nx, kBlock), nrhs);
        hipLaunchKernelGGL((k_po<K>), grid, dim3(kBlock), 0, s, kappa, tau, A, W, xi, zeta, eta,
                           f, ny, nx, bc);
        return hipGetLastError();
    });
}

hipError_t launch_grad(const double *coef, const double *A, const double *W, const double *Y,
                       const double *X, const double *Lm, int k, int f, int ny, int nx, int bc,
                       double *dkappa, double *dtau, double *dA, double *dW, double *dY,
                       double *partial, hipStream_t s) {
    const int nblk = grad_blocks(ny * nx);
    hipError_t e = dispatch_k(k, [&](auto tag) {
        constexpr int K = decltype(tag)::value;
        hipLaunchKernelGGL((k_grad<K>), dim3(nblk), dim3(kBlock), 0, s, coef, A, W, Y, X, Lm, f,
                           ny, nx, bc, dW, dY, partial);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_grad_fin, dim3(1), dim3(kBlock), 0, s, partial, grad_nv(k, f), nblk, k,
                       dkappa, dtau, dA);
    return hipGetLastError();
}

}  // namespace sylv
