// Device helpers shared by the kernel translation units of libsylv (not part of the ABI).
#pragma once

#include "sylv_internal.h"
#include "sylv.h"

#include <math.h>

#define GAS __attribute__((address_space(1)))

namespace sylv {
namespace dev {

constexpr int kXcd = 8;

template <typename T>
__device__ __forceinline__ GAS T *gp(T *p) { return (GAS T *)p; }
template <typename T>
__device__ __forceinline__ const GAS T *gp(const T *p) { return (const GAS T *)p; }

__device__ __forceinline__ int wrapi(int v, int n) {
    while (v < 0) v += n;
    while (v >= n) v -= n;
    return v;
}

// Grid boundary of the pixel graph (template parameter of the stencil kernels).
enum { BC_PERIODIC = SYLV_BC_PERIODIC, BC_FACE = SYLV_BC_FACE };

// Number of 4-neighbours of pixel (ix, iy) inside an nx x ny face (the minus diagonal of D).
__device__ __forceinline__ int face_deg(int ix, int iy, int nx, int ny) {
    return (ix > 0) + (ix < nx - 1) + (iy > 0) + (iy < ny - 1);
}

// Give XCD x (which receives workgroups x, x+8, x+16, ...) a contiguous range of logical ids.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int q = nb / kXcd, rem = nb % kXcd;
    const int x = b % kXcd, slot = b / kXcd;
    return x * q + min(x, rem) + slot;
}

__device__ __forceinline__ int find_inst(const int *__restrict__ prefix, int ninst, int L) {
    int lo = 0, hi = ninst;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= L) lo = mid; else hi = mid;
    }
    return lo;
}

template <int K>
__host__ __device__ constexpr int pidx(int i, int j) {
    return (i <= j) ? (i * K - (i * (i - 1)) / 2 + (j - i)) : (j * K - (j * (j - 1)) / 2 + (i - j));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-reduce NV values (fixed order) and store this workgroup's partial of quantity i at
// partial[(slot0 + i) * nred + blk].
template <int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], double *partial, int nred,
                                               int slot0, int blk) {
    __shared__ double sm[NV][kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) sm[i][wid] = v[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        GAS double *pp = gp(partial);
#pragma unroll
        for (int i = 0; i < NV; ++i)
            pp[(size_t)(slot0 + i) * nred + blk] = (sm[i][0] + sm[i][1]) + (sm[i][2] + sm[i][3]);
    }
}

// Fixed-order sum over nblocks partials of quantities slot0..slot0+NV-1; every thread of the
// workgroup receives the result.
template <int NV>
__device__ __forceinline__ void consume(const double *partial, int nred, int slot0, int nblocks,
                                        double (&out)[NV]) {
    __shared__ double sm[NV][kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const GAS double *pp = gp(partial);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += kBlock) s += pp[(size_t)(slot0 + i) * nred + b];
        s = wave_sum(s);
        if (lane == 0) sm[i][wid] = s;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) out[i] = (sm[i][0] + sm[i][1]) + (sm[i][2] + sm[i][3]);
}

__device__ __forceinline__ bool finite_d(double v) { return isfinite(v); }

// ---- vector access helpers (clang vector types: usable in the global address space) --------
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void ld4(const GAS double *p, double (&v)[4]) {
    const dvec2 a = reinterpret_cast<const GAS dvec2 *>(p)[0];
    const dvec2 b = reinterpret_cast<const GAS dvec2 *>(p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ __forceinline__ void ld4(const GAS float *p, float (&v)[4]) {
    const fvec4 a = reinterpret_cast<const GAS fvec4 *>(p)[0];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}
__device__ __forceinline__ void st4(GAS double *p, const double (&v)[4]) {
    dvec2 a, b;
    a.x = v[0]; a.y = v[1]; b.x = v[2]; b.y = v[3];
    reinterpret_cast<GAS dvec2 *>(p)[0] = a;
    reinterpret_cast<GAS dvec2 *>(p)[1] = b;
}
__device__ __forceinline__ void st4(GAS float *p, const float (&v)[4]) {
    fvec4 a;
    a.x = v[0]; a.y = v[1]; a.z = v[2]; a.w = v[3];
    reinterpret_cast<GAS fvec4 *>(p)[0] = a;
}

// bfloat16 planes (the preconditioner factor of CG runs): the top 16 bits of a float32.
typedef unsigned short hvec4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float bf16_value(unsigned short h) {
    return __uint_as_float((unsigned)h << 16);
}
// float32 -> bfloat16, rounding to nearest with ties to even; NaN stays NaN.
__device__ __forceinline__ unsigned short bf16_round(float v) {
    const unsigned u = __float_as_uint(v);
    if (v != v) return (unsigned short)((u >> 16) | 0x40u);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ void ld4(const GAS unsigned short *p, float (&v)[4]) {
    const hvec4 a = reinterpret_cast<const GAS hvec4 *>(p)[0];
    v[0] = bf16_value(a.x); v[1] = bf16_value(a.y); v[2] = bf16_value(a.z); v[3] = bf16_value(a.w);
}

// Field selectors by precision (all return global-address-space pointers).
template <typename T> struct Sel;
template <> struct Sel<double> {
    static __device__ __forceinline__ const GAS double *M(const Inst &I) { return gp(I.M64); }
    static __device__ __forceinline__ const GAS double *P(const Inst &I) { return gp(I.P64); }
    static __device__ __forceinline__ GAS double *x(const Inst &I) { return gp(I.x); }
    static __device__ __forceinline__ GAS double *r(const Inst &I) { return gp(I.r); }
    static __device__ __forceinline__ GAS double *z(const Inst &I) { return gp(I.z); }
    static __device__ __forceinline__ GAS double *p(const Inst &I, int i) { return gp(I.p[i & 1]); }
    static __device__ __forceinline__ GAS double *q(const Inst &I) { return gp(I.q); }
    static __device__ __forceinline__ DevState *st(const Inst &I) { return I.st; }
};

// Preconditioner of CG runs (both precisions): the block inverse as Pinv = G^T G with
// G = L^-1 (L the Cholesky factor of the diagonal block), G stored in bfloat16.  A
// preconditioner only has to be fixed and positive definite; G^T G stays so whatever the
// rounding of G's entries (its diagonal stays positive), so the solve converges to the same
// solution while reading a quarter of the bytes of float64 blocks.
__device__ __forceinline__ const GAS unsigned short *Pcg(const Inst &I) { return gp(I.P16); }
template <> struct Sel<float> {
    static __device__ __forceinline__ const GAS float *M(const Inst &I) { return gp(I.M32); }
    static __device__ __forceinline__ const GAS float *P(const Inst &I) { return gp(I.P32); }
    static __device__ __forceinline__ GAS float *x(const Inst &I) { return gp(I.d32); }
    static __device__ __forceinline__ GAS float *r(const Inst &I) { return gp(I.r32); }
    static __device__ __forceinline__ GAS float *z(const Inst &I) { return gp(I.z32); }
    static __device__ __forceinline__ GAS float *p(const Inst &I, int i) { return gp(I.p32[i & 1]); }
    static __device__ __forceinline__ GAS float *q(const Inst &I) { return gp(I.q32); }
    static __device__ __forceinline__ DevState *st(const Inst &I) { return I.st_in; }
};

// z = Pinv r at one pixel for the three preconditioner kinds; P planes (element type PT) are
// read at `pix` and the product is formed in T.
template <typename T, int K, typename PT>
__device__ __forceinline__ void precond_pixel(int pc, const GAS PT *P, int n_pix, int pix,
                                              const T (&r)[K], T (&z)[K]) {
    if (pc == SYLV_PC_BLOCK) {
        constexpr int MK = K * (K + 1) / 2;
        T pm[MK];
#pragma unroll
        for (int e = 0; e < MK; ++e) pm[e] = (T)P[(size_t)e * n_pix + pix];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            T s = 0;
#pragma unroll
            for (int i = 0; i < K; ++i) s += pm[pidx<K>(j, i)] * r[i];
            z[j] = s;
        }
    } else if (pc == SYLV_PC_JACOBI) {
#pragma unroll
        for (int j = 0; j < K; ++j) z[j] = (T)P[(size_t)j * n_pix + pix] * r[j];
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j) z[j] = r[j];
    }
}

// z = G^T (G r) at one pixel from the bfloat16 factor planes (block kind: G[a][c], a >= c, at
// plane pidx(c, a); Jacobi kind: one plane per component holding 1 / diagonal).
template <typename T, int K>
__device__ __forceinline__ void precond_cg_pixel(int pc, const GAS unsigned short *F, int n_pix,
                                                 int pix, const T (&r)[K], T (&z)[K]) {
    if (pc == SYLV_PC_BLOCK) {
        constexpr int MK = K * (K + 1) / 2;
        T g[MK];
#pragma unroll
        for (int e = 0; e < MK; ++e) g[e] = (T)bf16_value(F[(size_t)e * n_pix + pix]);
        T t[K];
#pragma unroll
        for (int a = 0; a < K; ++a) {
            T s = 0;
#pragma unroll
            for (int c = 0; c <= a; ++c) s += g[pidx<K>(c, a)] * r[c];
            t[a] = s;
        }
#pragma unroll
        for (int c = 0; c < K; ++c) {
            T s = 0;
#pragma unroll
            for (int a = c; a < K; ++a) s += g[pidx<K>(c, a)] * t[a];
            z[c] = s;
        }
    } else if (pc == SYLV_PC_JACOBI) {
#pragma unroll
        for (int j = 0; j < K; ++j) z[j] = (T)bf16_value(F[(size_t)j * n_pix + pix]) * r[j];
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j) z[j] = r[j];
    }
}

template <typename T, int K>
__device__ __forceinline__ void precond_cg_vec4(int pc, const GAS unsigned short *F, int n_pix,
                                                int p0, const T (&r)[K][4], T (&z)[K][4]) {
    if (pc == SYLV_PC_BLOCK) {
        constexpr int MK = K * (K + 1) / 2;
        T g[MK][4];
#pragma unroll
        for (int e = 0; e < MK; ++e) {
            float tmp[4];
            ld4(F + (size_t)e * n_pix + p0, tmp);
#pragma unroll
            for (int q = 0; q < 4; ++q) g[e][q] = (T)tmp[q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            T t[K];
#pragma unroll
            for (int a = 0; a < K; ++a) {
                T s = 0;
#pragma unroll
                for (int c = 0; c <= a; ++c) s += g[pidx<K>(c, a)][q] * r[c][q];
                t[a] = s;
            }
#pragma unroll
            for (int c = 0; c < K; ++c) {
                T s = 0;
#pragma unroll
                for (int a = c; a < K; ++a) s += g[pidx<K>(c, a)][q] * t[a];
                z[c][q] = s;
            }
        }
    } else if (pc == SYLV_PC_JACOBI) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            float d[4];
            ld4(F + (size_t)j * n_pix + p0, d);
#pragma unroll
            for (int q = 0; q < 4; ++q) z[j][q] = (T)d[q] * r[j][q];
        }
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) z[j][q] = r[j][q];
    }
}

template <int K>
struct KTag {
    static constexpr int value = K;
};

template <typename F>
hipError_t dispatch_k(int k, F &&fn) {
    switch (k) {
        case 1: return fn(KTag<1>{});
        case 2: return fn(KTag<2>{});
        case 3: return fn(KTag<3>{});
        case 4: return fn(KTag<4>{});
        case 5: return fn(KTag<5>{});
        case 6: return fn(KTag<6>{});
        case 7: return fn(KTag<7>{});
        case 8: return fn(KTag<8>{});
        default: return hipErrorInvalidValue;
    }
}

inline unsigned blocks_for(long n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace dev
}  // namespace sylv
