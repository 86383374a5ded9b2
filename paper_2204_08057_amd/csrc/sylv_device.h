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

// Periodic wrap of v into [0, n) for the stencil kernels, whose indices lie at most 66 outside:
// one conditional step on grids of 128 or more, the loop on smaller ones (a uniform branch).
__device__ __forceinline__ int wrapf(int v, int n) {
    if (n >= 128) {
        v += (v < 0) ? n : 0;
        v -= (v >= n) ? n : 0;
        return v;
    }
    return wrapi(v, n);
}

// Plane access through buffer resources.  A plane (n elements of T at a base that is the same
// for the whole wavefront: callers build plane pointers from workgroup-uniform values only) is
// described by a resource held in scalar registers; each access gives a 32-bit byte offset per
// lane, so no 64-bit address arithmetic is spent per access, and the hardware range check
// returns 0 for a load (drops a store) outside [0, n).  Every problem has fewer than 2^29
// pixels, so n * sizeof(T) < 2^32.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
constexpr int kRsrcWord3 = 0x00020000;   // raw buffer, 32-bit data format (gfx9 family)
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const GAS T *plane, uint32_t n) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)uniform_u64((uint64_t)plane), 0,
                                             (int)(n * (uint32_t)sizeof(T)), kRsrcWord3);
}
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
// Vector elements are read by value (a.x) and converted with __uint_as_float / join_f64: this
// compiler mis-reads __builtin_bit_cast of a vector element expression (it reads element 0).
// float64 from / to its two 32-bit halves (low word first in memory)
__device__ __forceinline__ double join_f64(unsigned lo, unsigned hi) {
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ unsigned lo_f64(double v) {
    return (unsigned)__builtin_bit_cast(unsigned long long, v);
}
__device__ __forceinline__ unsigned hi_f64(double v) {
    return (unsigned)(__builtin_bit_cast(unsigned long long, v) >> 32);
}

// AUX: the cache-policy bits of the buffer instruction; kNT (the non-temporal bit) streams data
// that the kernel touches once past the caches (see k_apply / k_update).
constexpr int kNT = 2;
template <int AUX = 0>
__device__ __forceinline__ float bld(const GAS float *plane, uint32_t n, uint32_t i) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(plane_rsrc(plane, n), i * 4u, 0, AUX));
}
template <int AUX = 0>
__device__ __forceinline__ double bld(const GAS double *plane, uint32_t n, uint32_t i) {
    const u32x2 a = __builtin_amdgcn_raw_buffer_load_b64(plane_rsrc(plane, n), i * 8u, 0, AUX);
    return join_f64(a.x, a.y);
}
template <int AUX = 0>
__device__ __forceinline__ void bst(GAS float *plane, uint32_t n, uint32_t i, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), plane_rsrc((const GAS float *)plane, n), i * 4u, 0, AUX);
}
template <int AUX = 0>
__device__ __forceinline__ void bst(GAS double *plane, uint32_t n, uint32_t i, double v) {
    const u32x2 a = {lo_f64(v), hi_f64(v)};
    __builtin_amdgcn_raw_buffer_store_b64(a, plane_rsrc((const GAS double *)plane, n), i * 8u, 0, AUX);
}
// four consecutive elements starting at i (i % 4 == 0, planes 16-byte aligned)
template <int AUX = 0>
__device__ __forceinline__ void bld4(const GAS float *plane, uint32_t n, uint32_t i, float (&v)[4]) {
    const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(plane_rsrc(plane, n), i * 4u, 0, AUX);
    v[0] = __uint_as_float(a.x); v[1] = __uint_as_float(a.y);
    v[2] = __uint_as_float(a.z); v[3] = __uint_as_float(a.w);
}
template <int AUX = 0>
__device__ __forceinline__ void bld4(const GAS double *plane, uint32_t n, uint32_t i, double (&v)[4]) {
    const __amdgpu_buffer_rsrc_t r = plane_rsrc(plane, n);
    const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, i * 8u, 0, AUX);
    const u32x4 b = __builtin_amdgcn_raw_buffer_load_b128(r, i * 8u + 16u, 0, AUX);
    v[0] = join_f64(a.x, a.y); v[1] = join_f64(a.z, a.w);
    v[2] = join_f64(b.x, b.y); v[3] = join_f64(b.z, b.w);
}
template <int AUX = 0>
__device__ __forceinline__ void bld4(const GAS unsigned short *plane, uint32_t n, uint32_t i,
                                     float (&v)[4]) {
    const u32x2 a = __builtin_amdgcn_raw_buffer_load_b64(plane_rsrc(plane, n), i * 2u, 0, AUX);
    v[0] = __uint_as_float(a.x << 16); v[1] = __uint_as_float(a.x & 0xffff0000u);
    v[2] = __uint_as_float(a.y << 16); v[3] = __uint_as_float(a.y & 0xffff0000u);
}
template <int AUX = 0>
__device__ __forceinline__ void bst4(GAS float *plane, uint32_t n, uint32_t i, const float (&v)[4]) {
    const u32x4 a = {__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]),
                     __float_as_uint(v[3])};
    __builtin_amdgcn_raw_buffer_store_b128(a, plane_rsrc((const GAS float *)plane, n), i * 4u, 0, AUX);
}
template <int AUX = 0>
__device__ __forceinline__ void bst4(GAS double *plane, uint32_t n, uint32_t i, const double (&v)[4]) {
    const __amdgpu_buffer_rsrc_t r = plane_rsrc((const GAS double *)plane, n);
    const u32x4 a = {lo_f64(v[0]), hi_f64(v[0]), lo_f64(v[1]), hi_f64(v[1])};
    const u32x4 b = {lo_f64(v[2]), hi_f64(v[2]), lo_f64(v[3]), hi_f64(v[3])};
    __builtin_amdgcn_raw_buffer_store_b128(a, r, i * 8u, 0, AUX);
    __builtin_amdgcn_raw_buffer_store_b128(b, r, i * 8u + 16u, 0, AUX);
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
// workgroup receives the result.  Each thread keeps four independent running sums so that four
// loads are in flight at a time (the partials are read from L2 with its full latency).
template <int NV>
__device__ __forceinline__ void consume(const double *partial, int nred, int slot0, int nblocks,
                                        double (&out)[NV]) {
    __shared__ double sm[NV][kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const GAS double *pp = gp(partial) + (size_t)(slot0 + i) * nred;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int b = threadIdx.x;
        for (; b + 3 * kBlock < nblocks; b += 4 * kBlock) {
            a0 += pp[b];
            a1 += pp[b + kBlock];
            a2 += pp[b + 2 * kBlock];
            a3 += pp[b + 3 * kBlock];
        }
        for (; b < nblocks; b += kBlock) a0 += pp[b];
        double s = (a0 + a1) + (a2 + a3);
        s = wave_sum(s);
        if (lane == 0) sm[i][wid] = s;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) out[i] = (sm[i][0] + sm[i][1]) + (sm[i][2] + sm[i][3]);
}

// Two reduced quantities with different producers: slot a over na workgroup partials and slot b
// over nb (one shared table and one barrier, like consume<2>).
__device__ __forceinline__ void consume_pair(const double *partial, int nred, int slot_a, int na,
                                             int slot_b, int nb, double (&out)[2]) {
    __shared__ double sm[2][kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const GAS double *pp = gp(partial) + (size_t)(i ? slot_b : slot_a) * nred;
        const int nblocks = i ? nb : na;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int b = threadIdx.x;
        for (; b + 3 * kBlock < nblocks; b += 4 * kBlock) {
            a0 += pp[b];
            a1 += pp[b + kBlock];
            a2 += pp[b + 2 * kBlock];
            a3 += pp[b + 3 * kBlock];
        }
        for (; b < nblocks; b += kBlock) a0 += pp[b];
        double s = (a0 + a1) + (a2 + a3);
        s = wave_sum(s);
        if (lane == 0) sm[i][wid] = s;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i) out[i] = (sm[i][0] + sm[i][1]) + (sm[i][2] + sm[i][3]);
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

template <typename T, int K, int AUX = 0>
__device__ __forceinline__ void precond_cg_vec4(int pc, const GAS unsigned short *F, int n_pix,
                                                int p0, const T (&r)[K][4], T (&z)[K][4]) {
    if (pc == SYLV_PC_BLOCK) {
        constexpr int MK = K * (K + 1) / 2;
        T g[MK][4];
#pragma unroll
        for (int e = 0; e < MK; ++e) {
            float tmp[4];
            bld4<AUX>(F + (size_t)e * n_pix, (uint32_t)n_pix, (uint32_t)p0, tmp);
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
            bld4<AUX>(F + (size_t)j * n_pix, (uint32_t)n_pix, (uint32_t)p0, d);
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
