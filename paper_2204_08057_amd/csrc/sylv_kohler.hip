// Kernels of the sparse-dense Sylvester solver of Section 3.3.1 (Alg. 3) for eq. (Axb-Sylv),
//
//     N^-1 D2 M + M Lhat = F,   Lhat = A^T T A P^-1,   F = Y^T T A P^-1,
//
// with the small coefficient Lhat = W R W^-1 (R upper triangular; W orthogonal for the Schur
// form of Alg. 3, or Lemma 2's eigenvectors when the columns are decoupled).  Column i of the
// transformed unknown Xhat = M W solves the shifted sparse system
//
//     (D2 + R_ii N) xhat_i = N (F W e_i - sum_(l < i) xhat_l R_li)
//
// (Alg. 3's shifted solve multiplied through by N, so that its matrix is symmetric positive
// definite); the host runs each such system as a one-component problem of the conjugate-gradient
// solver.  These kernels form the right-hand sides and the back-transform M = Xhat W^-1.  F comes
// from the Lanczos start kernel (the start block Yhat of Alg. 5 is the same matrix).

#include "sylv_device.h"

namespace sylv {
namespace {

using namespace dev;

// b_i = n (.) (Yh Fw e_i - sum_(l < i) Rc[l][i] xhat_l) for the columns i in [i0, i1) (Rc is
// zero when the columns are decoupled).  Planes are [k][n_pix]; b_i goes to plane i of b.
template <int K>
__global__ __launch_bounds__(kBlock) void k_kh_rhs(const double *__restrict__ Yh,
                                                   const double *__restrict__ n,
                                                   const double *__restrict__ Xh, KhCoef c,
                                                   int i0, int i1, int n_pix,
                                                   double *__restrict__ b) {
    const int chunk = xcd_remap(blockIdx.x, gridDim.x);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int p = chunk * kChunk + e * kBlock + threadIdx.x;
        if (p >= n_pix) continue;
        double y[K];
#pragma unroll
        for (int j = 0; j < K; ++j) y[j] = gp(Yh)[(size_t)j * n_pix + p];
        const double np = gp(n)[p];
        for (int i = i0; i < i1; ++i) {
            double v = 0.0;
#pragma unroll
            for (int j = 0; j < K; ++j) v += y[j] * c.Fw[j][i];
            for (int l = 0; l < i; ++l) v -= c.Rc[l][i] * gp(Xh)[(size_t)l * n_pix + p];
            gp(b)[(size_t)i * n_pix + p] = np * v;
        }
    }
}

// X[j][p] = sum_i Xhat[i][p] T[i][j]  (M = Xhat W^-1).
template <int K>
__global__ __launch_bounds__(kBlock) void k_kh_back(const double *__restrict__ Xh, KhBack t,
                                                    int n_pix, double *__restrict__ X) {
    const int chunk = xcd_remap(blockIdx.x, gridDim.x);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int p = chunk * kChunk + e * kBlock + threadIdx.x;
        if (p >= n_pix) continue;
        double xh[K];
#pragma unroll
        for (int i = 0; i < K; ++i) xh[i] = gp(Xh)[(size_t)i * n_pix + p];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            double v = 0.0;
#pragma unroll
            for (int i = 0; i < K; ++i) v += xh[i] * t.T[i][j];
            gp(X)[(size_t)j * n_pix + p] = v;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_kh_zero(double *__restrict__ x, long n) {
    const long i = (long)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) gp(x)[i] = 0.0;
}

// ||b - G x|| / ||b|| of eq. (Axb) from the squared norms of the Lanczos residual pass.
__global__ void k_kh_relres(const LzState *st, double *out) {
    if (threadIdx.x == 0) *out = st->bb > 0.0 ? sqrt(st->rr / st->bb) : 0.0;
}

}  // namespace

hipError_t kh_launch_rhs(const double *Yh, const double *n, const double *Xh, const KhCoef &c,
                         int k, int i0, int i1, int n_pix, double *b, hipStream_t s) {
    return dispatch_k(k, [&](auto kt) -> hipError_t {
        constexpr int K = decltype(kt)::value;
        hipLaunchKernelGGL((k_kh_rhs<K>), dim3(blocks_for(n_pix, kChunk)), dim3(kBlock), 0, s,
                           Yh, n, Xh, c, i0, i1, n_pix, b);
        return hipGetLastError();
    });
}

hipError_t kh_launch_back(const double *Xh, const KhBack &t, int k, int n_pix, double *X,
                          hipStream_t s) {
    return dispatch_k(k, [&](auto kt) -> hipError_t {
        constexpr int K = decltype(kt)::value;
        hipLaunchKernelGGL((k_kh_back<K>), dim3(blocks_for(n_pix, kChunk)), dim3(kBlock), 0, s,
                           Xh, t, n_pix, X);
        return hipGetLastError();
    });
}

hipError_t kh_launch_zero(double *x, long n, hipStream_t s) {
    hipLaunchKernelGGL(k_kh_zero, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, x, n);
    return hipGetLastError();
}

hipError_t kh_launch_relres(const LzState *st, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_kh_relres, dim3(1), dim3(64), 0, s, st, out);
    return hipGetLastError();
}

}  // namespace sylv
