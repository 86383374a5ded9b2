// The passes of the Fourier preconditioner in float64 on periodic grids (Fourier transforms).

#include "sylv_fourier_impl.h"

namespace sylv {

hipError_t fp_apply_f64_periodic(const InstSet &set, int k, int inner, const void *rin,
                                 void *zout, int upd, int it, hipStream_t s) {
    return fp_apply_impl<double, false>(set, k, inner, rin, zout, upd, it, s);
}

}  // namespace sylv
