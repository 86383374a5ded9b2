// The passes of the Fourier preconditioner in float32 on face grids (cosine transforms).

#include "sylv_fourier_impl.h"

namespace sylv {

hipError_t fp_apply_f32_face(const InstSet &set, int k, int inner, const void *rin,
                             void *zout, int upd, int it, hipStream_t s) {
    return fp_apply_impl<float, true>(set, k, inner, rin, zout, upd, it, s);
}

}  // namespace sylv
