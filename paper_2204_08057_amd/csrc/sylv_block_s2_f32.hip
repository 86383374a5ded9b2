// Block conjugate gradients: the launches for s = 2 right-hand sides in float32 (the inner runs of the mixed path).

#include "sylv_block_impl.h"

namespace sylv {

template struct BlockLaunch<2, float>;

}  // namespace sylv
