// Block conjugate gradients: the launches for s = 4 right-hand sides in float32 (the inner runs of the mixed path).

#include "sylv_block_impl.h"

namespace sylv {

template struct BlockLaunch<4, float>;

}  // namespace sylv
