// Block conjugate gradients: the launches for s = 4 right-hand sides in float64.

#include "sylv_block_impl.h"

namespace sylv {

template struct BlockLaunch<4, double>;

}  // namespace sylv
