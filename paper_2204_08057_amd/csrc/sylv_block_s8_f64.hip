// Block conjugate gradients: the launches for s = 8 right-hand sides in float64.

#include "sylv_block_impl.h"

namespace sylv {

template struct BlockLaunch<8, double>;

}  // namespace sylv
