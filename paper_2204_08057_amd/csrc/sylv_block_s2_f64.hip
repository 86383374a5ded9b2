// Block conjugate gradients: the launches for s = 2 right-hand sides in float64.

#include "sylv_block_impl.h"

namespace sylv {

template struct BlockLaunch<2, double>;

}  // namespace sylv
