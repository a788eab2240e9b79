// 1D/2D sweep kernel in float, G = 2: instantiations and dispatch.
#include "bte_sweep2d_launch.h"

namespace bte {

BTE2D_UNIT(float, 2, f2)

}  // namespace bte
