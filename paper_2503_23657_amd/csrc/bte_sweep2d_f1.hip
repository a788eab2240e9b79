// 1D/2D sweep kernel in float, G = 1: instantiations and dispatch.
#include "bte_sweep2d_launch.h"

namespace bte {

BTE2D_UNIT_WITH_SECOND(float, 1, f1)

}  // namespace bte
