// 1D/2D sweep kernel in double, G = 1: instantiations and dispatch.
#include "bte_sweep2d_launch.h"

namespace bte {

BTE2D_UNIT_WITH_SECOND(double, 1, d1)

}  // namespace bte
