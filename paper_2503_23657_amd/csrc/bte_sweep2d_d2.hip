// 1D/2D sweep kernel in double, G = 2: instantiations and dispatch.
#include "bte_sweep2d_launch.h"

namespace bte {

BTE2D_UNIT(double, 2, d2)

}  // namespace bte
