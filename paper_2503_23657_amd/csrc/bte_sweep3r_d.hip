// 3D rows-per-lane sweep kernel in double: instantiations and dispatch.
#include "bte_sweep2d_launch.h"

namespace bte {

BTE3R_UNIT(double, d)

}  // namespace bte
