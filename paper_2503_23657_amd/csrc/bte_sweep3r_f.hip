// 3D rows-per-lane sweep kernel in float: instantiations and dispatch.
#include "bte_sweep2d_launch.h"

namespace bte {

BTE3R_UNIT(float, f)

}  // namespace bte
