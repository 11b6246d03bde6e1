// march_f64.hip -- marching-kernel instantiations for this storage type.
#include "march_dispatch.hpp"

namespace lbm {

using List_f64 = ShapeList<Shape<ST_F64, 2, 10, 32, 512, true>, Shape<ST_F64, 1, 12, 34, 512, true>,
                           Shape<ST_F64, 2, 12, 28, 512, true>, Shape<ST_F64, 1, 14, 30, 512, true>,
                           Shape<ST_F64, 2, 10, 32, 512, true, 2>, Shape<ST_F64, 1, 12, 34, 512, true, 2>>;

hipError_t launch_march_f64(bool walls, bool force, const MarchPlan& p, const MarchArgs& a, hipStream_t s)
{
    return List_f64::launch(walls, force, p, a, s);
}

int max_blocks_f64(bool walls, bool force, const MarchPlan& p) { return List_f64::max_blocks(walls, force, p); }

}  // namespace lbm
