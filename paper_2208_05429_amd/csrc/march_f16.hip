// march_f16.hip -- marching-kernel instantiations for this storage type.
#include "march_dispatch.hpp"

namespace lbm {

using List_f16 = ShapeList<PRShape<ST_F16, 2, 16, 64, true>, PRShape<ST_F16, 1, 16, 64, true>, Shape<ST_F16, 2, 16, 64, 512, true>, Shape<ST_F16, 1, 16, 64, 512, true>, PRShape<ST_F16, 2, 32, 32, true>, PRShape<ST_F16, 1, 32, 32, true>, Shape<ST_F16, 2, 32, 32, 512, true>, Shape<ST_F16, 1, 32, 32, 512, true>, PRShape<ST_F16, 2, 16, 64, true, 2>, PRShape<ST_F16, 1, 16, 64, true, 2>, Shape<ST_F16, 2, 16, 16, 448, true>, Shape<ST_F16, 1, 16, 16, 448, true>, Shape<ST_F16, 2, 12, 28, 512, true>, Shape<ST_F16, 1, 14, 30, 512, true>>;

hipError_t launch_march_f16(bool walls, bool force, const MarchPlan& p, const MarchArgs& a, hipStream_t s)
{
    return List_f16::launch(walls, force, p, a, s);
}

int max_blocks_f16(bool walls, bool force, const MarchPlan& p) { return List_f16::max_blocks(walls, force, p); }

}  // namespace lbm
