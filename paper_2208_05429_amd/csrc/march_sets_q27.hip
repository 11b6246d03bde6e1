// march_sets_q27.hip -- marching-kernel instantiations for the D3Q27 velocity
// set: FP64 and FP32 storage, one and two merged steps (its own translation
// unit, so the sets compile in parallel).
#include "march_sets.hpp"

namespace lbm {

// the D3Q27 shapes of kSetShapes (march_sets.hpp)
using List_q27_f32 = ShapeList<SetShape<D3Q27, ST_F32, 2, 12, 28, 512>, SetShape<D3Q27, ST_F32, 1, 14, 30, 512>,
                               SetShape<D3Q27, ST_F32, 2, 16, 32, 512>, SetShape<D3Q27, ST_F32, 1, 16, 32, 512>>;
using List_q27_f64 = ShapeList<SetShape<D3Q27, ST_F64, 2, 8, 24, 384>, SetShape<D3Q27, ST_F64, 1, 10, 26, 384>,
                               SetShape<D3Q27, ST_F64, 2, 8, 32, 448>, SetShape<D3Q27, ST_F64, 1, 10, 32, 448>,
                               SetShape<D3Q27, ST_F64, 2, 10, 26, 448>>;

hipError_t launch_march_q27(int storage, bool walls, bool force, const MarchPlan& p, const MarchArgs& a, hipStream_t s)
{
    return storage == ST_F64 ? List_q27_f64::launch(walls, force, p, a, s) : List_q27_f32::launch(walls, force, p, a, s);
}

int max_blocks_q27(int storage, bool walls, bool force, const MarchPlan& p)
{
    return storage == ST_F64 ? List_q27_f64::max_blocks(walls, force, p) : List_q27_f32::max_blocks(walls, force, p);
}

}  // namespace lbm
