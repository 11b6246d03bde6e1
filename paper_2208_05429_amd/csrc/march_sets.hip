// march_sets.hip -- marching-kernel instantiations for the D3Q15 velocity
// set (FP64 and FP32 storage, one and two merged steps) and the dispatch of
// both other sets (D3Q27: march_sets_q27.hip; 16-bit storage:
// march_sets_16.hip).
#include "march_sets.hpp"

namespace lbm {

// the D3Q15 shapes of kSetShapes (march_sets.hpp)
using List_q15_f32 = ShapeList<PRSetShape<D3Q15, ST_F32, 2, 16, 64>, PRSetShape<D3Q15, ST_F32, 1, 16, 64>,
                               SetShape<D3Q15, ST_F32, 2, 12, 28, 512>, SetShape<D3Q15, ST_F32, 1, 14, 30, 512>,
                               SetShape<D3Q15, ST_F32, 2, 16, 32, 512>, SetShape<D3Q15, ST_F32, 1, 16, 32, 512>,
                               SetShape<D3Q15, ST_F32, 2, 16, 64, 512>, SetShape<D3Q15, ST_F32, 1, 16, 64, 512>>;
using List_q15_f64 = ShapeList<SetShape<D3Q15, ST_F64, 2, 12, 28, 512>, SetShape<D3Q15, ST_F64, 1, 14, 30, 512>,
                               SetShape<D3Q15, ST_F64, 2, 10, 32, 512>, SetShape<D3Q15, ST_F64, 1, 12, 34, 512>>;

hipError_t launch_march_set(int lat, int storage, bool walls, bool force, const MarchPlan& p, const MarchArgs& a,
                            hipStream_t s)
{
    if (storage == ST_F16 || storage == ST_BF16) return launch_march_set16(lat, storage, walls, force, p, a, s);
    if (lat == 15) return storage == ST_F64 ? List_q15_f64::launch(walls, force, p, a, s)
                                            : List_q15_f32::launch(walls, force, p, a, s);
    if (lat == 27) return launch_march_q27(storage, walls, force, p, a, s);
    return hipErrorInvalidValue;
}

int max_blocks_set(int lat, int storage, bool walls, bool force, const MarchPlan& p)
{
    if (storage == ST_F16 || storage == ST_BF16) return max_blocks_set16(lat, storage, walls, force, p);
    if (lat == 15) return storage == ST_F64 ? List_q15_f64::max_blocks(walls, force, p)
                                            : List_q15_f32::max_blocks(walls, force, p);
    if (lat == 27) return max_blocks_q27(storage, walls, force, p);
    return 0;
}

}  // namespace lbm
