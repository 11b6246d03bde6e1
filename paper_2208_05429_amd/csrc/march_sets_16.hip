// march_sets_16.hip -- marching-kernel instantiations for the D3Q15 and D3Q27
// velocity sets with FP16/BF16 offset storage (FP32 arithmetic): the default
// tiles of FP32, one and two merged steps.
#include "march_sets.hpp"

namespace lbm {

template <int S>
using List_q15_16 = ShapeList<PRSetShape<D3Q15, S, 2, 16, 64>, PRSetShape<D3Q15, S, 1, 16, 64>,
                              SetShape<D3Q15, S, 2, 16, 64, 512>, SetShape<D3Q15, S, 1, 16, 64, 512>,
                              SetShape<D3Q15, S, 2, 12, 28, 512>, SetShape<D3Q15, S, 1, 14, 30, 512>>;
template <int S>
using List_q27_16 = ShapeList<SetShape<D3Q27, S, 2, 16, 32, 512>, SetShape<D3Q27, S, 1, 16, 32, 512>,
                              SetShape<D3Q27, S, 2, 12, 28, 512>, SetShape<D3Q27, S, 1, 14, 30, 512>>;

hipError_t launch_march_set16(int lat, int storage, bool walls, bool force, const MarchPlan& p, const MarchArgs& a,
                              hipStream_t s)
{
    if (lat == 15) return storage == ST_F16 ? List_q15_16<ST_F16>::launch(walls, force, p, a, s)
                                            : List_q15_16<ST_BF16>::launch(walls, force, p, a, s);
    if (lat == 27) return storage == ST_F16 ? List_q27_16<ST_F16>::launch(walls, force, p, a, s)
                                            : List_q27_16<ST_BF16>::launch(walls, force, p, a, s);
    return hipErrorInvalidValue;
}

int max_blocks_set16(int lat, int storage, bool walls, bool force, const MarchPlan& p)
{
    if (lat == 15) return storage == ST_F16 ? List_q15_16<ST_F16>::max_blocks(walls, force, p)
                                            : List_q15_16<ST_BF16>::max_blocks(walls, force, p);
    if (lat == 27) return storage == ST_F16 ? List_q27_16<ST_F16>::max_blocks(walls, force, p)
                                            : List_q27_16<ST_BF16>::max_blocks(walls, force, p);
    return 0;
}

}  // namespace lbm
