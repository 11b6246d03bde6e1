// march_sets.hip -- marching-kernel instantiations for the D3Q15 and D3Q27
// velocity sets: the one-column-per-thread layout of march.hpp, FP64 and
// FP32 storage, one and two merged steps, one round per pass.
#include "march_sets.hpp"

namespace lbm {

template <class LT, int S, int M, int TY, int TZ, int NT>
struct SetShape {
    static bool match(const MarchPlan& p)
    {
        return p.pr == 0 && p.pf == 1 && p.M == M && p.TY == TY && p.TZ == TZ && p.NT == NT;
    }
    static hipError_t launch(bool walls, bool force, const MarchPlan& p, const MarchArgs& a, hipStream_t s)
    {
        if (force)
            return walls ? launch_march_shape<S, M, TY, TZ, NT, true, true, false, LT>(p, a, s)
                         : launch_march_shape<S, M, TY, TZ, NT, false, true, false, LT>(p, a, s);
        return walls ? launch_march_shape<S, M, TY, TZ, NT, true, false, false, LT>(p, a, s)
                     : launch_march_shape<S, M, TY, TZ, NT, false, false, false, LT>(p, a, s);
    }
    static int max_blocks(bool walls, bool force)
    {
        if (force)
            return walls ? max_blocks_shape<S, M, TY, TZ, NT, true, true, false, LT>()
                         : max_blocks_shape<S, M, TY, TZ, NT, false, true, false, LT>();
        return walls ? max_blocks_shape<S, M, TY, TZ, NT, true, false, false, LT>()
                     : max_blocks_shape<S, M, TY, TZ, NT, false, false, false, LT>();
    }
};

template <class LT, int S, int M, int TY, int TZ>
struct PRSetShape {
    static constexpr int NT = TY * TZ / 2;
    static bool match(const MarchPlan& p)
    {
        return p.pr == 1 && p.pf == 1 && p.M == M && p.TY == TY && p.TZ == TZ && p.NT == NT;
    }
    static hipError_t launch(bool walls, bool force, const MarchPlan& p, const MarchArgs& a, hipStream_t s)
    {
        if (force)
            return walls ? launch_march_pr_shape<S, M, TY, TZ, true, true, 1, LT>(p, a, s)
                         : launch_march_pr_shape<S, M, TY, TZ, false, true, 1, LT>(p, a, s);
        return walls ? launch_march_pr_shape<S, M, TY, TZ, true, false, 1, LT>(p, a, s)
                     : launch_march_pr_shape<S, M, TY, TZ, false, false, 1, LT>(p, a, s);
    }
    static int max_blocks(bool walls, bool force)
    {
        if (force)
            return walls ? max_blocks_pr_shape<S, M, TY, TZ, true, true, 1, LT>()
                         : max_blocks_pr_shape<S, M, TY, TZ, false, true, 1, LT>();
        return walls ? max_blocks_pr_shape<S, M, TY, TZ, true, false, 1, LT>()
                     : max_blocks_pr_shape<S, M, TY, TZ, false, false, 1, LT>();
    }
};

// the shapes of kSetShapes (march_sets.hpp)
using List_q15_f32 = ShapeList<PRSetShape<D3Q15, ST_F32, 2, 16, 64>, PRSetShape<D3Q15, ST_F32, 1, 16, 64>,
                               SetShape<D3Q15, ST_F32, 2, 12, 28, 512>, SetShape<D3Q15, ST_F32, 1, 14, 30, 512>,
                               SetShape<D3Q15, ST_F32, 2, 16, 32, 512>, SetShape<D3Q15, ST_F32, 1, 16, 32, 512>,
                               SetShape<D3Q15, ST_F32, 2, 16, 64, 512>, SetShape<D3Q15, ST_F32, 1, 16, 64, 512>>;
using List_q15_f64 = ShapeList<SetShape<D3Q15, ST_F64, 2, 12, 28, 512>, SetShape<D3Q15, ST_F64, 1, 14, 30, 512>>;
using List_q27_f32 = ShapeList<SetShape<D3Q27, ST_F32, 2, 12, 28, 512>, SetShape<D3Q27, ST_F32, 1, 14, 30, 512>,
                               SetShape<D3Q27, ST_F32, 2, 16, 32, 512>, SetShape<D3Q27, ST_F32, 1, 16, 32, 512>>;
using List_q27_f64 = ShapeList<SetShape<D3Q27, ST_F64, 2, 8, 24, 384>, SetShape<D3Q27, ST_F64, 1, 10, 26, 384>>;

hipError_t launch_march_set(int lat, int storage, bool walls, bool force, const MarchPlan& p, const MarchArgs& a,
                            hipStream_t s)
{
    if (lat == 15) return storage == ST_F64 ? List_q15_f64::launch(walls, force, p, a, s)
                                            : List_q15_f32::launch(walls, force, p, a, s);
    if (lat == 27) return storage == ST_F64 ? List_q27_f64::launch(walls, force, p, a, s)
                                            : List_q27_f32::launch(walls, force, p, a, s);
    return hipErrorInvalidValue;
}

int max_blocks_set(int lat, int storage, bool walls, bool force, const MarchPlan& p)
{
    if (lat == 15) return storage == ST_F64 ? List_q15_f64::max_blocks(walls, force, p)
                                            : List_q15_f32::max_blocks(walls, force, p);
    if (lat == 27) return storage == ST_F64 ? List_q27_f64::max_blocks(walls, force, p)
                                            : List_q27_f32::max_blocks(walls, force, p);
    return 0;
}

}  // namespace lbm
