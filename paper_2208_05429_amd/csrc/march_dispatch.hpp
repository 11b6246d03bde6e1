// march_dispatch.hpp -- compiled shapes of the marching kernel and their
// dispatch from a runtime plan.  Each storage type instantiates its own list
// in its own translation unit (march_<type>.hip).
#pragma once

#include "march.hpp"
#include "march_pr.hpp"

namespace lbm {

// A plain-layout shape (march.hpp).  PF is how many planes ahead the loads
// run; walls and a body force use PF = 1 (their extra registers leave no room
// for a second plane of loads).
template <int S, int M, int TY, int TZ, int NT, bool ALLOW_FORCE, int PF = 1>
struct Shape {
    static bool match(const MarchPlan& p)
    {
        return p.pr == 0 && p.pf == PF && p.M == M && p.TY == TY && p.TZ == TZ && p.NT == NT;
    }
    // FP64 always runs the build with the band edge code; the other storages
    // only for planes that run in rounds
    template <bool R>
    static hipError_t launch_r(bool walls, bool force, const MarchPlan& p, const MarchArgs& a, hipStream_t s)
    {
        if constexpr (ALLOW_FORCE) {
            if (force)
                return walls ? launch_march_shape<S, M, TY, TZ, NT, true, true, R>(p, a, s)
                             : launch_march_shape<S, M, TY, TZ, NT, false, true, R>(p, a, s);
        } else {
            if (force) return hipErrorInvalidValue;
        }
        return walls ? launch_march_shape<S, M, TY, TZ, NT, true, false, R>(p, a, s)
                     : launch_march_shape<S, M, TY, TZ, NT, false, false, R, D3Q19, PF>(p, a, s);
    }
    template <bool R>
    static int max_blocks_r(bool walls, bool force)
    {
        if constexpr (ALLOW_FORCE) {
            if (force)
                return walls ? max_blocks_shape<S, M, TY, TZ, NT, true, true, R>()
                             : max_blocks_shape<S, M, TY, TZ, NT, false, true, R>();
        } else {
            if (force) return 0;
        }
        return walls ? max_blocks_shape<S, M, TY, TZ, NT, true, false, R>()
                     : max_blocks_shape<S, M, TY, TZ, NT, false, false, R, D3Q19, PF>();
    }
    static hipError_t launch(bool walls, bool force, const MarchPlan& p, const MarchArgs& a, hipStream_t s)
    {
        if constexpr (S == ST_F64) {
            return launch_r<true>(walls, force, p, a, s);
        } else {
            return p.nbands > 1 ? launch_r<true>(walls, force, p, a, s) : launch_r<false>(walls, force, p, a, s);
        }
    }
    static int max_blocks(bool walls, bool force)
    {
        if constexpr (S == ST_F64) {
            return max_blocks_r<true>(walls, force);
        } else {
            const int a = max_blocks_r<false>(walls, force), b = max_blocks_r<true>(walls, force);
            return a < b ? a : b;
        }
    }
};

// A pair-and-ring shape (march_pr.hpp): NT = TY*TZ/2, needs an even nz.  PF is
// how many planes ahead the loads run; a body force always uses PF = 1 (its
// extra registers leave no room for a second plane of loads).
template <int S, int M, int TY, int TZ, bool ALLOW_FORCE, int PF = 1>
struct PRShape {
    static constexpr int NT = TY * TZ / 2;
    static bool match(const MarchPlan& p)
    {
        return p.pr == 1 && p.pf == PF && p.M == M && p.TY == TY && p.TZ == TZ && p.NT == NT;
    }
    static hipError_t launch(bool walls, bool force, const MarchPlan& p, const MarchArgs& a, hipStream_t s)
    {
        if constexpr (ALLOW_FORCE) {
            if (force)
                return walls ? launch_march_pr_shape<S, M, TY, TZ, true, true, 1>(p, a, s)
                             : launch_march_pr_shape<S, M, TY, TZ, false, true, 1>(p, a, s);
        } else {
            if (force) return hipErrorInvalidValue;
        }
        return walls ? launch_march_pr_shape<S, M, TY, TZ, true, false, PF>(p, a, s)
                     : launch_march_pr_shape<S, M, TY, TZ, false, false, PF>(p, a, s);
    }
    static int max_blocks(bool walls, bool force)
    {
        if constexpr (ALLOW_FORCE) {
            if (force)
                return walls ? max_blocks_pr_shape<S, M, TY, TZ, true, true, 1>()
                             : max_blocks_pr_shape<S, M, TY, TZ, false, true, 1>();
        } else {
            if (force) return 0;
        }
        return walls ? max_blocks_pr_shape<S, M, TY, TZ, true, false, PF>()
                     : max_blocks_pr_shape<S, M, TY, TZ, false, false, PF>();
    }
};

template <class... Shapes>
struct ShapeList {
    static hipError_t launch(bool walls, bool force, const MarchPlan& p, const MarchArgs& a, hipStream_t s)
    {
        hipError_t r = hipErrorInvalidValue;
        bool done = false;
        ((!done && Shapes::match(p) ? (r = Shapes::launch(walls, force, p, a, s), done = true) : false), ...);
        return r;
    }
    static int max_blocks(bool walls, bool force, const MarchPlan& p)
    {
        int r = 0;
        bool done = false;
        ((!done && Shapes::match(p) ? (r = Shapes::max_blocks(walls, force), done = true) : false), ...);
        return r;
    }
};

// Shapes per storage type, {M, TY, TZ, NT, pair_ring, prefetch planes}, in
// variant order (variant v uses entries 2v (M = 2) and 2v+1 (M = 1)).
// Pair-and-ring shapes need an even nz; the planner falls back to variant 1
// (plain layout) otherwise.
struct ShapeEntry {
    int M, TY, TZ, NT, pr, pf;
};
// FP64: 10 x 32 tiles first (rows of 32 doubles are whole cache lines, and a
// 1024-wide plane takes 32 tiles per row: eight rows fill 256 workgroups),
// 12 x 28 as variant 1, and as variant 2 the 10 x 32 tile with loads two
// planes ahead (periodic without a force; measured 1-2 % slower than
// variant 0).
constexpr ShapeEntry kShapesF64[] = {{2, 10, 32, 512, 0, 1}, {1, 12, 34, 512, 0, 1},
                                     {2, 12, 28, 512, 0, 1}, {1, 14, 30, 512, 0, 1},
                                     {2, 10, 32, 512, 0, 2}, {1, 12, 34, 512, 0, 2}};
// 32- and 16-bit storage (variant v takes entries 2v and 2v+1): 16 x 64
// pair-and-ring tiles; the plain layout of 16 x 64; 32 x 32 pair-and-ring and
// plain; 16 x 64 pair-and-ring with loads two planes ahead; 16 x 16 plain
// tiles of 448 threads for lattices that give the others under half the
// device's workgroups (128 x 64 x 64 channel with walls and a force: 41.7
// against 70.0 us per step; slower from 128^3 up); and 12 x 28 plain tiles,
// whose 12-row height also serves planes in rounds across a periodic y seam
// where every 16-row multiple would leave a last row thinner than the halo.
constexpr ShapeEntry kShapesF32[] = {{2, 16, 64, 512, 1, 1}, {1, 16, 64, 512, 1, 1}, {2, 16, 64, 512, 0, 1},
                                     {1, 16, 64, 512, 0, 1}, {2, 32, 32, 512, 1, 1}, {1, 32, 32, 512, 1, 1},
                                     {2, 32, 32, 512, 0, 1}, {1, 32, 32, 512, 0, 1}, {2, 16, 64, 512, 1, 2},
                                     {1, 16, 64, 512, 1, 2}, {2, 16, 16, 448, 0, 1}, {1, 16, 16, 448, 0, 1},
                                     {2, 12, 28, 512, 0, 1}, {1, 14, 30, 512, 0, 1}};
// Three merged steps (plain layout, FP32; variant v of LBM_SWAP3 takes entry
// v): 16 x 32 tiles with two frame columns per thread (a 22 x 38 frame, three
// exchange levels in 139 KB of LDS; 512^3 43.7 GLUPS), then one column per
// thread, (TY + 6) x (TZ + 6) <= 512, on 10 x 26 and 16 x 16 tiles (30.4).
constexpr ShapeEntry kShapesM3F32[] = {{3, 16, 32, 512, 0, 1}, {3, 10, 26, 512, 0, 1}, {3, 16, 16, 512, 0, 1}};

hipError_t launch_march_f64(bool walls, bool force, const MarchPlan& p, const MarchArgs& a, hipStream_t s);
hipError_t launch_march_f32(bool walls, bool force, const MarchPlan& p, const MarchArgs& a, hipStream_t s);
hipError_t launch_march_f16(bool walls, bool force, const MarchPlan& p, const MarchArgs& a, hipStream_t s);
hipError_t launch_march_bf16(bool walls, bool force, const MarchPlan& p, const MarchArgs& a, hipStream_t s);
int max_blocks_f64(bool walls, bool force, const MarchPlan& p);
int max_blocks_f32(bool walls, bool force, const MarchPlan& p);
int max_blocks_f16(bool walls, bool force, const MarchPlan& p);
int max_blocks_bf16(bool walls, bool force, const MarchPlan& p);

}  // namespace lbm
