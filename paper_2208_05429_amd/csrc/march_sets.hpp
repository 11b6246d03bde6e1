// march_sets.hpp -- compiled shapes of the marching kernel for the D3Q15 and
// D3Q27 velocity sets (march_sets.hip instantiates them) and their launchers.
#pragma once

#include "march_dispatch.hpp"

namespace lbm {

// D3Q15 / D3Q27: {M, TY, TZ, NT, pair-and-ring} for two and one
// merged steps, by set, storage and variant (0: the default, the fastest
// measured at 256^3).  D3Q15 in FP32 has the pair-and-ring layout of
// march_pr.hpp (an interior pair and a ring column per thread; even nz); in
// the plain layout a frame of (TY + 2M) x (TZ + 2M) columns takes one to
// three columns per thread;
// D3Q27 in FP64 takes a smaller tile so that its 24 exchanged directions fit
// in LDS.
struct SetShapes {
    int lat, storage, variant;
    ShapeEntry m2, m1;
};
constexpr SetShapes kSetShapes[] = {
    {15, ST_F32, 0, {2, 16, 64, 512, 1, 1}, {1, 16, 64, 512, 1, 1}},  // pair and ring (even nz; else variant 1)
    {15, ST_F32, 1, {2, 16, 64, 512, 0, 1}, {1, 16, 64, 512, 0, 1}},  // three columns per thread
    {15, ST_F32, 2, {2, 16, 32, 512, 0, 1}, {1, 16, 32, 512, 0, 1}},
    {15, ST_F32, 3, {2, 12, 28, 512, 0, 1}, {1, 14, 30, 512, 0, 1}},
    {15, ST_F64, 0, {2, 10, 32, 512, 0, 1}, {1, 12, 34, 512, 0, 1}},  // whole cache-line rows (as D3Q19 FP64)
    {15, ST_F64, 1, {2, 12, 28, 512, 0, 1}, {1, 14, 30, 512, 0, 1}},
    {27, ST_F32, 0, {2, 16, 32, 512, 0, 1}, {1, 16, 32, 512, 0, 1}},  // two columns per thread
    {27, ST_F32, 1, {2, 12, 28, 512, 0, 1}, {1, 14, 30, 512, 0, 1}},
    {27, ST_F64, 0, {2, 8, 32, 448, 0, 1}, {1, 10, 32, 448, 0, 1}},  // whole cache-line rows; 256 tiles of 256^2
    {27, ST_F64, 1, {2, 8, 24, 384, 0, 1}, {1, 10, 26, 384, 0, 1}},
    {27, ST_F64, 2, {2, 10, 26, 448, 0, 1}, {1, 10, 26, 384, 0, 1}},  // a 10-row height for periodic y seams
    // FP16/BF16 offset storage: the default tiles of FP32 (and the plain
    // 16 x 64 tile that D3Q15 takes for odd nz)
    {15, ST_F16, 0, {2, 16, 64, 512, 1, 1}, {1, 16, 64, 512, 1, 1}},
    {15, ST_F16, 1, {2, 16, 64, 512, 0, 1}, {1, 16, 64, 512, 0, 1}},
    {15, ST_BF16, 0, {2, 16, 64, 512, 1, 1}, {1, 16, 64, 512, 1, 1}},
    {15, ST_BF16, 1, {2, 16, 64, 512, 0, 1}, {1, 16, 64, 512, 0, 1}},
    {27, ST_F16, 0, {2, 16, 32, 512, 0, 1}, {1, 16, 32, 512, 0, 1}},
    {27, ST_BF16, 0, {2, 16, 32, 512, 0, 1}, {1, 16, 32, 512, 0, 1}},
    // a 12-row height, for planes in rounds across a periodic y seam
    {15, ST_F16, 2, {2, 12, 28, 512, 0, 1}, {1, 14, 30, 512, 0, 1}},
    {15, ST_BF16, 2, {2, 12, 28, 512, 0, 1}, {1, 14, 30, 512, 0, 1}},
    {27, ST_F16, 1, {2, 12, 28, 512, 0, 1}, {1, 14, 30, 512, 0, 1}},
    {27, ST_BF16, 1, {2, 12, 28, 512, 0, 1}, {1, 14, 30, 512, 0, 1}},
};
hipError_t launch_march_set(int lat, int storage, bool walls, bool force, const MarchPlan& p, const MarchArgs& a,
                            hipStream_t s);
int max_blocks_set(int lat, int storage, bool walls, bool force, const MarchPlan& p);
hipError_t launch_march_q27(int storage, bool walls, bool force, const MarchPlan& p, const MarchArgs& a, hipStream_t s);
int max_blocks_q27(int storage, bool walls, bool force, const MarchPlan& p);
hipError_t launch_march_set16(int lat, int storage, bool walls, bool force, const MarchPlan& p, const MarchArgs& a,
                              hipStream_t s);
int max_blocks_set16(int lat, int storage, bool walls, bool force, const MarchPlan& p);

// A plain-layout shape of a set.  Planes that run in rounds launch the build
// with the band edge code (ROUNDS), the others the build without it.
template <class LT, int S, int M, int TY, int TZ, int NT>
struct SetShape {
    static bool match(const MarchPlan& p)
    {
        return p.pr == 0 && p.pf == 1 && p.M == M && p.TY == TY && p.TZ == TZ && p.NT == NT;
    }
    template <bool R>
    static hipError_t launch_r(bool walls, bool force, const MarchPlan& p, const MarchArgs& a, hipStream_t s)
    {
        if (force)
            return walls ? launch_march_shape<S, M, TY, TZ, NT, true, true, R, LT>(p, a, s)
                         : launch_march_shape<S, M, TY, TZ, NT, false, true, R, LT>(p, a, s);
        return walls ? launch_march_shape<S, M, TY, TZ, NT, true, false, R, LT>(p, a, s)
                     : launch_march_shape<S, M, TY, TZ, NT, false, false, R, LT>(p, a, s);
    }
    template <bool R>
    static int max_blocks_r(bool walls, bool force)
    {
        if (force)
            return walls ? max_blocks_shape<S, M, TY, TZ, NT, true, true, R, LT>()
                         : max_blocks_shape<S, M, TY, TZ, NT, false, true, R, LT>();
        return walls ? max_blocks_shape<S, M, TY, TZ, NT, true, false, R, LT>()
                     : max_blocks_shape<S, M, TY, TZ, NT, false, false, R, LT>();
    }
    static hipError_t launch(bool walls, bool force, const MarchPlan& p, const MarchArgs& a, hipStream_t s)
    {
        return p.nbands > 1 ? launch_r<true>(walls, force, p, a, s) : launch_r<false>(walls, force, p, a, s);
    }
    static int max_blocks(bool walls, bool force)
    {
        const int a = max_blocks_r<false>(walls, force), b = max_blocks_r<true>(walls, force);
        return a < b ? a : b;
    }
};

// A pair-and-ring shape of a set (march_pr.hpp: its band edge code is always
// built in).
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

}  // namespace lbm
