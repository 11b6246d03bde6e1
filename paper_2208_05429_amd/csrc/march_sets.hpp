// march_sets.hpp -- compiled shapes of the marching kernel for the D3Q15 and
// D3Q27 velocity sets (march_sets.hip instantiates them) and their launchers.
#pragma once

#include "march_dispatch.hpp"

namespace lbm {

// D3Q15 / D3Q27 (one round): {M, TY, TZ, NT, pair-and-ring} for two and one
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
    {15, ST_F64, 0, {2, 12, 28, 512, 0, 1}, {1, 14, 30, 512, 0, 1}},
    {27, ST_F32, 0, {2, 16, 32, 512, 0, 1}, {1, 16, 32, 512, 0, 1}},  // two columns per thread
    {27, ST_F32, 1, {2, 12, 28, 512, 0, 1}, {1, 14, 30, 512, 0, 1}},
    {27, ST_F64, 0, {2, 8, 24, 384, 0, 1}, {1, 10, 26, 384, 0, 1}},
};
hipError_t launch_march_set(int lat, int storage, bool walls, bool force, const MarchPlan& p, const MarchArgs& a,
                            hipStream_t s);
int max_blocks_set(int lat, int storage, bool walls, bool force, const MarchPlan& p);

}  // namespace lbm
