// march_sets.hpp -- compiled shapes of the marching kernel for the D3Q15 and
// D3Q27 velocity sets (march_sets.hip instantiates them) and their launchers.
#pragma once

#include "march_dispatch.hpp"

namespace lbm {

// D3Q15 / D3Q27 (plain layout, one round): {M, TY, TZ, NT} for two and one
// merged steps, by set, storage and variant (0: the default, the fastest
// measured at 256^3).  A frame of (TY + 2M) x (TZ + 2M) columns takes one to
// three columns per thread;
// D3Q27 in FP64 takes a smaller tile so that its 24 exchanged directions fit
// in LDS.
struct SetShapes {
    int lat, storage, variant;
    ShapeEntry m2, m1;
};
constexpr SetShapes kSetShapes[] = {
    {15, ST_F32, 0, {2, 16, 64, 512, 0, 1}, {1, 16, 64, 512, 0, 1}},  // three columns per thread
    {15, ST_F32, 1, {2, 16, 32, 512, 0, 1}, {1, 16, 32, 512, 0, 1}},
    {15, ST_F32, 2, {2, 12, 28, 512, 0, 1}, {1, 14, 30, 512, 0, 1}},
    {15, ST_F64, 0, {2, 12, 28, 512, 0, 1}, {1, 14, 30, 512, 0, 1}},
    {27, ST_F32, 0, {2, 16, 32, 512, 0, 1}, {1, 16, 32, 512, 0, 1}},  // two columns per thread
    {27, ST_F32, 1, {2, 12, 28, 512, 0, 1}, {1, 14, 30, 512, 0, 1}},
    {27, ST_F64, 0, {2, 8, 24, 384, 0, 1}, {1, 10, 26, 384, 0, 1}},
};
hipError_t launch_march_set(int lat, int storage, bool walls, bool force, const MarchPlan& p, const MarchArgs& a,
                            hipStream_t s);
int max_blocks_set(int lat, int storage, bool walls, bool force, const MarchPlan& p);

}  // namespace lbm
