// march_plan.hpp -- how an in-place marching pass is laid out and launched:
// the compiled shape a configuration takes, its tiles, x segments and rounds
// (make_plan), the work-buffer layout, the device's co-residency cap, and the
// launch of one pass round by round.  Host code behind the C ABI; nothing
// here is exported.
#pragma once

#include <stddef.h>

#include <string>

#include "../../include/lbm.h"
#include "lbm_internal.hpp"

namespace lbm {

constexpr int kMaxResident = 256;  // MI355X: 256 CUs, one marching workgroup per CU
constexpr size_t kAlign = 256;
// Progress counters are polled by every wave of every workgroup each plane;
// packed into a few cache lines they become a memory hot spot, so each gets
// its own stretch of memory.
constexpr int kFlagStride = 1024;  // ints (4 KB)

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
// the velocity set: 19 (the default, also for 0), 15 or 27
inline int lat_of(const lbm_config& c) { return c.velocities == 0 ? 19 : c.velocities; }
inline size_t elem_size(int storage) { return storage == LBM_F64 ? 8 : (storage == LBM_F32 ? 4 : 2); }
inline size_t real_size(int storage) { return storage == LBM_F64 ? 8 : 4; }

inline lbm_status fail(std::string* where, lbm_status st, const std::string& msg)
{
    if (where) *where = msg;
    return st;
}

// The compiled tile shape for M merged steps of this storage, variant and
// velocity set (plain: the one-column-per-thread layout of the same tile).
bool march_shape_of(int storage, int M, int variant, int nz, bool plain, MarchPlan* r, int lat = 19);
// A plain-layout shape whose last tile row across a periodic y seam is at
// least as thick as the halo (or whole).
bool plain_shape_for_seam(int storage, int M, int ny, MarchPlan* r, int lat = 19);
// Tiles, segments, rounds and the hazard neighbourhood of one pass of M
// steps for at most cap co-resident workgroups (last_segments: a short last
// band of tile rows may take x segments of its own).
lbm_status make_plan(const lbm_config& c, int M, int cap, MarchPlan* p, std::string* why, bool last_segments = true);
// Offsets of the work buffer's parts (off[6]) and its size; fills the plans
// of the pass lengths the scheme runs.
lbm_status layout(const lbm_config& c, int cap, MarchPlan plans[4], size_t off[6], size_t* total, std::string* why,
                  bool last_segments = true);
// Workgroups of the plan's kernel the device holds at once.
int device_cap(const lbm_config& c, const MarchPlan& p);

// The buffers of one marching pass (src == dst: in place).
struct PassBuffers {
    const void* src;
    void* dst;
    void* side;            // saved planes of the segment ends
    int* flags;            // [0] the time-out word, then one progress counter per work item
    unsigned char* shell;  // saved band boundary rows (rounds only)
    const void* force;     // body force or nullptr
};
// Launches the marching kernel of plan p once per round (band of tile rows);
// the prepass and band boundary copy of an in-place pass must precede it on
// the same stream.  force_timeout: the test hook that makes every hazard
// wait give up.  Returns the first launch error.
hipError_t launch_march_pass(const lbm_config& cfg, const Geom& g, const MarchPlan& p, const PassBuffers& b,
                             bool force_timeout, hipStream_t s);

}  // namespace lbm
