// lbm_internal.hpp -- argument blocks and launcher declarations shared by the
// HIP kernels and the C-ABI implementation.  Nothing here is exported.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lbm {

// Geometry and physics common to every kernel.
struct Geom {
    int nx, ny, nz;
    long long N;      // nx*ny*nz
    long long PL;     // ny*nz, cells per x-plane
    int wall[3];      // 1 if the axis has walls (0: periodic)
    int moving_face;  // -1 or 0..5 (-x,+x,-y,+y,-z,+z)
    double uw[3];     // moving-face velocity
    double omega;     // 1/tau
    int lat;          // velocity set: 19 (D3Q19), 15 (D3Q15) or 27 (D3Q27)
};

// One in-place marching pass (M = steps merged per pass).
struct MarchPlan {
    int M = 0;
    int TY = 0, TZ = 0, NT = 0;  // interior tile and threads per workgroup
    int pr = 0;                  // 1: pair-and-ring kernel layout
    int pf = 1;                  // planes the loads run ahead
    int nty = 0, ntz = 0;        // tiles along y and z
    int nseg = 0, seg_len = 0;   // x segments
    int ry = 1, rz = 1;          // neighbourhood radius (in tiles) of the hazard check
    int blocks = 0;              // nty*ntz*nseg work items, all co-resident
    int cap = 0;                 // co-resident workgroups the plan was made for
    int xcd_remap = 0;           // map consecutive work items onto one XCD
    size_t side_bytes = 0;       // side planes: nseg * M planes * 19 values
    int flag_stride = 1;         // ints between two progress counters
    size_t flag_bytes = 0;       // timeout word + one counter per work item
    // y-z planes with more tiles than can be co-resident run as rounds over
    // bands of nty_band tile rows (both kernel layouts)
    int nbands = 1, nty_band = 0;
    // a last band with fewer tile rows marches in x segments of its own (more
    // of them, to fill the device); 0: the same segments as the other bands.
    // Its side planes follow the others' in the side buffer, at side_off_last.
    int nseg_last = 0, seg_len_last = 0;
    size_t side_off_last = 0;
    size_t shell_bytes = 0;      // the M boundary rows of every band, all x: nbands * 2 * M rows
    int lockstep = 0;            // 1: a plane is stored once the neighbours finished the previous iteration
};

struct MarchArgs {
    Geom g;
    void* f;            // distributions read (time t)
    void* fo;           // distributions written (time t+M): f itself in place, else another buffer
    int inplace;        // fo == f: side planes and progress counters guard the in-place update
    void* side;         // time-t copies of the first M planes of every segment
    const void* force;  // 3N or null
    int* flags;         // progress (planes loaded) of every work item
    int nty, ntz, nseg, seg_len, ry, rz, xcd_remap;
    int fstride;  // ints between two progress counters (counter of tile (seg, ty, tz) at
                  // flags[(1 + (seg * nty + ty) * ntz + tz) * fstride])
    // round over a band of tile rows [band_ty0, band_ty0 + nty_band); halo rows
    // of bands already updated come from their saved boundary rows
    int band_ty0, nty_band;
    const void* shell_lo;  // rows below the band: [x][q][M][nz] copy, or null (read f)
    const void* shell_hi;  // rows above the band, likewise
    int items;             // work items of this launch; the grid may be padded to a multiple of 8
    // bounded hazard wait: polls before giving up (and reporting a time-out),
    // and a bias added to the progress a wait requires (0; a test hook sets an
    // unreachable one so that every wait gives up)
    int spin_limit, need_bias;
    int nt_store;  // 1: the in-place stores of the pair-and-ring march are non-temporal
};

// One merged two-step adjoint pass (out of place).
struct Adj2Args {
    Geom g;
    const void* ft;    // state f_t (storage type)
    const void* F;     // 3N force or null
    const void* lin;   // lambda_{t+2}, 19N of the arithmetic type
    void* lout;        // lambda_t
    void* gF;          // 3N force gradient, accumulated (may be null)
    int nty, ntz, nseg, seg_len;
    int items;         // tiles x segments; the grid is padded to a multiple of 8
};

// Launchers; each returns the hipError_t of its launch.
hipError_t launch_init(int storage, const Geom& g, void* f, const double* rho0, const double* u0, hipStream_t s);
hipError_t launch_two_array(int storage, bool force, const Geom& g, const void* src, void* dst, const void* F,
                            hipStream_t s);
hipError_t launch_copy(int storage, const Geom& g, const void* src, void* dst, hipStream_t s);
hipError_t launch_prepass(int storage, const Geom& g, const MarchPlan& p, const void* f, void* side, int* flags,
                          hipStream_t s);
hipError_t launch_shells(int storage, const Geom& g, const MarchPlan& p, int TY, const void* f, void* shell,
                         hipStream_t s);
hipError_t launch_clear_word(int* w, hipStream_t s);  // w[0] = 0, as a kernel (safe inside a captured graph)

constexpr int SUM_BLOCKS = 1024;  // fixed grid of the reduction: deterministic order
hipError_t launch_macro(int storage, bool force, const Geom& g, const void* f, const void* F, double* rho, double* u,
                        double* unorm, double* partials, double* sums, hipStream_t s);
hipError_t launch_macro_adjoint(int storage, bool force, const Geom& g, const void* f, const void* F,
                                const void* grad_u, void* lambda, void* grad_force, hipStream_t s);
hipError_t launch_step_adjoint(int storage, bool force, int k, const Geom& g, const void* f_t, const void* F,
                               const void* lam_in, void* lam_out, void* grad_force, hipStream_t s);
// measurement probes (k_probe.hip)
hipError_t launch_probe_copy(const void* src, void* dst, long long n16, int blocks, hipStream_t s);
hipError_t launch_probe_pattern(int storage, const Geom& g, const MarchPlan& p, void* f, hipStream_t s);
hipError_t launch_step_adjoint2(int storage, const Geom& g, const void* f_t, const void* F, const void* lam_in,
                                void* lam_out, void* grad_force, hipStream_t s);

}  // namespace lbm
