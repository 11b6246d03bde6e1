/*
 * lbm_cpu.h -- C ABI of liblbm_cpu.so: the paper's own sequential CPU
 * algorithms for the single-copy D3Q19 update, kept beside the GPU library
 * as host context (their relative speeds are what the paper reports on its
 * manycore CPUs; Sec. 5.2).  Fu & Song, "Designing a 3D Parallel
 * Memory-Aware Lattice Boltzmann Algorithm on Manycore Systems":
 *
 *   lbm_cpu_fuse_swap  Sec. 3, Alg. 1: single copy, swap streaming and loop
 *                      fusion; per step, the cells of the bounding box are
 *                      collided and reverted first, the bulk is swept with
 *                      collide + swap_stream, and the bounding box swaps last.
 *   lbm_cpu_two_step   Sec. 4.1, Alg. 2: two collision-streaming steps merged
 *                      per sweep; the second computation of a cell follows the
 *                      first computation of its neighbour one cell further in
 *                      x, y and z, cells on the last row or column of a layer
 *                      take theirs as soon as their dependencies are met, and
 *                      the top layer finishes after the sweep.  With tile > 0
 *                      the sweep follows the prism traversal of stride tile
 *                      (Sec. 4.1, Fig. 3).
 *
 * Both run on one host thread in FP64 and compute the same model as the GPU
 * library (include/lbm.h): D3Q19 with c_1..c_9 the preceding neighbours of a
 * cell in an x-slowest, z-fastest sweep and c_{q+9} = -c_q, BGK with
 * relaxation time tau, halfway bounce-back on wall faces with the moving-face
 * term -6 w_q (c_q . u_w) on every link that crosses it, no body force.
 *
 * Layout     host memory, array of structures as the paper's CPU framework
 *            keeps it: cell (x, y, z) holds its 19 values at
 *            g[((x*ny + y)*nz + z)*19 + q]; the stored value is the offset
 *            g_q = f_q - w_q (FP64).  After any call the array holds the
 *            post-stream state: slot q of a cell holds f_q - w_q.
 * Config     the lbm_config of include/lbm.h; storage, scheme and variant are
 *            ignored; use_force must be 0 and velocities 0 or 19 (D3Q19).
 *            lbm_cpu_two_step needs a wall (or moving wall) on every face, as
 *            the lid-driven cavity of Sec. 5.1 has.
 * Errors     LBM_EINVAL for a bad configuration or a NULL pointer,
 *            LBM_EUNSUPPORTED for what is not built (a body force; periodic
 *            faces in the two-step sweep); nothing aborts.  The array is
 *            owned by the caller; the library allocates only the scratch of
 *            lbm_cpu_two_step's checked mode.
 */
#ifndef LBM_CPU_H
#define LBM_CPU_H

#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* g := equilibrium of (rho0, u0) in the layout above; rho0: N doubles or NULL
 * (rho = 1), u0: 3N doubles (SoA u[c*N + cell]) or NULL (u = 0). */
lbm_status lbm_cpu_init(const lbm_config* cfg, double* g, const double* rho0, const double* u0);

/* n >= 0 steps of Alg. 1 (Sec. 3) in place. */
lbm_status lbm_cpu_fuse_swap(const lbm_config* cfg, double* g, int64_t n);

/* n >= 0 steps as n/2 merged two-step sweeps of Alg. 2 (Sec. 4.1) in place,
 * plus one step of Alg. 1 for an odd n.  tile = 0: lexicographic sweep;
 * tile > 0: prism traversal of that stride.  checked != 0 additionally keeps
 * a state per cell and verifies, before each computation, that every
 * neighbour it swaps with or depends on is in the state the swap algorithm
 * requires (LBM_ESTATE on a violation, the state then being undefined);
 * for tests of the schedule, not for timing. */
lbm_status lbm_cpu_two_step(const lbm_config* cfg, double* g, int64_t n, int32_t tile, int32_t checked);

#ifdef __cplusplus
}
#endif

#endif /* LBM_CPU_H */
