/*
 * lbm.h -- C ABI of liblbm.so, an MI355X (gfx950) implementation of the
 * memory-aware 3D lattice Boltzmann update of Fu & Song, "Designing a 3D
 * Parallel Memory-Aware Lattice Boltzmann Algorithm on Manycore Systems":
 * a fused D3Q19 BGK collide-and-stream done in place on a single copy of the
 * distributions (Sec. 3, Alg. 1), with two collision-streaming steps merged
 * per pass over memory (Sec. 4.1, Alg. 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Lattice   D3Q19.  c_0 = 0; c_1..c_9 = (-1,0,0) (0,-1,0) (0,0,-1) (-1,-1,0)
 *           (-1,1,0) (-1,0,-1) (-1,0,1) (0,-1,-1) (0,-1,1); c_{q+9} = -c_q
 *           (directions 1..9 are the neighbours that precede a cell in an
 *           x-slowest, z-fastest sweep, Sec. 3).  Weights 1/3, 1/18, 1/36.
 *           With lbm_config.velocities, the other two cubic sets (Q values
 *           per cell, c_{q+H} = -c_q, H = (Q-1)/2, c_1..c_H preceding):
 *           D3Q15  c_1..c_7 = (-1,0,0) (0,-1,0) (0,0,-1) (-1,-1,-1) (-1,-1,1)
 *                  (-1,1,-1) (-1,1,1); weights 2/9, 1/9, 1/72 by |c|^2 = 0, 1, 3.
 *           D3Q27  c_1..c_9 as D3Q19, c_10..c_13 = (-1,-1,-1) (-1,-1,1)
 *                  (-1,1,-1) (-1,1,1); weights 8/27, 2/27, 1/54, 1/216.
 * Model     BGK with relaxation time tau (> 1/2); rho = sum f,
 *           u = (sum c f + F/2)/rho; second-order equilibrium; Guo forcing
 *           when a body-force field F is attached; halfway bounce-back on wall
 *           faces, with the momentum term -6 w_q (c_q . u_w) of a moving face
 *           (wall density 1) on every link that crosses it.
 * Step      one collide followed by one stream (Sec. 3).  After any call the
 *           distribution buffer holds the post-stream state of the last step,
 *           in natural layout: slot q of cell x holds f_q(x).
 * Layout    f[q][x][y][z], z fastest: element q*N + (x*ny + y)*nz + z with
 *           N = nx*ny*nz (q < Q, the set's size; 19 unless stated); the
 *           stored value is the offset g = f - w_q, in the
 *           storage type of the configuration.  Vector fields (u, F, their
 *           gradients) are SoA: a[c*N + cell], c = 0 (x), 1 (y), 2 (z).
 * Memory    every pointer named *_dev is device memory owned by the caller
 *           (e.g. a torch tensor) and must stay valid while a context uses
 *           it.  The library never allocates device memory: its scratch
 *           (side planes, progress flags, reduction partials, the second
 *           lattice of the two-array scheme) lives in the caller's work
 *           buffer, sized by lbm_buffer_sizes (lbm_step_static alone uses a
 *           fixed static array instead).  Device pointers must be 256-byte
 *           aligned.
 * Streams   every call is enqueued asynchronously on the context's stream
 *           (a hipStream_t passed as void*; NULL is the legacy default
 *           stream), except lbm_macroscopic with sums_host != NULL, which
 *           waits for its result.  A context is not thread-safe; calls on
 *           contexts that share a work buffer must not overlap.
 * Errors    every entry point returns an lbm_status and never aborts.
 *           Arguments are validated before any device work; on failure the
 *           context keeps a message for lbm_last_error.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,       /* bad argument: tau <= 1/2, dims < 1, null pointer, bad face codes */
    LBM_EUNSUPPORTED = -2, /* valid but not built: e.g. three merged steps for D3Q15/D3Q27 */
    LBM_EDEVICE = -3,      /* a HIP call or kernel launch failed; message kept */
    LBM_ESTATE = -4        /* call on a NULL or failed context */
} lbm_status;

typedef enum {
    LBM_F64 = 0,     /* double storage and double arithmetic */
    LBM_F32 = 1,     /* float storage and float arithmetic */
    LBM_F16_OFS = 2, /* IEEE binary16 storage of f - w (round to nearest even), float arithmetic */
    LBM_BF16_OFS = 3 /* bfloat16 storage of f - w (round to nearest even), float arithmetic */
} lbm_storage;

typedef enum {
    LBM_TWO_ARRAY = 0, /* plain baseline: collide + push-stream into a second lattice (work buffer) */
    LBM_SWAP1 = 1,     /* in place, single copy, one step per pass (Sec. 3, Alg. 1) */
    LBM_SWAP2 = 2,     /* in place, single copy, two steps merged per pass (Sec. 4.1, Alg. 2) */
    LBM_SWAP3 = 3      /* in place, single copy, three steps merged per pass (the deeper merging the
                          conclusion, Sec. 6, names as the next step); FP32 storage only */
} lbm_scheme;

typedef enum { LBM_PERIODIC = 0, LBM_WALL = 1, LBM_MOVING_WALL = 2 } lbm_face;

typedef struct {
    int32_t nx, ny, nz; /* lattice size, x slowest, z fastest; each >= 1; ny*nz < 2^31 and
                           ny*nz*(value size) < 4 GiB (LBM_EUNSUPPORTED otherwise) */
    double tau;         /* BGK relaxation time, > 0.5 */
    int32_t storage;    /* lbm_storage */
    int32_t scheme;     /* lbm_scheme */
    int32_t face[6];    /* -x,+x,-y,+y,-z,+z: lbm_face; both faces of an axis periodic or neither;
                           at most one LBM_MOVING_WALL */
    double wall_u[3];   /* velocity of the moving-wall face (ignored without one) */
    int32_t use_force;  /* 1: a body-force density field F (3N, double for LBM_F64, float otherwise) */
    int32_t variant;    /* 0 = default kernel shape; other values select alternative compiled tile shapes
                           (e.g. D3Q19 FP64: 0 = 10x32 tiles, 1 = 12x28, 2 = 10x32 with loads two planes
                           ahead; D3Q19 32/16-bit: 5 = 16x16 tiles for small lattices, 6 = 12x28 plain
                           tiles); LBM_EUNSUPPORTED for a value with no compiled shape */
    int32_t velocities; /* velocity set: 0 or 19 = D3Q19 (the paper's); 15 = D3Q15, 27 = D3Q27 (Sec. 4.1 names
                           both as sets the two-step rule holds for): every storage (16-bit: the default
                           tiles), LBM_TWO_ARRAY, LBM_SWAP1 and LBM_SWAP2 (large planes in rounds), the adjoint;
                           no probes */
} lbm_config;

/* Bytes the caller must provide for the distribution buffer (Q*N values of
 * the storage type, Q = 19 for D3Q19: the single copy of Sec. 3, which the in-place schemes
 * update without a second lattice) and for the work buffer of this
 * configuration (the saved planes that stand in for the bounding-box stages of
 * Alg. 1 and the slab borders of Sec. 4.2, progress counters, reduction
 * partials; the two-array baseline's second lattice).  Either output may be
 * NULL; returns the status lbm_init would return for the configuration.  In-place schemes march y-z tiles with one workgroup
 * each; a plane with more tiles than the device holds workgroups at once runs
 * in rounds over bands of tile rows, whose boundary rows the work buffer then
 * also holds, with the saved planes of a short last band's own x segments
 * (across a periodic y axis a ragged last tile row then takes the
 * one-column-per-thread layout, with another tile height where the row would
 * be thinner than the halo).  LBM_EUNSUPPORTED, with the reason, where that is
 * not built: rounds across a periodic y axis whose last tile row is thinner
 * than the halo for every tile height built. */
lbm_status lbm_buffer_sizes(const lbm_config* cfg, size_t* f_bytes, size_t* work_bytes);

/* Create a context and set f to the equilibrium of (rho0, u0) (Sec. 5.1: one
 * cavity is built once and every algorithm runs on it).  rho0_dev: N doubles
 * or NULL (rho = 1); u0_dev: 3N doubles (SoA) or NULL (u = 0).  force_dev is
 * required iff cfg->use_force.  On success *out owns a new context (release
 * with lbm_destroy); on failure *out is set to NULL. */
lbm_status lbm_init(const lbm_config* cfg, void* f_dev, void* work_dev, const void* force_dev,
                    const double* rho0_dev, const double* u0_dev, void* hip_stream, lbm_ctx** out);

/* Create a context that adopts the state already in f_dev (resume from a
 * checkpoint: the single copy of the distributions is the whole state of the
 * method, Sec. 3), without initialising it.  Arguments, ownership and errors
 * as for lbm_init. */
lbm_status lbm_attach(const lbm_config* cfg, void* f_dev, void* work_dev, const void* force_dev,
                      void* hip_stream, lbm_ctx** out);

/* Advance n >= 0 time steps (Sec. 3: N steps; Sec. 5.1: N/2 merged passes).
 * LBM_SWAP2 runs n/2 merged passes and, if n is odd, one single-step pass;
 * LBM_SWAP3 runs n/3 three-step passes and one pass of the n%3 remaining steps;
 * LBM_TWO_ARRAY copies the state back into f_dev after an odd number of steps. */
lbm_status lbm_step(lbm_ctx* ctx, int64_t n);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): lbm_step
 * without a context or a work buffer.  Advances the distributions in f_dev
 * (layout and storage of cfg, as lbm_init writes them) by n >= 0 steps in
 * place, on hip_stream and the current device, exactly as lbm_step on a
 * context made from cfg over the same buffers would (same kernels, same
 * results); force_dev as for lbm_init.  Its scratch (progress counters, saved
 * planes, band boundary rows; the second lattice of LBM_TWO_ARRAY) is a
 * static 64 MiB device array that every device the library runs on holds
 * until the process ends; a configuration whose lbm_buffer_sizes work bytes
 * exceed it is rejected with LBM_EUNSUPPORTED (512^3 FP32 LBM_SWAP2 needs
 * 39 MiB).  Every call on a device shares that device's array: calls that
 * overlap on one device (other streams, other threads) race and must not be
 * made.  The array keeps the last call's contents; each call clears what it
 * needs clear.  No device or host memory is allocated on the way to the
 * kernels (a failure's message is kept in host memory).  Asynchronous,
 * unless timed_out_host is not NULL: it then waits for the passes and
 * stores 1 if a hazard wait of this call gave up (the state is then not to
 * be trusted), 0 otherwise.  Errors as for lbm_init, message from
 * lbm_last_error(NULL). */
lbm_status lbm_step_static(const lbm_config* cfg, void* f_dev, const void* force_dev, int64_t n, void* hip_stream,
                           int32_t* timed_out_host);

/* Advance k in {1, 2} steps from the state f_src into f_dst, out of place:
 * f_src is read only and the context's own distribution buffer is neither
 * read nor changed.  Both buffers have the size and layout of f (Q*N values
 * of the storage type), must not overlap and must be 256-byte aligned.  With
 * LBM_SWAP2 and k = 2 this is one merged pass, the same kernel and the same
 * bytes moved as an in-place pass (no side planes or progress counters are
 * needed: nothing is overwritten that is still to be read).  Used by the
 * adjoint's recomputation of the states of a checkpoint interval, which
 * then needs no copies. */
lbm_status lbm_step_into(lbm_ctx* ctx, const void* f_src, void* f_dst, int32_t k);

/* Per-cell density, velocity u = (sum c f + F/2)/rho and velocity norm |u|
 * (the quantity compared across algorithms in Sec. 5.1), all as doubles
 * computed in double from the stored state.  rho_dev: N, u_dev: 3N (SoA),
 * unorm_dev: N; each may be NULL.  If sums_host is not NULL it receives
 * { sum rho, sum_q c_x f, sum_q c_y f, sum_q c_z f } over all cells (the
 * populations' mass and momentum, accumulated in double on the device in a
 * fixed order), and the call waits for them.  That call also reports
 * LBM_EDEVICE if any in-place pass of this context so far gave up waiting
 * for a neighbouring workgroup (a bounded wait; the state is then not to be
 * trusted, and the report stays set for the life of the context). */
lbm_status lbm_macroscopic(lbm_ctx* ctx, double* rho_dev, double* u_dev, double* unorm_dev, double* sums_host);

/* Discrete adjoint, seed: given dL/du of the velocity field of the state
 * f_dev (grad_u_dev: 3N of the arithmetic type), write lambda = dL/df
 * (lambda_dev: 19N of the arithmetic type, not offset) and add the direct
 * dL/dF = dL/du / (2 rho) to grad_force_dev (3N; may be NULL without a force).
 * Every storage (16-bit states are decoded; lambda and gradients are FP32)
 * and every velocity set (lambda_dev: Q N values). */
lbm_status lbm_macro_adjoint(lbm_ctx* ctx, const void* f_dev, const void* grad_u_dev, void* lambda_dev,
                             void* grad_force_dev);

/* Discrete adjoint of k in {1, 2} forward steps taken from the state f_t_dev
 * (storage type and layout of f, left unchanged): lambda_in_dev holds
 * dL/df_{t+k}; lambda_out_dev receives dL/df_t (non-overlapping buffers, 19N
 * of the arithmetic type; every buffer 256-byte aligned, LBM_EINVAL
 * otherwise); grad_force_dev (3N) accumulates the force gradient of the
 * k steps (required with a force, may be NULL without).  The reverse of the
 * step of Sec. 3: the transposed stream gathers lambda_q from the link's
 * target (the own lambda of the opposite direction on a wall link), then the
 * transposed collision acts per cell.  With k = 2 the state f_{t+1} is
 * recomputed on chip, so one call reads f_t once: the adjoint of the two-step
 * merged pass of Sec. 4.1 (132 bytes per lattice update at FP32).  Every
 * storage: with FP16/BF16 the state is decoded and the adjoint computes in
 * FP32, the adjoint of the FP32 arithmetic between 16-bit stores (rounding
 * has no useful derivative).  Every velocity set (lambda buffers of Q N
 * values). */
lbm_status lbm_step_adjoint(lbm_ctx* ctx, const void* f_t_dev, const void* lambda_in_dev, void* lambda_out_dev,
                            void* grad_force_dev, int32_t k);

/* Measurement hook.  While enabled, every launch of the lattice-update kernel
 * itself (the marching kernel of LBM_SWAP1/LBM_SWAP2 without its prepass, or
 * the two-array kernel) is bracketed by a pair of HIP events recorded on the
 * context's stream.  lbm_kernel_time waits for the recorded launches and
 * returns their summed duration in milliseconds and their count, split by the
 * number of steps each launch merged (index 0: one step, 1: two steps, 2:
 * three steps; total_ms and launches point to arrays of 3), then forgets them.  Events are
 * host-side objects owned by the context; no device memory is allocated. */
lbm_status lbm_set_kernel_timing(lbm_ctx* ctx, int32_t enable);
lbm_status lbm_kernel_time(lbm_ctx* ctx, double* total_ms, int64_t* launches);

/* Measurement probes: they compute nothing of the method and bound what the
 * marching kernel can reach on the device's memory (the roofline argument of
 * the measurement).  Asynchronous on hip_stream; errors as for lbm_init, with
 * the message from lbm_last_error(NULL).
 *
 * lbm_probe_copy: copy `bytes` (a multiple of 16) from src_dev to dst_dev
 * (non-overlapping, 256-byte aligned) with 16-byte loads and stores per lane,
 * one launch of `blocks` workgroups of 512 threads (256: the marching
 * kernel's grid on this device).
 *
 * lbm_probe_pattern: the access pattern of one marching pass of
 * steps_per_pass (1 or 2) steps of cfg over f_dev (19N values of the 32- or
 * 16-bit storage, even nz, one round of 16 x 64 tiles: LBM_EUNSUPPORTED
 * otherwise): the same work items and pair layout, 19 pair loads of each
 * plane and 19 pair stores, in place, steps_per_pass planes behind, without
 * halo, LDS exchange, compute or hazard checks.  It stores back what it
 * loaded, so f_dev is unchanged. */
lbm_status lbm_probe_copy(const void* src_dev, void* dst_dev, size_t bytes, int32_t blocks, void* hip_stream);
lbm_status lbm_probe_pattern(const lbm_config* cfg, void* f_dev, int32_t steps_per_pass, void* hip_stream);

/* Test hook for the failure path of the in-place hazard wait: with enable != 0
 * every wait of later in-place passes requires progress no neighbour can
 * reach and gives up after a few polls, as if a neighbouring workgroup had
 * stalled.  The passes still run to the end with every access in bounds, but
 * their results are not to be trusted, and lbm_macroscopic with sums reports
 * the time-out (LBM_EDEVICE) from then on.  Not for production use. */
lbm_status lbm_test_force_wait_timeout(lbm_ctx* ctx, int32_t enable);

/* Rebind the context to another stream (a hipStream_t as void*). */
lbm_status lbm_set_stream(lbm_ctx* ctx, void* hip_stream);

/* Message of the last failed call on ctx (or, when ctx is NULL, of this
 * thread's last failed call that takes no context: lbm_init, lbm_attach,
 * lbm_step_static, the probes); "" if none.  Valid until the next call. */
const char* lbm_last_error(const lbm_ctx* ctx);

/* Release a context; NULL is allowed.  Device buffers stay the caller's. */
void lbm_destroy(lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
