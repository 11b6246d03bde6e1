// lbm_api.cpp -- the C ABI declared in include/lbm.h: argument validation,
// work-buffer layout, pass planning and kernel dispatch.  All device memory
// belongs to the caller; this file never allocates any.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_internal.hpp"
#include "march_plan.hpp"

using namespace lbm;

// Scratch of lbm_step_static, the entry point for callers that cannot
// allocate device memory: one copy on every device the library runs on,
// loaded with the library and held until the process ends.  Host code uses
// the per-device address from hipGetSymbolAddress (static_scratch below),
// never the array's name, which is only a host-side stand-in.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

struct lbm_ctx {
    lbm_config cfg;
    Geom g;
    void* f = nullptr;
    unsigned char* work = nullptr;
    const void* force = nullptr;
    hipStream_t stream = nullptr;
    std::string err;
    MarchPlan plan[4];  // indexed by M
    size_t off_partials = 0, off_sums = 0, off_second = 0, off_flags = 0, off_side = 0, off_shell = 0;
    bool force_wait_timeout = false;  // test hook: every hazard wait gives up
    // measurement hook: event pairs around update-kernel launches
    bool timing = false;
    std::vector<hipEvent_t> ev;  // 2 per recorded launch, reused
    std::vector<int> ev_steps;   // steps merged by each recorded launch
    size_t ev_used = 0;
    ~lbm_ctx()
    {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

namespace {

thread_local std::string g_create_err;

lbm_status validate(const lbm_config* c, std::string* why)
{
    if (!c) return fail(why, LBM_EINVAL, "config is NULL");
    if (c->nx < 1 || c->ny < 1 || c->nz < 1) return fail(why, LBM_EINVAL, "lattice dimensions must be >= 1");
    if ((long long)c->ny * (long long)c->nz >= (1LL << 31))
        return fail(why, LBM_EINVAL, "ny*nz must be below 2^31");
    if (!(c->tau > 0.5) || !isfinite(c->tau)) return fail(why, LBM_EINVAL, "tau must be a finite number > 0.5");
    if (c->storage < LBM_F64 || c->storage > LBM_BF16_OFS) return fail(why, LBM_EINVAL, "unknown storage type");
    // the kernels address a cell within one direction's y-z plane by a 32-bit byte offset
    if ((unsigned long long)c->ny * (unsigned long long)c->nz * elem_size(c->storage) >= (1ULL << 32))
        return fail(why, LBM_EUNSUPPORTED, "one direction's y-z plane must hold less than 4 GiB (ny*nz*value size)");
    if (c->scheme < LBM_TWO_ARRAY || c->scheme > LBM_SWAP3) return fail(why, LBM_EINVAL, "unknown scheme");
    if (c->use_force != 0 && c->use_force != 1) return fail(why, LBM_EINVAL, "use_force must be 0 or 1");
    int moving = 0;
    for (int a = 0; a < 3; ++a) {
        const int lo = c->face[2 * a], hi = c->face[2 * a + 1];
        if (lo < LBM_PERIODIC || lo > LBM_MOVING_WALL || hi < LBM_PERIODIC || hi > LBM_MOVING_WALL)
            return fail(why, LBM_EINVAL, "unknown face code");
        if ((lo == LBM_PERIODIC) != (hi == LBM_PERIODIC))
            return fail(why, LBM_EINVAL, "both faces of an axis must be periodic, or neither");
        moving += (lo == LBM_MOVING_WALL) + (hi == LBM_MOVING_WALL);
    }
    if (moving > 1) return fail(why, LBM_EINVAL, "at most one moving-wall face");
    for (int a = 0; a < 3; ++a)
        if (!isfinite(c->wall_u[a])) return fail(why, LBM_EINVAL, "wall velocity must be finite");
    if (c->variant < 0) return fail(why, LBM_EINVAL, "variant must be >= 0");
    if (c->velocities != 0 && c->velocities != 15 && c->velocities != 19 && c->velocities != 27)
        return fail(why, LBM_EINVAL, "velocities must be 0 (D3Q19), 15, 19 or 27");
    if (lat_of(*c) != 19 && c->scheme == LBM_SWAP3)
        return fail(why, LBM_EUNSUPPORTED, "three merged steps are built for D3Q19 only");
    return LBM_OK;
}

bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) % kAlign) == 0; }

lbm_status device_err(lbm_ctx* ctx, hipError_t e, const char* what)
{
    if (e == hipSuccess) return LBM_OK;
    ctx->err = std::string(what) + ": " + hipGetErrorString(e);
    return LBM_EDEVICE;
}

// Fills a context for cfg over the given buffers: geometry, pass plans for
// the device's co-residency and the work-buffer offsets.  work_cap: bytes
// available at work_dev (checked against the layout), or 0 when the caller
// sized the buffer with lbm_buffer_sizes.
lbm_status setup(lbm_ctx* ctx, const lbm_config* cfg, void* f_dev, void* work_dev, const void* force_dev, void* stream,
                 size_t work_cap, std::string* why)
{
    lbm_status st = validate(cfg, why);
    if (st != LBM_OK) return st;
    if (!f_dev || !work_dev) return fail(why, LBM_EINVAL, "f_dev and work_dev are required");
    if (!aligned(f_dev) || !aligned(work_dev)) return fail(why, LBM_EINVAL, "device buffers must be 256-byte aligned");
    if (cfg->use_force && !force_dev) return fail(why, LBM_EINVAL, "use_force needs force_dev");
    if (force_dev && !aligned(force_dev)) return fail(why, LBM_EINVAL, "force_dev must be 256-byte aligned");
    ctx->cfg = *cfg;
    ctx->f = f_dev;
    ctx->work = static_cast<unsigned char*>(work_dev);
    ctx->force = cfg->use_force ? force_dev : nullptr;
    ctx->stream = static_cast<hipStream_t>(stream);
    Geom& g = ctx->g;
    g.nx = cfg->nx;
    g.ny = cfg->ny;
    g.nz = cfg->nz;
    g.N = (long long)cfg->nx * cfg->ny * cfg->nz;
    g.PL = (long long)cfg->ny * cfg->nz;
    g.moving_face = -1;
    for (int a = 0; a < 3; ++a) {
        g.wall[a] = cfg->face[2 * a] != LBM_PERIODIC;
        g.uw[a] = cfg->wall_u[a];
    }
    for (int fc = 0; fc < 6; ++fc)
        if (cfg->face[fc] == LBM_MOVING_WALL) g.moving_face = fc;
    g.omega = 1.0 / cfg->tau;
    g.lat = lat_of(*cfg);

    size_t off[6], total = 0, sized = 0;
    int cap = kMaxResident;
    MarchPlan probe[4];
    st = layout(*cfg, cap, probe, off, &sized, why);  // what lbm_buffer_sizes reported
    if (st != LBM_OK) return st;
    if (work_cap && sized > work_cap) {
        char msg[160];
        snprintf(msg, sizeof msg, "this configuration needs %zu bytes of scratch, more than the %zu available", sized,
                 work_cap);
        return fail(why, LBM_EUNSUPPORTED, msg);
    }
    if (cfg->scheme != LBM_TWO_ARRAY) {
        // the device may hold fewer marching workgroups than the sizing bound
        for (int M = 1; M <= 3; ++M) {
            if (probe[M].M == 0) continue;
            const int dc = device_cap(*cfg, probe[M]);
            if (dc <= 0) return fail(why, LBM_EDEVICE, "cannot query the co-residency of the marching kernel");
            if (dc < cap) cap = dc;
        }
    }
    st = layout(*cfg, cap, ctx->plan, off, &total, why);
    if (st != LBM_OK) return st;
    if (total > sized && cap < kMaxResident) {
        // a smaller cap can leave a short last band whose own x segments need
        // more side planes than the size reported: run it in the others'
        st = layout(*cfg, cap, ctx->plan, off, &total, why, false);
        if (st != LBM_OK) return st;
    }
    if (total > sized)
        return fail(why, LBM_EUNSUPPORTED,
                    "this device holds fewer co-resident marching workgroups than the work-buffer size assumed");
    ctx->off_partials = off[0];
    ctx->off_sums = off[1];
    ctx->off_second = off[2];
    ctx->off_flags = off[3];
    ctx->off_side = off[4];
    ctx->off_shell = off[5];
    return LBM_OK;
}

lbm_status create(const lbm_config* cfg, void* f_dev, void* work_dev, const void* force_dev, void* stream,
                  lbm_ctx** out)
{
    if (out) *out = nullptr;
    g_create_err.clear();
    if (!out) return fail(&g_create_err, LBM_EINVAL, "out is NULL");
    lbm_status st = validate(cfg, &g_create_err);
    if (st != LBM_OK) return st;
    lbm_ctx* ctx = new (std::nothrow) lbm_ctx();
    if (!ctx) return fail(&g_create_err, LBM_EDEVICE, "out of host memory");
    st = setup(ctx, cfg, f_dev, work_dev, force_dev, stream, 0, &g_create_err);
    if (st != LBM_OK) {
        delete ctx;
        return st;
    }
    if (cfg->scheme != LBM_TWO_ARRAY) {
        // the timeout report of the in-place passes starts clear (the work
        // buffer arrives uninitialised) and is never cleared by a pass
        st = device_err(ctx, launch_clear_word(reinterpret_cast<int*>(ctx->work + ctx->off_flags), ctx->stream),
                        "timeout word clear");
        if (st != LBM_OK) {
            g_create_err = ctx->err;
            delete ctx;
            return st;
        }
    }
    *out = ctx;
    return LBM_OK;
}

lbm_status check_ctx(const lbm_ctx* ctx) { return ctx ? LBM_OK : LBM_ESTATE; }

// records the first event of a launch pair; returns its index or -1
long timing_begin(lbm_ctx* ctx, int steps)
{
    if (!ctx->timing) return -1;
    if (ctx->ev_used + 2 > ctx->ev.size()) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess) return -1;
        if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            return -1;
        }
        ctx->ev.push_back(a);
        ctx->ev.push_back(b);
    }
    const long idx = long(ctx->ev_used);
    if (hipEventRecord(ctx->ev[idx], ctx->stream) != hipSuccess) return -1;
    ctx->ev_used += 2;
    ctx->ev_steps.resize(ctx->ev_used / 2);
    ctx->ev_steps[idx / 2] = steps;
    return idx;
}

void timing_end(lbm_ctx* ctx, long idx)
{
    if (idx >= 0) (void)hipEventRecord(ctx->ev[idx + 1], ctx->stream);
}

// One marching pass of M steps from src into dst (dst == src: in place).
lbm_status march_pass(lbm_ctx* ctx, int M, const void* src, void* dst)
{
    const MarchPlan& p = ctx->plan[M];
    int* flags = reinterpret_cast<int*>(ctx->work + ctx->off_flags);
    void* side = ctx->work + ctx->off_side;
    const bool inplace = src == dst;
    unsigned char* shell = ctx->work + ctx->off_shell;
    if (inplace) {
        lbm_status st = device_err(ctx, launch_prepass(ctx->cfg.storage, ctx->g, p, src, side, flags, ctx->stream),
                                   "prepass launch");
        if (st != LBM_OK) return st;
        if (p.nseg_last > 0) {
            // the side planes of the last band's own segments (and its counters)
            MarchPlan pl = p;
            pl.nseg = p.nseg_last;
            pl.seg_len = p.seg_len_last;
            st = device_err(ctx,
                            launch_prepass(ctx->cfg.storage, ctx->g, pl, src,
                                           static_cast<unsigned char*>(side) + p.side_off_last, flags, ctx->stream),
                            "prepass launch");
            if (st != LBM_OK) return st;
        }
        if (p.nbands > 1) {
            st = device_err(ctx, launch_shells(ctx->cfg.storage, ctx->g, p, p.TY, src, shell, ctx->stream),
                            "band boundary copy launch");
            if (st != LBM_OK) return st;
        }
    }
    PassBuffers b;
    b.src = src;
    b.dst = dst;
    b.side = side;
    b.flags = flags;
    b.shell = shell;
    b.force = ctx->force;
    const long tix = timing_begin(ctx, M);
    const hipError_t e = launch_march_pass(ctx->cfg, ctx->g, p, b, ctx->force_wait_timeout, ctx->stream);
    timing_end(ctx, tix);
    return device_err(ctx, e, "marching kernel launch");
}

// Device address of this device's copy of the static scratch, looked up once
// per device with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices];

lbm_status static_scratch(void** out, std::string* why)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(why, LBM_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(why, LBM_EUNSUPPORTED, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(why, LBM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return LBM_OK;
}

// n > 0 steps on a prepared context (the body of lbm_step)
lbm_status step_n(lbm_ctx* ctx, int64_t n)
{
    lbm_status st = LBM_OK;
    switch (ctx->cfg.scheme) {
    case LBM_TWO_ARRAY: {
        void* second = ctx->work + ctx->off_second;
        for (int64_t k = 0; k < n && st == LBM_OK; ++k) {
            const void* src = (k & 1) ? second : ctx->f;
            void* dst = (k & 1) ? ctx->f : second;
            const long tix = timing_begin(ctx, 1);
            st = device_err(ctx,
                            launch_two_array(ctx->cfg.storage, ctx->force != nullptr, ctx->g, src, dst, ctx->force,
                                             ctx->stream),
                            "two-array step launch");
            timing_end(ctx, tix);
        }
        if (st == LBM_OK && (n & 1))
            st = device_err(ctx, launch_copy(ctx->cfg.storage, ctx->g, second, ctx->f, ctx->stream), "state copy");
        break;
    }
    case LBM_SWAP1:
        for (int64_t k = 0; k < n && st == LBM_OK; ++k) st = march_pass(ctx, 1, ctx->f, ctx->f);
        break;
    case LBM_SWAP2:
        for (int64_t k = 0; k < n / 2 && st == LBM_OK; ++k) st = march_pass(ctx, 2, ctx->f, ctx->f);
        if (st == LBM_OK && (n & 1)) st = march_pass(ctx, 1, ctx->f, ctx->f);
        break;
    default:
        for (int64_t k = 0; k < n / 3 && st == LBM_OK; ++k) st = march_pass(ctx, 3, ctx->f, ctx->f);
        if (st == LBM_OK && n % 3) st = march_pass(ctx, int(n % 3), ctx->f, ctx->f);
        break;
    }
    return st;
}

}  // namespace

extern "C" {

lbm_status lbm_buffer_sizes(const lbm_config* cfg, size_t* f_bytes, size_t* work_bytes)
{
    std::string why;
    lbm_status st = validate(cfg, &why);
    if (st != LBM_OK) return st;
    MarchPlan plans[4];
    size_t off[6], total = 0;
    st = layout(*cfg, kMaxResident, plans, off, &total, &why);
    if (st != LBM_OK) return st;
    if (f_bytes)
        *f_bytes = size_t(lat_of(*cfg)) * size_t(cfg->nx) * size_t(cfg->ny) * size_t(cfg->nz) * elem_size(cfg->storage);
    if (work_bytes) *work_bytes = total;
    return LBM_OK;
}

lbm_status lbm_init(const lbm_config* cfg, void* f_dev, void* work_dev, const void* force_dev, const double* rho0_dev,
                    const double* u0_dev, void* hip_stream, lbm_ctx** out)
{
    if ((rho0_dev && !aligned(rho0_dev)) || (u0_dev && !aligned(u0_dev))) {
        if (out) *out = nullptr;
        g_create_err = "rho0_dev and u0_dev must be 256-byte aligned";
        return LBM_EINVAL;
    }
    lbm_status st = create(cfg, f_dev, work_dev, force_dev, hip_stream, out);
    if (st != LBM_OK) return st;
    lbm_ctx* ctx = *out;
    st = device_err(ctx, launch_init(cfg->storage, ctx->g, ctx->f, rho0_dev, u0_dev, ctx->stream), "init launch");
    if (st != LBM_OK) {
        g_create_err = ctx->err;
        delete ctx;
        *out = nullptr;
    }
    return st;
}

lbm_status lbm_attach(const lbm_config* cfg, void* f_dev, void* work_dev, const void* force_dev, void* hip_stream,
                      lbm_ctx** out)
{
    return create(cfg, f_dev, work_dev, force_dev, hip_stream, out);
}

lbm_status lbm_step(lbm_ctx* ctx, int64_t n)
{
    if (check_ctx(ctx) != LBM_OK) return LBM_ESTATE;
    ctx->err.clear();
    if (n < 0) return fail(&ctx->err, LBM_EINVAL, "n must be >= 0");
    if (n == 0) return LBM_OK;
    return step_n(ctx, n);
}

lbm_status lbm_step_static(const lbm_config* cfg, void* f_dev, const void* force_dev, int64_t n, void* hip_stream,
                           int32_t* timed_out_host)
{
    g_create_err.clear();
    if (timed_out_host) *timed_out_host = 0;
    lbm_status st = validate(cfg, &g_create_err);
    if (st != LBM_OK) return st;
    if (n < 0) return fail(&g_create_err, LBM_EINVAL, "n must be >= 0");
    void* work = nullptr;
    st = static_scratch(&work, &g_create_err);
    if (st != LBM_OK) return st;
    lbm_ctx ctx;  // on the stack: no allocation on the way to the kernels
    st = setup(&ctx, cfg, f_dev, work, force_dev, hip_stream, kStaticScratchBytes, &g_create_err);
    if (st != LBM_OK) return st;
    if (n == 0) return LBM_OK;
    int* word = reinterpret_cast<int*>(ctx.work + ctx.off_flags);
    if (cfg->scheme != LBM_TWO_ARRAY) {
        // the scratch keeps the previous call's contents: the time-out report
        // starts clear for this call (progress counters and saved planes are
        // rewritten by every pass before they are read)
        st = device_err(&ctx, launch_clear_word(word, ctx.stream), "timeout word clear");
        if (st == LBM_OK) st = step_n(&ctx, n);
        if (st == LBM_OK && timed_out_host) {
            int t = 0;
            st = device_err(&ctx, hipMemcpyAsync(&t, word, sizeof(int), hipMemcpyDeviceToHost, ctx.stream),
                            "progress-word copy");
            if (st == LBM_OK) st = device_err(&ctx, hipStreamSynchronize(ctx.stream), "stream synchronize");
            if (st == LBM_OK) *timed_out_host = t != 0;
        }
    } else {
        st = step_n(&ctx, n);
    }
    if (st != LBM_OK) g_create_err = ctx.err;
    return st;
}

lbm_status lbm_step_into(lbm_ctx* ctx, const void* f_src, void* f_dst, int32_t k)
{
    if (check_ctx(ctx) != LBM_OK) return LBM_ESTATE;
    ctx->err.clear();
    if (k != 1 && k != 2) return fail(&ctx->err, LBM_EINVAL, "k must be 1 or 2");
    if (!f_src || !f_dst) return fail(&ctx->err, LBM_EINVAL, "f_src and f_dst are required");
    if (f_src == f_dst) return fail(&ctx->err, LBM_EINVAL, "f_src and f_dst must differ (lbm_step updates in place)");
    if (!aligned(f_src) || !aligned(f_dst)) return fail(&ctx->err, LBM_EINVAL, "buffers must be 256-byte aligned");
    const size_t bytes = size_t(ctx->g.lat) * size_t(ctx->g.N) * elem_size(ctx->cfg.storage);
    const char* a0 = static_cast<const char*>(f_src);
    const char* b0 = static_cast<const char*>(f_dst);
    if (a0 < b0 + bytes && b0 < a0 + bytes) return fail(&ctx->err, LBM_EINVAL, "f_src and f_dst overlap");
    switch (ctx->cfg.scheme) {
    case LBM_TWO_ARRAY: {
        void* second = ctx->work + ctx->off_second;
        const bool force = ctx->force != nullptr;
        if (k == 1)
            return device_err(ctx, launch_two_array(ctx->cfg.storage, force, ctx->g, f_src, f_dst, ctx->force, ctx->stream),
                              "two-array step launch");
        lbm_status st = device_err(
            ctx, launch_two_array(ctx->cfg.storage, force, ctx->g, f_src, second, ctx->force, ctx->stream),
            "two-array step launch");
        if (st != LBM_OK) return st;
        return device_err(ctx, launch_two_array(ctx->cfg.storage, force, ctx->g, second, f_dst, ctx->force, ctx->stream),
                          "two-array step launch");
    }
    case LBM_SWAP1: {
        lbm_status st = march_pass(ctx, 1, f_src, f_dst);
        if (st == LBM_OK && k == 2) st = march_pass(ctx, 1, f_dst, f_dst);
        return st;
    }
    default:
        return march_pass(ctx, k, f_src, f_dst);
    }
}

lbm_status lbm_macroscopic(lbm_ctx* ctx, double* rho_dev, double* u_dev, double* unorm_dev, double* sums_host)
{
    if (check_ctx(ctx) != LBM_OK) return LBM_ESTATE;
    ctx->err.clear();
    if ((rho_dev && !aligned(rho_dev)) || (u_dev && !aligned(u_dev)) || (unorm_dev && !aligned(unorm_dev)))
        return fail(&ctx->err, LBM_EINVAL, "output buffers must be 256-byte aligned");
    double* partials = reinterpret_cast<double*>(ctx->work + ctx->off_partials);
    double* sums = reinterpret_cast<double*>(ctx->work + ctx->off_sums);
    lbm_status st = device_err(ctx,
                               launch_macro(ctx->cfg.storage, ctx->force != nullptr, ctx->g, ctx->f, ctx->force,
                                            rho_dev, u_dev, unorm_dev, partials, sums_host ? sums : nullptr,
                                            ctx->stream),
                               "macroscopic launch");
    if (st != LBM_OK || !sums_host) return st;
    st = device_err(ctx, hipMemcpyAsync(sums_host, sums, 4 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream),
                    "sums copy");
    int timeout = 0;
    if (st == LBM_OK && ctx->cfg.scheme != LBM_TWO_ARRAY)
        st = device_err(ctx,
                        hipMemcpyAsync(&timeout, ctx->work + ctx->off_flags, sizeof(int), hipMemcpyDeviceToHost,
                                       ctx->stream),
                        "progress-word copy");
    if (st == LBM_OK) st = device_err(ctx, hipStreamSynchronize(ctx->stream), "stream synchronize");
    if (st == LBM_OK && timeout)
        return fail(&ctx->err, LBM_EDEVICE, "a marching pass timed out waiting for a neighbouring workgroup");
    return st;
}

lbm_status lbm_macro_adjoint(lbm_ctx* ctx, const void* f_dev, const void* grad_u_dev, void* lambda_dev,
                             void* grad_force_dev)
{
    if (check_ctx(ctx) != LBM_OK) return LBM_ESTATE;
    ctx->err.clear();
    if (!f_dev || !grad_u_dev || !lambda_dev) return fail(&ctx->err, LBM_EINVAL, "f, grad_u and lambda are required");
    if (ctx->force && !grad_force_dev) return fail(&ctx->err, LBM_EINVAL, "grad_force is required with a force");
    return device_err(ctx,
                      launch_macro_adjoint(ctx->cfg.storage, ctx->force != nullptr, ctx->g, f_dev, ctx->force,
                                           grad_u_dev, lambda_dev, grad_force_dev, ctx->stream),
                      "adjoint seed launch");
}

lbm_status lbm_step_adjoint(lbm_ctx* ctx, const void* f_t_dev, const void* lambda_in_dev, void* lambda_out_dev,
                            void* grad_force_dev, int32_t k)
{
    if (check_ctx(ctx) != LBM_OK) return LBM_ESTATE;
    ctx->err.clear();
    if (k != 1 && k != 2) return fail(&ctx->err, LBM_EINVAL, "k must be 1 or 2");
    if (!f_t_dev || !lambda_in_dev || !lambda_out_dev)
        return fail(&ctx->err, LBM_EINVAL, "f_t, lambda_in and lambda_out are required");
    if (ctx->force && !grad_force_dev) return fail(&ctx->err, LBM_EINVAL, "grad_force is required with a force");
    if (!aligned(f_t_dev) || !aligned(lambda_in_dev) || !aligned(lambda_out_dev) ||
        (grad_force_dev && !aligned(grad_force_dev)))
        return fail(&ctx->err, LBM_EINVAL, "device buffers must be 256-byte aligned");
    // lambda_out is written while lambda_in is still read by other workgroups
    const size_t lam_bytes = size_t(ctx->g.lat) * size_t(ctx->g.N) * real_size(ctx->cfg.storage);
    const char* li = static_cast<const char*>(lambda_in_dev);
    const char* lo = static_cast<const char*>(lambda_out_dev);
    if (li < lo + lam_bytes && lo < li + lam_bytes)
        return fail(&ctx->err, LBM_EINVAL, "lambda_in and lambda_out must not overlap");
    return device_err(ctx,
                      launch_step_adjoint(ctx->cfg.storage, ctx->force != nullptr, k, ctx->g, f_t_dev, ctx->force,
                                          lambda_in_dev, lambda_out_dev, grad_force_dev, ctx->stream),
                      "adjoint step launch");
}

lbm_status lbm_probe_copy(const void* src_dev, void* dst_dev, size_t bytes, int32_t blocks, void* hip_stream)
{
    g_create_err.clear();
    if (!src_dev || !dst_dev) return fail(&g_create_err, LBM_EINVAL, "src_dev and dst_dev are required");
    if (!aligned(src_dev) || !aligned(dst_dev))
        return fail(&g_create_err, LBM_EINVAL, "device buffers must be 256-byte aligned");
    if (bytes % 16 != 0) return fail(&g_create_err, LBM_EINVAL, "bytes must be a multiple of 16");
    if (blocks < 1 || blocks > (1 << 20)) return fail(&g_create_err, LBM_EINVAL, "blocks must be in [1, 2^20]");
    const char* a0 = static_cast<const char*>(src_dev);
    const char* b0 = static_cast<const char*>(dst_dev);
    if (a0 < b0 + bytes && b0 < a0 + bytes) return fail(&g_create_err, LBM_EINVAL, "src and dst overlap");
    const hipError_t e = launch_probe_copy(src_dev, dst_dev, (long long)(bytes / 16), blocks,
                                           static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(&g_create_err, LBM_EDEVICE, std::string("copy probe: ") + hipGetErrorString(e));
    return LBM_OK;
}

lbm_status lbm_probe_pattern(const lbm_config* cfg, void* f_dev, int32_t steps_per_pass, void* hip_stream)
{
    g_create_err.clear();
    lbm_status st = validate(cfg, &g_create_err);
    if (st != LBM_OK) return st;
    if (!f_dev || !aligned(f_dev)) return fail(&g_create_err, LBM_EINVAL, "f_dev must be a 256-byte aligned buffer");
    if (steps_per_pass != 1 && steps_per_pass != 2)
        return fail(&g_create_err, LBM_EINVAL, "steps_per_pass must be 1 or 2");
    if (cfg->storage == LBM_F64 || cfg->nz % 2 != 0 || cfg->variant != 0 || lat_of(*cfg) != 19)
        return fail(&g_create_err, LBM_EUNSUPPORTED,
                    "the pattern probe replicates the pair layout: 32- or 16-bit storage, even nz, variant 0");
    MarchPlan p;
    st = make_plan(*cfg, steps_per_pass, kMaxResident, &p, &g_create_err);
    if (st != LBM_OK) return st;
    if (!p.pr || p.TY != 16 || p.TZ != 64 || p.nbands != 1)
        return fail(&g_create_err, LBM_EUNSUPPORTED, "the pattern probe is built for one round of 16x64 tiles");
    Geom g{};
    g.nx = cfg->nx;
    g.ny = cfg->ny;
    g.nz = cfg->nz;
    g.N = (long long)cfg->nx * cfg->ny * cfg->nz;
    g.PL = (long long)cfg->ny * cfg->nz;
    g.lat = 19;
    const hipError_t e = launch_probe_pattern(cfg->storage, g, p, f_dev, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess)
        return fail(&g_create_err, LBM_EDEVICE, std::string("pattern probe: ") + hipGetErrorString(e));
    return LBM_OK;
}

lbm_status lbm_set_kernel_timing(lbm_ctx* ctx, int32_t enable)
{
    if (check_ctx(ctx) != LBM_OK) return LBM_ESTATE;
    ctx->timing = enable != 0;
    ctx->ev_used = 0;
    ctx->ev_steps.clear();
    return LBM_OK;
}

lbm_status lbm_kernel_time(lbm_ctx* ctx, double* total_ms, int64_t* launches)
{
    if (check_ctx(ctx) != LBM_OK) return LBM_ESTATE;
    ctx->err.clear();
    if (!total_ms || !launches) return fail(&ctx->err, LBM_EINVAL, "total_ms and launches are required");
    total_ms[0] = total_ms[1] = total_ms[2] = 0.0;
    launches[0] = launches[1] = launches[2] = 0;
    if (ctx->ev_used) {
        lbm_status st = device_err(ctx, hipEventSynchronize(ctx->ev[ctx->ev_used - 1]), "event synchronize");
        if (st != LBM_OK) return st;
    }
    for (size_t i = 0; i + 1 < ctx->ev_used; i += 2) {
        float ms = 0.0f;
        lbm_status st = device_err(ctx, hipEventElapsedTime(&ms, ctx->ev[i], ctx->ev[i + 1]), "event elapsed time");
        if (st != LBM_OK) return st;
        const int k = ctx->ev_steps[i / 2] - 1;
        total_ms[k] += ms;
        launches[k] += 1;
    }
    ctx->ev_used = 0;
    ctx->ev_steps.clear();
    return LBM_OK;
}

lbm_status lbm_test_force_wait_timeout(lbm_ctx* ctx, int32_t enable)
{
    if (check_ctx(ctx) != LBM_OK) return LBM_ESTATE;
    ctx->force_wait_timeout = enable != 0;
    return LBM_OK;
}

lbm_status lbm_set_stream(lbm_ctx* ctx, void* hip_stream)
{
    if (check_ctx(ctx) != LBM_OK) return LBM_ESTATE;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return LBM_OK;
}

const char* lbm_last_error(const lbm_ctx* ctx)
{
    if (!ctx) return g_create_err.c_str();
    return ctx->err.c_str();
}

void lbm_destroy(lbm_ctx* ctx) { delete ctx; }

}  // extern "C"
