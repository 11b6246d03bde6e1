// k_basic.hip -- equilibrium initialisation, the plain two-array baseline step,
// the marching-pass prepass, macroscopic fields with FP64 conservation sums,
// and the storage-type dispatch of every launcher.
#include "d3q19.hpp"
#include "lattices.hpp"
#include "lbm_internal.hpp"

namespace lbm {

// ------------------------------------------------------------------------
// f := f_eq(rho0, u0), stored as g = f - w (Sec. 5.1: every algorithm starts
// from the same constructed state).  Evaluated in double, rounded once.
// ------------------------------------------------------------------------
template <class LT, int S>
__global__ __launch_bounds__(256) void k_init(Geom g, typename Codec<S>::T* f, const double* rho0, const double* u0)
{
    using Cd = Codec<S>;
    using R = typename Cd::R;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= g.N) return;
    const double rho = rho0 ? rho0[i] : 1.0;
    const double ux = u0 ? u0[i] : 0.0, uy = u0 ? u0[g.N + i] : 0.0, uz = u0 ? u0[2 * g.N + i] : 0.0;
    const double usq = ux * ux + uy * uy + uz * uz;
    sfor<0, LT::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const double cu = LT::cx(q) * ux + LT::cy(q) * uy + LT::cz(q) * uz;
        const double geq = LT::template w<double>(q) * ((rho - 1.0) + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * usq));
        f[q * g.N + i] = Cd::enc(R(geq));
    });
}

// ------------------------------------------------------------------------
// Plain baseline: one collide + push-stream step from src into dst (a second
// lattice), one thread per cell.  Same per-cell arithmetic as the in-place
// kernels, so the three schemes agree to the last bit.
// ------------------------------------------------------------------------
template <class LT, int S, bool WALLS, bool FORCE>
__global__ __launch_bounds__(256) void k_two_array(Geom g, const typename Codec<S>::T* __restrict__ src,
                                                   typename Codec<S>::T* __restrict__ dst,
                                                   const typename Codec<S>::R* __restrict__ F)
{
    using Cd = Codec<S>;
    using R = typename Cd::R;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= g.N) return;
    const int z = int(i % g.nz);
    const long long r = i / g.nz;
    const int y = int(r % g.ny), x = int(r / g.ny);
    R v[LT::Q];
#pragma unroll
    for (int q = 0; q < LT::Q; ++q) v[q] = Cd::dec(src[q * g.N + i]);
    R Fx = R(0), Fy = R(0), Fz = R(0);
    if constexpr (FORCE) {
        Fx = F[i];
        Fy = F[g.N + i];
        Fz = F[2 * g.N + i];
    }
    LT::template collide<R, FORCE>(v, R(g.omega), Fx, Fy, Fz);
    const int n[3] = {g.nx, g.ny, g.nz};
    sfor<0, LT::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const int c[3] = {LT::cx(q), LT::cy(q), LT::cz(q)};
        int p[3] = {x + c[0], y + c[1], z + c[2]};
        bool out = false, moving = false;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            if (c[ax] == 0 || (p[ax] >= 0 && p[ax] < n[ax])) continue;
            const int face = 2 * ax + (p[ax] >= n[ax] ? 1 : 0);
            if (WALLS && g.wall[ax]) {
                out = true;
                if (face == g.moving_face) moving = true;
            } else {
                p[ax] = p[ax] < 0 ? p[ax] + n[ax] : p[ax] - n[ax];
            }
        }
        if (WALLS && out) {
            R val = v[q];
            if (moving) val += wall_term_l<LT, LT::opp(q)>(R(g.uw[0]), R(g.uw[1]), R(g.uw[2]));
            dst[LT::opp(q) * g.N + i] = Cd::enc(val);
        } else {
            dst[q * g.N + ((long long)p[0] * g.ny + p[1]) * g.nz + p[2]] = Cd::enc(v[q]);
        }
    });
}

// ------------------------------------------------------------------------
// Prepass of a marching pass: save the time-t copies of the first M planes of
// every segment and clear the progress counters (flags[0] is the timeout
// word, flags[(1 + w) * fstride] the counter of work item w).
// ------------------------------------------------------------------------
// One contiguous run of len values, copied by the blocks of one grid row:
// 16-byte accesses when the caller has checked that both runs are 16-byte
// aligned and len is a whole number of 16-byte units.
template <class T>
__device__ __forceinline__ void copy_run(const T* __restrict__ src, T* __restrict__ dst, long long len, bool vec)
{
    const long long t0 = (long long)blockIdx.x * 256 + threadIdx.x, stride = (long long)gridDim.x * 256;
    if (vec) {
        const long long n16 = len * (long long)sizeof(T) / 16;
        const uint4* __restrict__ s4 = reinterpret_cast<const uint4*>(src);
        uint4* __restrict__ d4 = reinterpret_cast<uint4*>(dst);
        for (long long i = t0; i < n16; i += stride) d4[i] = s4[i];
    } else {
        for (long long i = t0; i < len; i += stride) dst[i] = src[i];
    }
}

// Grid rows walk the runs (run it = (b * M + j) * Q + q: plane j of segment b,
// direction q, one y-z plane long); the blocks of a row split the run.
template <class T>
__global__ __launch_bounds__(256) void k_prepass(Geom g, const T* __restrict__ f, T* __restrict__ side, int* flags,
                                                 int nflags, int fstride, int M, int seg_len, int nseg, int vec)
{
    const int nitems = nseg * M * g.lat;
    for (int it = blockIdx.y; it < nitems; it += gridDim.y) {
        const int q = it % g.lat, bj = it / g.lat;
        const int b = bj / M, j = bj - b * M;
        const int plane = (b * seg_len + j) % g.nx;
        copy_run(f + (long long)q * g.N + (long long)plane * g.PL, side + (long long)it * g.PL, g.PL, vec != 0);
    }
    // progress counters 1 .. nflags-1; word 0, the timeout report, is left as
    // it is: it stays set once any pass of the context has timed out
    if (blockIdx.y == 0)
        for (long long t = (long long)blockIdx.x * 256 + threadIdx.x + 1; t < nflags; t += (long long)gridDim.x * 256)
            flags[t * fstride] = 0;
}

__global__ __launch_bounds__(64) void k_clear_word(int* w)
{
    if (threadIdx.x == 0) w[0] = 0;
}

hipError_t launch_clear_word(int* w, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(64), 0, s, w);
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// Macroscopic fields in double from the stored state, and per-block FP64
// partial sums of (sum g, j) reduced with wavefront shuffles.
// ------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double* sh)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sh[k];
    return t;
}

template <class LT, int S, bool FORCE>
__global__ __launch_bounds__(256) void k_macro(Geom g, const typename Codec<S>::T* __restrict__ f,
                                               const typename Codec<S>::R* __restrict__ F, double* rho_out,
                                               double* u_out, double* un_out, double* partials)
{
    using Cd = Codec<S>;
    __shared__ double sh[4];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < g.N; i += (long long)gridDim.x * 256) {
        double gq[LT::Q];
#pragma unroll
        for (int q = 0; q < LT::Q; ++q) gq[q] = double(Cd::dec(f[q * g.N + i]));
        double drho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
        sfor<0, LT::Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            drho += gq[q];
            if constexpr (LT::cx(q) != 0) jx += LT::cx(q) * gq[q];
            if constexpr (LT::cy(q) != 0) jy += LT::cy(q) * gq[q];
            if constexpr (LT::cz(q) != 0) jz += LT::cz(q) * gq[q];
        });
        acc[0] += drho;
        acc[1] += jx;
        acc[2] += jy;
        acc[3] += jz;
        const double rho = 1.0 + drho;
        double Fx = 0.0, Fy = 0.0, Fz = 0.0;
        if constexpr (FORCE) {
            Fx = double(F[i]);
            Fy = double(F[g.N + i]);
            Fz = double(F[2 * g.N + i]);
        }
        const double ux = (jx + 0.5 * Fx) / rho, uy = (jy + 0.5 * Fy) / rho, uz = (jz + 0.5 * Fz) / rho;
        if (rho_out) rho_out[i] = rho;
        if (u_out) {
            u_out[i] = ux;
            u_out[g.N + i] = uy;
            u_out[2 * g.N + i] = uz;
        }
        if (un_out) un_out[i] = sqrt(ux * ux + uy * uy + uz * uz);
    }
    if (partials) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double t = block_sum(acc[k], sh);
            if (threadIdx.x == 0) partials[blockIdx.x * 4 + k] = t;
        }
    }
}

// sums = { N + sum g, sum j } from the per-block partials, in a fixed order
__global__ __launch_bounds__(256) void k_sums(const double* partials, int nblocks, double ncell, double* sums)
{
    __shared__ double sh[4];
    for (int k = 0; k < 4; ++k) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += 256) v += partials[b * 4 + k];
        const double t = block_sum(v, sh);
        if (threadIdx.x == 0) sums[k] = (k == 0 ? ncell : 0.0) + t;
    }
}

// ------------------------------------------------------------------------
// dispatch
// ------------------------------------------------------------------------
static unsigned grid_for(long long n) { return unsigned((n + 255) / 256); }

template <class LT, int S>
static hipError_t init_s(const Geom& g, void* f, const double* rho0, const double* u0, hipStream_t s)
{
    hipLaunchKernelGGL((k_init<LT, S>), dim3(grid_for(g.N)), dim3(256), 0, s, g,
                       static_cast<typename Codec<S>::T*>(f), rho0, u0);
    return hipGetLastError();
}

// D3Q15 and D3Q27 are built for FP64 and FP32 storage
template <class LT>
static hipError_t init_set(int storage, const Geom& g, void* f, const double* rho0, const double* u0, hipStream_t s)
{
    switch (storage) {
    case ST_F64: return init_s<LT, ST_F64>(g, f, rho0, u0, s);
    case ST_F32: return init_s<LT, ST_F32>(g, f, rho0, u0, s);
    case ST_F16: return init_s<LT, ST_F16>(g, f, rho0, u0, s);
    case ST_BF16: return init_s<LT, ST_BF16>(g, f, rho0, u0, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_init(int storage, const Geom& g, void* f, const double* rho0, const double* u0, hipStream_t s)
{
    if (g.lat == 15) return init_set<D3Q15>(storage, g, f, rho0, u0, s);
    if (g.lat == 27) return init_set<D3Q27>(storage, g, f, rho0, u0, s);
    switch (storage) {
    case ST_F64: return init_s<D3Q19, ST_F64>(g, f, rho0, u0, s);
    case ST_F32: return init_s<D3Q19, ST_F32>(g, f, rho0, u0, s);
    case ST_F16: return init_s<D3Q19, ST_F16>(g, f, rho0, u0, s);
    case ST_BF16: return init_s<D3Q19, ST_BF16>(g, f, rho0, u0, s);
    }
    return hipErrorInvalidValue;
}

template <int S, bool FORCE, class LT = D3Q19>
static hipError_t two_array_s(const Geom& g, const void* src, void* dst, const void* F, hipStream_t s)
{
    using Cd = Codec<S>;
    const bool walls = g.wall[0] || g.wall[1] || g.wall[2];
    auto sp = static_cast<const typename Cd::T*>(src);
    auto dp = static_cast<typename Cd::T*>(dst);
    auto fp = static_cast<const typename Cd::R*>(F);
    if (walls)
        hipLaunchKernelGGL((k_two_array<LT, S, true, FORCE>), dim3(grid_for(g.N)), dim3(256), 0, s, g, sp, dp, fp);
    else
        hipLaunchKernelGGL((k_two_array<LT, S, false, FORCE>), dim3(grid_for(g.N)), dim3(256), 0, s, g, sp, dp, fp);
    return hipGetLastError();
}

template <class LT>
static hipError_t two_array_set(int storage, bool force, const Geom& g, const void* src, void* dst, const void* F,
                                hipStream_t s)
{
    switch (storage) {
    case ST_F64:
        return force ? two_array_s<ST_F64, true, LT>(g, src, dst, F, s) : two_array_s<ST_F64, false, LT>(g, src, dst, F, s);
    case ST_F32:
        return force ? two_array_s<ST_F32, true, LT>(g, src, dst, F, s) : two_array_s<ST_F32, false, LT>(g, src, dst, F, s);
    case ST_F16:
        return force ? two_array_s<ST_F16, true, LT>(g, src, dst, F, s) : two_array_s<ST_F16, false, LT>(g, src, dst, F, s);
    case ST_BF16:
        return force ? two_array_s<ST_BF16, true, LT>(g, src, dst, F, s)
                     : two_array_s<ST_BF16, false, LT>(g, src, dst, F, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_two_array(int storage, bool force, const Geom& g, const void* src, void* dst, const void* F,
                            hipStream_t s)
{
    if (g.lat == 15) return two_array_set<D3Q15>(storage, force, g, src, dst, F, s);
    if (g.lat == 27) return two_array_set<D3Q27>(storage, force, g, src, dst, F, s);
    switch (storage) {
    case ST_F64: return force ? two_array_s<ST_F64, true>(g, src, dst, F, s) : two_array_s<ST_F64, false>(g, src, dst, F, s);
    case ST_F32: return force ? two_array_s<ST_F32, true>(g, src, dst, F, s) : two_array_s<ST_F32, false>(g, src, dst, F, s);
    case ST_F16: return force ? two_array_s<ST_F16, true>(g, src, dst, F, s) : two_array_s<ST_F16, false>(g, src, dst, F, s);
    case ST_BF16:
        return force ? two_array_s<ST_BF16, true>(g, src, dst, F, s) : two_array_s<ST_BF16, false>(g, src, dst, F, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_copy(int storage, const Geom& g, const void* src, void* dst, hipStream_t s)
{
    const size_t elem = storage == ST_F64 ? 8 : (storage == ST_F32 ? 4 : 2);
    return hipMemcpyAsync(dst, src, size_t(g.lat) * size_t(g.N) * elem, hipMemcpyDeviceToDevice, s);
}

static bool aligned16(const void* p)
{
    return (reinterpret_cast<uintptr_t>(p) & 15u) == 0;
}

// Grid for nitems runs of `units` copy units each: rows walk the runs, about
// four units per thread along a row.
static dim3 run_grid(long long units, int nitems)
{
    long long bx = (units + 1023) / 1024;
    if (bx < 1) bx = 1;
    if (bx > 1024) bx = 1024;
    const int by = nitems < 1 ? 1 : (nitems > 65535 ? 65535 : nitems);
    return dim3(unsigned(bx), unsigned(by));
}

template <class T>
static hipError_t prepass_t(const Geom& g, const MarchPlan& p, const void* f, void* side, int* flags, hipStream_t s)
{
    const int nitems = p.nseg * p.M * g.lat;
    const bool vec = (g.PL * (long long)sizeof(T)) % 16 == 0 && aligned16(f) && aligned16(side);
    const dim3 grid = run_grid(vec ? g.PL * (long long)sizeof(T) / 16 : g.PL, nitems);
    const int nflags = p.nty * p.ntz * p.nseg + 1;  // every tile of every round, and the timeout word
    hipLaunchKernelGGL(k_prepass<T>, grid, dim3(256), 0, s, g, static_cast<const T*>(f), static_cast<T*>(side), flags,
                       nflags, p.flag_stride, p.M, p.seg_len, p.nseg, int(vec));
    return hipGetLastError();
}

// The M boundary rows of every band of tile rows, at time t, before a pass in
// rounds: shell[((band * 2 + part) * nx + x) * Q + q][row][z], part 0 the
// band's first M rows, part 1 its last M rows.
template <class T>
__global__ __launch_bounds__(256) void k_shells(Geom g, const T* __restrict__ f, T* __restrict__ shell, int M,
                                                int band_rows, int nbands, int vec)
{
    const long long len = (long long)M * g.nz;  // M consecutive rows: one contiguous run of the lattice
    const int nitems = nbands * 2 * g.nx * g.lat;
    for (int it = blockIdx.y; it < nitems; it += gridDim.y) {
        int r = it;
        const int q = r % g.lat;
        r /= g.lat;
        const int x = r % g.nx;
        r /= g.nx;
        const int part = r % 2, band = r / 2;
        const int y0 = band * band_rows, y1 = min(g.ny, y0 + band_rows);
        const int y = part == 0 ? y0 : y1 - M;
        copy_run(f + (long long)q * g.N + ((long long)x * g.ny + y) * g.nz, shell + (long long)it * len, len, vec != 0);
    }
}

template <class T>
static hipError_t shells_t(const Geom& g, const MarchPlan& p, int TY, const void* f, void* shell, hipStream_t s)
{
    const int nitems = p.nbands * 2 * g.nx * g.lat;
    const long long len = (long long)p.M * g.nz;
    const bool vec = (g.nz * (long long)sizeof(T)) % 16 == 0 && aligned16(f) && aligned16(shell);
    hipLaunchKernelGGL(k_shells<T>, run_grid(vec ? len * (long long)sizeof(T) / 16 : len, nitems), dim3(256), 0, s, g,
                       static_cast<const T*>(f), static_cast<T*>(shell), p.M, p.nty_band * TY, p.nbands, int(vec));
    return hipGetLastError();
}

hipError_t launch_shells(int storage, const Geom& g, const MarchPlan& p, int TY, const void* f, void* shell,
                         hipStream_t s)
{
    switch (storage) {
    case ST_F64: return shells_t<double>(g, p, TY, f, shell, s);
    case ST_F32: return shells_t<float>(g, p, TY, f, shell, s);
    default: return shells_t<uint16_t>(g, p, TY, f, shell, s);
    }
}

hipError_t launch_prepass(int storage, const Geom& g, const MarchPlan& p, const void* f, void* side, int* flags,
                          hipStream_t s)
{
    switch (storage) {
    case ST_F64: return prepass_t<double>(g, p, f, side, flags, s);
    case ST_F32: return prepass_t<float>(g, p, f, side, flags, s);
    default: return prepass_t<uint16_t>(g, p, f, side, flags, s);
    }
}

template <int S, bool FORCE, class LT = D3Q19>
static hipError_t macro_s(const Geom& g, const void* f, const void* F, double* rho, double* u, double* un,
                          double* partials, double* sums, hipStream_t s)
{
    using Cd = Codec<S>;
    hipLaunchKernelGGL((k_macro<LT, S, FORCE>), dim3(SUM_BLOCKS), dim3(256), 0, s, g,
                       static_cast<const typename Cd::T*>(f), static_cast<const typename Cd::R*>(F), rho, u, un,
                       sums ? partials : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !sums) return e;
    hipLaunchKernelGGL(k_sums, dim3(1), dim3(256), 0, s, partials, SUM_BLOCKS, double(g.N), sums);
    return hipGetLastError();
}

template <class LT>
static hipError_t macro_set(int storage, bool force, const Geom& g, const void* f, const void* F, double* rho,
                            double* u, double* unorm, double* partials, double* sums, hipStream_t s)
{
    switch (storage) {
    case ST_F64:
        return force ? macro_s<ST_F64, true, LT>(g, f, F, rho, u, unorm, partials, sums, s)
                     : macro_s<ST_F64, false, LT>(g, f, F, rho, u, unorm, partials, sums, s);
    case ST_F32:
        return force ? macro_s<ST_F32, true, LT>(g, f, F, rho, u, unorm, partials, sums, s)
                     : macro_s<ST_F32, false, LT>(g, f, F, rho, u, unorm, partials, sums, s);
    case ST_F16:
        return force ? macro_s<ST_F16, true, LT>(g, f, F, rho, u, unorm, partials, sums, s)
                     : macro_s<ST_F16, false, LT>(g, f, F, rho, u, unorm, partials, sums, s);
    case ST_BF16:
        return force ? macro_s<ST_BF16, true, LT>(g, f, F, rho, u, unorm, partials, sums, s)
                     : macro_s<ST_BF16, false, LT>(g, f, F, rho, u, unorm, partials, sums, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_macro(int storage, bool force, const Geom& g, const void* f, const void* F, double* rho, double* u,
                        double* unorm, double* partials, double* sums, hipStream_t s)
{
    if (g.lat == 15) return macro_set<D3Q15>(storage, force, g, f, F, rho, u, unorm, partials, sums, s);
    if (g.lat == 27) return macro_set<D3Q27>(storage, force, g, f, F, rho, u, unorm, partials, sums, s);
    switch (storage) {
    case ST_F64:
        return force ? macro_s<ST_F64, true>(g, f, F, rho, u, unorm, partials, sums, s)
                     : macro_s<ST_F64, false>(g, f, F, rho, u, unorm, partials, sums, s);
    case ST_F32:
        return force ? macro_s<ST_F32, true>(g, f, F, rho, u, unorm, partials, sums, s)
                     : macro_s<ST_F32, false>(g, f, F, rho, u, unorm, partials, sums, s);
    case ST_F16:
        return force ? macro_s<ST_F16, true>(g, f, F, rho, u, unorm, partials, sums, s)
                     : macro_s<ST_F16, false>(g, f, F, rho, u, unorm, partials, sums, s);
    case ST_BF16:
        return force ? macro_s<ST_BF16, true>(g, f, F, rho, u, unorm, partials, sums, s)
                     : macro_s<ST_BF16, false>(g, f, F, rho, u, unorm, partials, sums, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lbm
