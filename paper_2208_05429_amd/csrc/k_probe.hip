// k_probe.hip -- two measurement probes that bound what the marching kernel
// can reach on this memory system.  They compute nothing of the method.
//
// k_copy16: a streaming device copy, 16-byte loads and stores per lane, one
// launch over a persistent grid (by default the marching kernel's: 256
// workgroups of 512 threads), four independent 16-byte accesses in flight
// per lane.  Its read+write rate is the achievable rate of a 1:1 read/write
// mix, the mix of an in-place pass.
//
// k_pattern: the marching kernel's HBM access pattern without its compute,
// LDS exchange, halo or hazard checks.  The same work items (tiles of the
// y-z plane by x segments, the same XCD-aware order), the same pair layout
// (each thread owns two z-adjacent cells of a TY x TZ tile), and per plane
// the same accesses: 19 pair loads of plane x, one per direction, and 19
// pair stores to plane x - M, in place.  What it stores is what it loaded M
// planes earlier, so the lattice is left unchanged.
#include "lbm_internal.hpp"
#include "march.hpp"

namespace lbm {

__global__ __launch_bounds__(512) void k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, long long n)
{
    const long long stride = (long long)gridDim.x * 512;
    long long i = (long long)blockIdx.x * 512 + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

struct PatternArgs {
    void* f;
    long long N, PL;
    int nx, ny, nz;
    int nty, ntz, nseg, seg_len, items, xcd_remap;
};

// W: bytes of one pair (8 for 32-bit storage, 4 for 16-bit)
template <int W, int M, int TY, int TZ>
__global__ __launch_bounds__(TY * TZ / 2) void k_pattern(PatternArgs a)
{
    using V = typename std::conditional<W == 8, unsigned long long, uint32_t>::type;
    constexpr int ES = W / 2;  // bytes per value
    int wid = blockIdx.x;
    if (a.xcd_remap) {
        const int per = gridDim.x >> 3;
        wid = (wid & 7) * per + (wid >> 3);
    }
    if (wid >= a.items) return;
    int tz, ty, seg;
    tile_of_item<TZ>(wid, a.nty, a.ntz, tz, ty, seg);
    const int s = seg * a.seg_len, e = min(s + a.seg_len, a.nx);
    const int tid = threadIdx.x;
    const int y = ty * TY + tid / (TZ / 2), z = tz * TZ + 2 * (tid % (TZ / 2));
    const uint32_t off = (y < a.ny && z < a.nz) ? uint32_t(y * a.nz + z) * uint32_t(ES) : kOffNone;
    const uint32_t plane_bytes = uint32_t(a.PL) * uint32_t(ES);
    const unsigned char* f = static_cast<const unsigned char*>(a.f);
    const long long qbytes = a.N * ES, pbytes = a.PL * ES;

    V ring[M + 1][Q];
#pragma unroll
    for (int b = 0; b <= M; ++b)
#pragma unroll
        for (int q = 0; q < Q; ++q) ring[b][q] = V(0);
    // plane x is loaded in iteration x - s and stored back in iteration x - s + M
    for (int i0 = 0; i0 < (e - s) + M; i0 += M + 1) {
        sfor<0, M + 1>([&](auto bc) {
            constexpr int b = decltype(bc)::value;
            constexpr int bs = (b + 1) % (M + 1);  // the slot loaded M iterations ago
            const int i = i0 + b, xl = s + i, xs = xl - M;
            const bool st = i < (e - s) + M && xs >= s;
            const bool ld = xl < e;
            if (st) {
                const unsigned char* bq = f + (long long)xs * pbytes;
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    if constexpr (W == 8) {
                        typedef unsigned int u2 __attribute__((ext_vector_type(2)));
                        u2 w;
                        w[0] = uint32_t(ring[bs][q]);
                        w[1] = uint32_t(ring[bs][q] >> 32);
                        __builtin_amdgcn_raw_buffer_store_b64(w, make_rsrc(bq, plane_bytes), off, 0, 0);
                    } else {
                        __builtin_amdgcn_raw_buffer_store_b32(ring[bs][q], make_rsrc(bq, plane_bytes), off, 0, 0);
                    }
                    bq += qbytes;
                }
            }
            const unsigned char* bq = f + (long long)(ld ? xl : 0) * pbytes;
            const uint32_t range = ld ? plane_bytes : 0u;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                if constexpr (W == 8) {
                    auto v = __builtin_amdgcn_raw_buffer_load_b64(make_rsrc(bq, range), off, 0, 0);
                    ring[b][q] = (unsigned long long)v[0] | ((unsigned long long)v[1] << 32);
                } else {
                    ring[b][q] = __builtin_amdgcn_raw_buffer_load_b32(make_rsrc(bq, range), off, 0, 0);
                }
                bq += qbytes;
            }
        });
    }
}

hipError_t launch_probe_copy(const void* src, void* dst, long long n16, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy16, dim3(blocks), dim3(512), 0, s, static_cast<const uint4*>(src), static_cast<uint4*>(dst),
                       n16);
    return hipGetLastError();
}

hipError_t launch_probe_pattern(int storage, const Geom& g, const MarchPlan& p, void* f, hipStream_t s)
{
    PatternArgs a;
    a.f = f;
    a.N = g.N;
    a.PL = g.PL;
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.nty = p.nty;
    a.ntz = p.ntz;
    a.nseg = p.nseg;
    a.seg_len = p.seg_len;
    a.items = p.nty * p.ntz * p.nseg;
    const int blocks = (a.items + 7) / 8 * 8;
    a.xcd_remap = 1;
    const bool w8 = storage == ST_F32;
    if (p.TY == 16 && p.TZ == 64 && p.M == 2) {
        if (w8)
            hipLaunchKernelGGL((k_pattern<8, 2, 16, 64>), dim3(blocks), dim3(512), 0, s, a);
        else
            hipLaunchKernelGGL((k_pattern<4, 2, 16, 64>), dim3(blocks), dim3(512), 0, s, a);
    } else if (p.TY == 16 && p.TZ == 64 && p.M == 1) {
        if (w8)
            hipLaunchKernelGGL((k_pattern<8, 1, 16, 64>), dim3(blocks), dim3(512), 0, s, a);
        else
            hipLaunchKernelGGL((k_pattern<4, 1, 16, 64>), dim3(blocks), dim3(512), 0, s, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lbm
