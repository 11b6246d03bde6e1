// d3q19.hpp -- device-side D3Q19 lattice, storage codecs and per-cell BGK
// collision for gfx950.  The numbering follows the public header: c_0 = 0,
// directions 1..9 point to the neighbours that precede a cell in an
// x-slowest, z-fastest sweep (Sec. 3 of the paper, Fig. 1a), c_{q+9} = -c_q.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace lbm {

constexpr int Q = 19;

// ---- velocity set, evaluated at compile time inside unrolled loops ----
__host__ __device__ constexpr int cxq(int q)
{
    constexpr int t[Q] = {0, -1, 0, 0, -1, -1, -1, -1, 0, 0, 1, 0, 0, 1, 1, 1, 1, 0, 0};
    return t[q];
}
__host__ __device__ constexpr int cyq(int q)
{
    constexpr int t[Q] = {0, 0, -1, 0, -1, 1, 0, 0, -1, -1, 0, 1, 0, 1, -1, 0, 0, 1, 1};
    return t[q];
}
__host__ __device__ constexpr int czq(int q)
{
    constexpr int t[Q] = {0, 0, 0, -1, 0, 0, -1, 1, -1, 1, 0, 0, 1, 0, 0, 1, -1, 1, -1};
    return t[q];
}
__host__ __device__ constexpr int oppq(int q) { return q == 0 ? 0 : (q <= 9 ? q + 9 : q - 9); }
__host__ __device__ constexpr int c2q(int q) { return cxq(q) * cxq(q) + cyq(q) * cyq(q) + czq(q) * czq(q); }
template <class R>
__host__ __device__ constexpr R wq(int q)
{
    return c2q(q) == 0 ? R(1) / R(3) : (c2q(q) == 1 ? R(1) / R(18) : R(1) / R(36));
}
// directions whose (y,z) part is nonzero move between columns of a plane
__host__ __device__ constexpr bool moves_yz(int q) { return cyq(q) != 0 || czq(q) != 0; }
// compact index 0..15 of the 16 column-moving directions
__host__ __device__ constexpr int yz_index(int q)
{
    int k = 0;
    for (int p = 0; p < q; ++p) k += moves_yz(p) ? 1 : 0;
    return k;
}
// compact index 0..4 of the five directions with c_x = +1
__host__ __device__ constexpr int xp_index(int q)
{
    int k = 0;
    for (int p = 0; p < q; ++p) k += cxq(p) == 1 ? 1 : 0;
    return k;
}

// compile-time loop: f(std::integral_constant<int, I>) for I in [B, E)
template <int B, int E, class F>
__device__ __forceinline__ void sfor(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(static_cast<F&&>(f));
    }
}

// ---- buffer access: uniform descriptor + 32-bit per-lane byte offset ----
// One descriptor covers `bytes` bytes from `base`; lanes whose offset is out of
// range read zero and their stores are dropped by the hardware range check.
constexpr int kBufDword3 = 0x00020000;  // gfx9 raw buffer: 32-bit data format, no swizzle
constexpr uint32_t kOffNone = 0xffffffffu;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufDword3);
}

template <class T>
struct Buf;
template <>
struct Buf<float> {
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, uint32_t off)
    {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    }
    static __device__ __forceinline__ void st(float v, __amdgpu_buffer_rsrc_t r, uint32_t off)
    {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, 0, 0);
    }
};
template <>
struct Buf<double> {
    static __device__ __forceinline__ double ld(__amdgpu_buffer_rsrc_t r, uint32_t off)
    {
        auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
        return __hiloint2double(int(v[1]), int(v[0]));
    }
    static __device__ __forceinline__ void st(double v, __amdgpu_buffer_rsrc_t r, uint32_t off)
    {
        typedef unsigned int u2 __attribute__((ext_vector_type(2)));
        u2 w;
        w[0] = uint32_t(__double2loint(v));
        w[1] = uint32_t(__double2hiint(v));
        __builtin_amdgcn_raw_buffer_store_b64(w, r, off, 0, 0);
    }
};
template <>
struct Buf<uint16_t> {
    static __device__ __forceinline__ uint16_t ld(__amdgpu_buffer_rsrc_t r, uint32_t off)
    {
        return __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
    }
    static __device__ __forceinline__ void st(uint16_t v, __amdgpu_buffer_rsrc_t r, uint32_t off)
    {
        __builtin_amdgcn_raw_buffer_store_b16(v, r, off, 0, 0);
    }
};

// ---- storage codecs: stored value is g = f - w_q ----
enum : int { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2, ST_BF16 = 3 };

template <int S>
struct Codec;
template <>
struct Codec<ST_F64> {
    using T = double;
    using R = double;
    static __device__ __forceinline__ R dec(T v) { return v; }
    static __device__ __forceinline__ T enc(R v) { return v; }
};
template <>
struct Codec<ST_F32> {
    using T = float;
    using R = float;
    static __device__ __forceinline__ R dec(T v) { return v; }
    static __device__ __forceinline__ T enc(R v) { return v; }
};
// The 16-bit codecs also encode two values into one 32-bit word (low half
// first), the form a pair store writes.  Both round to nearest even; gfx950
// converts a pair of floats in one instruction for either format.
typedef float f32x2 __attribute__((ext_vector_type(2)));
template <>
struct Codec<ST_F16> {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    using T = uint16_t;
    using R = float;
    // The conversion is exact; kept as its own instruction (the empty asm)
    // rather than fused by the compiler into a mixed-precision FMA, which
    // made the marching kernel 7 % slower.
    static __device__ __forceinline__ R dec(T v)
    {
        R r = __half2float(__ushort_as_half(v));
        asm("" : "+v"(r));
        return r;
    }
    static __device__ __forceinline__ T enc(R v) { return __half_as_ushort(__float2half_rn(v)); }
    static __device__ __forceinline__ uint32_t enc2(R a, R b)
    {
        const f32x2 v = {a, b};
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, h2));
    }
};
template <>
struct Codec<ST_BF16> {
    typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
    using T = uint16_t;
    using R = float;
    static __device__ __forceinline__ R dec(T v) { return __uint_as_float(uint32_t(v) << 16); }
    static __device__ __forceinline__ T enc(R v) { return __builtin_bit_cast(uint16_t, static_cast<__bf16>(v)); }
    static __device__ __forceinline__ uint32_t enc2(R a, R b)
    {
        const f32x2 v = {a, b};
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf2));
    }
};

// Momentum term of a moving wall for the population entering along c_q after
// bouncing: 6 w_q (c_q . u_w) (halfway bounce-back, wall density 1).  Every
// kernel uses this one expression so that the schemes agree to the last bit.
template <int q, class R>
__device__ __forceinline__ R wall_term(R uwx, R uwy, R uwz)
{
    R cu = R(0);
    if constexpr (cxq(q) != 0) cu += R(cxq(q)) * uwx;
    if constexpr (cyq(q) != 0) cu += R(cyq(q)) * uwy;
    if constexpr (czq(q) != 0) cu += R(czq(q)) * uwz;
    constexpr R w6 = R(6) * wq<R>(q);
    return w6 * cu;
}

// The moving-wall term, written into a table of Q values (entry q: the term
// received in direction q; entry 0 is zero), for kernels that keep it in LDS.
template <class R>
__device__ __forceinline__ void wall_terms_to(R* tab, int lane, R uwx, R uwy, R uwz)
{
    sfor<0, Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        if (lane == q) tab[q] = (q == 0) ? R(0) : wall_term<q>(uwx, uwy, uwz);
    });
}

// Moving wall, applied at the source.  A population whose link leaves the
// domain through the moving face has exactly one reader: the bounce-back
// into the opposite direction of its own cell.  Adding the wall term to it
// right after the collision is therefore the same single addition as adding
// it on receipt.  rmask: receiving directions q of this cell whose source lies
// beyond the moving face (bit q set: the cell's outgoing opp(q) gets term q).
// The populations that move in y or z are amended in the cell's own exchange
// slots (X[yz_index(q) * stride + slot], just written by this thread), the two
// x-only ones (q = 1, 10) in registers; nothing extra stays live.  The term
// table is read through a volatile pointer so the terms are loaded where they
// are used, on the few lanes next to the moving face.
template <class R>
__device__ __forceinline__ void moving_wall_out(R& v1, R& v10, R* X, int stride, int slot, uint32_t rmask,
                                                const R* tab)
{
    if (!__any(rmask != 0u)) return;  // wave-uniform: waves away from the moving face skip it
    const volatile R* t = tab;
    sfor<1, Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int qo = oppq(q);
        const bool hit = (rmask >> q) & 1u;
        if constexpr (moves_yz(qo)) {
            const R x = X[yz_index(qo) * stride + slot];
            X[yz_index(qo) * stride + slot] = hit ? x + t[q] : x;
        } else if constexpr (qo == 1) {
            v1 = hit ? v1 + t[q] : v1;
        } else {
            v10 = hit ? v10 + t[q] : v10;
        }
    });
}

// ---- per-cell physics in offset form ----
//
// With g_q = f_q - w_q: rho = 1 + sum g, j = sum c g, u = (j + F/2)/rho and
// geq_q = feq_q - w_q = w_q [ (rho - 1) + rho (3 c.u + 9/2 (c.u)^2 - 3/2 u.u) ].
// BGK: g*_q = g_q - omega (g_q - geq_q) + S_q, Guo forcing
// S_q = (1 - omega/2) w_q [3 (c_q - u) + 9 (c_q.u) c_q] . F.
// Each direction q in 1..9 is handled together with its opposite q+9: the
// equilibrium and forcing split into a part even in c and a part odd in c.
//
// The odd part, 3 w_q c_q . (omega rho u + (1 - omega/2) F), carries the
// momentum.  It is evaluated from j itself (rho u = j + F/2 exactly) with
// coefficients K1 = 3 w (|c| = 1) and K2 = 3 w (|c|^2 = 2) rounded so that
// 2 K1 + 8 K2 = 1 holds exactly in the arithmetic type: the collision then
// hands back exactly the momentum it received.  With K1 = fl(1/6) instead,
// every FP32 collision scales the momentum by (1 + omega * 3e-8), a bias that
// grows linearly in time (4e-6 of the velocity after 100 steps at tau = 0.8).

// 1/x.  FP32: the hardware reciprocal refined by one Newton step (within an
// ulp, a quarter of the instructions of the IEEE division); FP64 divides.
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float recip(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// c . a for a lattice direction with components in {-1, 0, 1}: the sum of
// the non-zero terms only (a leading 0 + would be kept for the sign of zero)
template <int cx, int cy, int cz, class R>
__device__ __forceinline__ R cdot(R ax, R ay, R az)
{
    R r = cx != 0 ? R(cx) * ax : (cy != 0 ? R(cy) * ay : R(cz) * az);
    if constexpr (cx != 0 && cy != 0) r += R(cy) * ay;
    if constexpr ((cx != 0 || cy != 0) && cz != 0) r += R(cz) * az;
    return r;
}

template <class R>
struct Moments {
    R drho, rho, jx, jy, jz;  // j includes F/2
    R ux, uy, uz;
};

template <class R, bool FORCE>
__device__ __forceinline__ Moments<R> moments(const R (&g)[Q], R Fx, R Fy, R Fz)
{
    R s[10], d[10];
    sfor<1, 10>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        s[q] = g[q] + g[q + 9];
        d[q] = g[q] - g[q + 9];
    });
    Moments<R> m;
    m.drho = g[0] + (((s[1] + s[2]) + (s[3] + s[4])) + ((s[5] + s[6]) + (s[7] + (s[8] + s[9]))));
    // j = sum_{q=1..9} c_q (g_q - g_{q+9}); every c_q here has components in {-1, 0, 1}
    m.jx = -((d[1] + d[4]) + (d[5] + (d[6] + d[7])));
    m.jy = -((d[2] + d[4]) + ((d[8] + d[9]) - d[5]));
    m.jz = -((d[3] + d[6]) + ((d[8] - d[9]) - d[7]));
    if constexpr (FORCE) {
        m.jx = fma(R(0.5), Fx, m.jx);
        m.jy = fma(R(0.5), Fy, m.jy);
        m.jz = fma(R(0.5), Fz, m.jz);
    }
    m.rho = R(1) + m.drho;
    const R inv = recip(m.rho);
    m.ux = m.jx * inv;
    m.uy = m.jy * inv;
    m.uz = m.jz * inv;
    return m;
}

// 3 w_q, rounded so that the odd parts return exactly the momentum they get
template <class R>
__device__ __forceinline__ constexpr R k_diag()
{
    return R(1) / R(12);
}
template <class R>
__device__ __forceinline__ constexpr R k_axis()
{
    return (R(1) - R(8) * k_diag<R>()) / R(2);
}

// Every multiply-add is an explicit fma() and the library is compiled without
// floating-point contraction, so this arithmetic is the same instruction
// sequence in every kernel: the three schemes agree to the last bit.
template <class R, bool FORCE>
__device__ __forceinline__ void collide(R (&g)[Q], R omega, R Fx = R(0), R Fy = R(0), R Fz = R(0))
{
    const Moments<R> m = moments<R, FORCE>(g, Fx, Fy, Fz);
    const R omw = R(1) - omega;
    const R usq15 = R(1.5) * fma(m.ux, m.ux, fma(m.uy, m.uy, m.uz * m.uz));
    const R od = omega * m.drho, orho = omega * m.rho;
    // odd-part momentum: omega (j + F/2) + (1 - omega/2) F
    R ax = omega * m.jx, ay = omega * m.jy, az = omega * m.jz;
    R kF = R(0), uF = R(0);
    if constexpr (FORCE) {
        kF = fma(R(-0.5), omega, R(1));
        uF = fma(m.ux, Fx, fma(m.uy, Fy, m.uz * Fz));
        ax = fma(kF, Fx, ax);
        ay = fma(kF, Fy, ay);
        az = fma(kF, Fz, az);
    }
    {
        constexpr R w0 = wq<R>(0);
        R e0 = w0 * fma(-orho, usq15, od);
        if constexpr (FORCE) e0 = fma(R(-3) * w0 * kF, uF, e0);
        g[0] = fma(omw, g[0], e0);
    }
    // even-part coefficients of the two weight classes: w omega rho, w omega drho
    const R wr1 = wq<R>(1) * orho, wd1 = wq<R>(1) * od;
    const R wr2 = wq<R>(4) * orho, wd2 = wq<R>(4) * od;
    sfor<1, 10>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr R w = wq<R>(q);
        constexpr int cx = cxq(q), cy = cyq(q), cz = czq(q);
        const R K = c2q(q) == 1 ? k_axis<R>() : k_diag<R>();
        const R cu = cdot<cx, cy, cz>(m.ux, m.uy, m.uz);
        const R ca = cdot<cx, cy, cz>(ax, ay, az);
        // even part w [omega drho + omega rho (9/2 cu^2 - 3/2 u^2)]
        R even = fma(c2q(q) == 1 ? wr1 : wr2, fma(R(4.5) * cu, cu, -usq15), c2q(q) == 1 ? wd1 : wd2);
        if constexpr (FORCE) {
            const R cF = cdot<cx, cy, cz>(Fx, Fy, Fz);
            even = fma(kF * w, fma(R(9) * cu, cF, R(-3) * uF), even);
        }
        const R odd = K * ca;
        g[q] = fma(omw, g[q], even + odd);
        g[q + 9] = fma(omw, g[q + 9], even - odd);
    });
}

}  // namespace lbm
