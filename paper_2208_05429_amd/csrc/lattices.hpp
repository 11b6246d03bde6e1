// lattices.hpp -- the velocity sets the marching kernel and the basic kernels
// are written over: D3Q19 (d3q19.hpp: the paper's set, Sec. 3) and the other
// two cubic sets for which Sec. 4.1 states that the two-step rule holds,
// D3Q15 and D3Q27.  Each descriptor gives Q, the velocities, weights and
// opposites, the compact indices the exchange uses, and the BGK collision.
//
// Numbering (part of the interface, include/lbm.h): c_0 = 0, directions
// 1..H (H = (Q-1)/2) are the neighbours that precede a cell in an x-slowest,
// z-fastest sweep with c_1 = (-1,0,0), and c_{q+H} = -c_q.
//   D3Q15  (-1,0,0) (0,-1,0) (0,0,-1) (-1,-1,-1) (-1,-1,1) (-1,1,-1) (-1,1,1)
//   D3Q27  the nine of D3Q19, then (-1,-1,-1) (-1,-1,1) (-1,1,-1) (-1,1,1)
// Weights by |c|^2 = 0, 1, 2, 3: D3Q15 2/9, 1/9, -, 1/72; D3Q27 8/27, 2/27,
// 1/54, 1/216; cs^2 = 1/3 for all.
#pragma once

#include "d3q19.hpp"

namespace lbm {

// D3Q19: the functions of d3q19.hpp, unchanged (the same instructions)
struct D3Q19 {
    static constexpr int Q = 19, H = 9;
    __host__ __device__ static constexpr int cx(int q) { return cxq(q); }
    __host__ __device__ static constexpr int cy(int q) { return cyq(q); }
    __host__ __device__ static constexpr int cz(int q) { return czq(q); }
    __host__ __device__ static constexpr int opp(int q) { return oppq(q); }
    template <class R>
    __host__ __device__ static constexpr R w(int q)
    {
        return wq<R>(q);
    }
    template <class R, bool FORCE>
    __device__ __forceinline__ static void collide(R (&g)[Q], R omega, R Fx, R Fy, R Fz)
    {
        lbm::collide<R, FORCE>(g, omega, Fx, Fy, Fz);
    }
};

namespace sets {
constexpr int N15[7][3] = {{-1, 0, 0}, {0, -1, 0}, {0, 0, -1}, {-1, -1, -1}, {-1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}};
constexpr int N27[13][3] = {{-1, 0, 0},  {0, -1, 0},  {0, 0, -1},   {-1, -1, 0},  {-1, 1, 0},
                            {-1, 0, -1}, {-1, 0, 1},  {0, -1, -1},  {0, -1, 1},   {-1, -1, -1},
                            {-1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}};
__host__ __device__ constexpr double rnd(double x) { return double((long long)(x + 0.5)); }
}  // namespace sets

// D3Q15 and D3Q27.  The BGK collision in offset form (g = f - w) is that of
// d3q19.hpp: each q in 1..H taken with q+H, an even part
// w [omega drho + omega rho (9/2 (c.u)^2 - 3/2 u.u)] (+ Guo) and an odd part
// K_q c_q . (omega j + (1 - omega/2) F) with K_q = 3 w_q rounded per speed so
// that the coefficients of the momentum they hand back sum to exactly 1 in
// the arithmetic type (2 K_1 + 8 K_3 = 1 for D3Q15; 2 K_1 + 8 K_2 + 8 K_3 = 1
// for D3Q27): a collision then returns the momentum it received without a
// systematic scale error, which in FP32 would grow linearly in time.
template <int NQ>
struct CubicSet {
    static_assert(NQ == 15 || NQ == 27, "D3Q15 or D3Q27");
    static constexpr int Q = NQ, H = (NQ - 1) / 2;
    __host__ __device__ static constexpr int neg(int k, int a) { return NQ == 15 ? sets::N15[k][a] : sets::N27[k][a]; }
    __host__ __device__ static constexpr int comp(int q, int a) { return q == 0 ? 0 : (q <= H ? neg(q - 1, a) : -neg(q - 1 - H, a)); }
    __host__ __device__ static constexpr int cx(int q) { return comp(q, 0); }
    __host__ __device__ static constexpr int cy(int q) { return comp(q, 1); }
    __host__ __device__ static constexpr int cz(int q) { return comp(q, 2); }
    __host__ __device__ static constexpr int opp(int q) { return q == 0 ? 0 : (q <= H ? q + H : q - H); }
    __host__ __device__ static constexpr int c2(int q) { return cx(q) * cx(q) + cy(q) * cy(q) + cz(q) * cz(q); }
    template <class R>
    __host__ __device__ static constexpr R w(int q)
    {
        return NQ == 15 ? (c2(q) == 0 ? R(2) / R(9) : (c2(q) == 1 ? R(1) / R(9) : R(1) / R(72)))
                        : (c2(q) == 0 ? R(8) / R(27)
                                      : (c2(q) == 1 ? R(2) / R(27) : (c2(q) == 2 ? R(1) / R(54) : R(1) / R(216))));
    }
    // odd-part coefficients by speed, exact in the arithmetic type R
    template <class R>
    __host__ __device__ static constexpr double kscale()
    {
        return NQ == 15 ? (sizeof(R) == 4 ? 134217728.0 : 72057594037927936.0)     // 2^27, 2^56
                        : (sizeof(R) == 4 ? 268435456.0 : 144115188075855872.0);  // 2^28, 2^57
    }
    template <class R>
    __host__ __device__ static constexpr double k3()  // corners, 3 w = 1/24 (D3Q15), 1/72 (D3Q27)
    {
        return sets::rnd(kscale<R>() / (NQ == 15 ? 24.0 : 72.0)) / kscale<R>();
    }
    template <class R>
    __host__ __device__ static constexpr double k2()  // edges (D3Q27), 3 w = 1/18
    {
        return NQ == 15 ? 0.0 : sets::rnd(kscale<R>() / 18.0) / kscale<R>();
    }
    template <class R>
    __host__ __device__ static constexpr double k1()  // axes: the rest of the unit sum
    {
        return (1.0 - 8.0 * k2<R>() - 8.0 * k3<R>()) / 2.0;
    }
    template <class R>
    __host__ __device__ static constexpr R K(int q)
    {
        return R(c2(q) == 1 ? k1<R>() : (c2(q) == 2 ? k2<R>() : k3<R>()));
    }

    template <class R, bool FORCE>
    __device__ __forceinline__ static void collide(R (&g)[Q], R omega, R Fx, R Fy, R Fz)
    {
        R s[H + 1], d[H + 1];
        sfor<1, H + 1>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            s[q] = g[q] + g[q + H];
            d[q] = g[q] - g[q + H];
        });
        R drho = g[0], jx = R(0), jy = R(0), jz = R(0);
        sfor<1, H + 1>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            drho += s[q];
            if constexpr (cx(q) != 0) jx = cx(q) > 0 ? jx + d[q] : jx - d[q];
            if constexpr (cy(q) != 0) jy = cy(q) > 0 ? jy + d[q] : jy - d[q];
            if constexpr (cz(q) != 0) jz = cz(q) > 0 ? jz + d[q] : jz - d[q];
        });
        if constexpr (FORCE) {
            jx = fma(R(0.5), Fx, jx);
            jy = fma(R(0.5), Fy, jy);
            jz = fma(R(0.5), Fz, jz);
        }
        const R rho = R(1) + drho;
        const R inv = recip(rho);
        const R ux = jx * inv, uy = jy * inv, uz = jz * inv;
        const R omw = R(1) - omega;
        const R usq15 = R(1.5) * fma(ux, ux, fma(uy, uy, uz * uz));
        const R od = omega * drho, orho = omega * rho;
        R ax = omega * jx, ay = omega * jy, az = omega * jz;
        R kF = R(0), uF = R(0);
        if constexpr (FORCE) {
            kF = fma(R(-0.5), omega, R(1));
            uF = fma(ux, Fx, fma(uy, Fy, uz * Fz));
            ax = fma(kF, Fx, ax);
            ay = fma(kF, Fy, ay);
            az = fma(kF, Fz, az);
        }
        {
            constexpr R w0 = w<R>(0);
            R e0 = w0 * fma(-orho, usq15, od);
            if constexpr (FORCE) e0 = fma(R(-3) * w0 * kF, uF, e0);
            g[0] = fma(omw, g[0], e0);
        }
        sfor<1, H + 1>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            constexpr R wv = w<R>(q);
            constexpr int ccx = cx(q), ccy = cy(q), ccz = cz(q);
            const R cu = cdot3<ccx, ccy, ccz>(ux, uy, uz);
            const R ca = cdot3<ccx, ccy, ccz>(ax, ay, az);
            R even = fma(wv * orho, fma(R(4.5) * cu, cu, -usq15), wv * od);
            if constexpr (FORCE) {
                const R cF = cdot3<ccx, ccy, ccz>(Fx, Fy, Fz);
                even = fma(kF * wv, fma(R(9) * cu, cF, R(-3) * uF), even);
            }
            const R odd = K<R>(q) * ca;
            g[q] = fma(omw, g[q], even + odd);
            g[q + H] = fma(omw, g[q + H], even - odd);
        });
    }

  private:
    // c . v for a direction with components in {-1, 0, 1}: the non-zero terms only
    template <int a_, int b_, int c_, class R>
    __device__ __forceinline__ static R cdot3(R a, R b, R c)
    {
        if constexpr (a_ != 0) {
            R r = a_ > 0 ? a : -a;
            if constexpr (b_ != 0) r = b_ > 0 ? r + b : r - b;
            if constexpr (c_ != 0) r = c_ > 0 ? r + c : r - c;
            return r;
        } else if constexpr (b_ != 0) {
            R r = b_ > 0 ? b : -b;
            if constexpr (c_ != 0) r = c_ > 0 ? r + c : r - c;
            return r;
        } else {
            return c_ > 0 ? c : -c;
        }
    }
};
using D3Q15 = CubicSet<15>;
using D3Q27 = CubicSet<27>;

// the coefficients are exact in each arithmetic type and sum to 1
template <class LT, class R>
constexpr bool k_sum_exact()
{
    return double(R(LT::template k1<R>())) == LT::template k1<R>() &&
           double(R(LT::template k2<R>())) == LT::template k2<R>() &&
           double(R(LT::template k3<R>())) == LT::template k3<R>() &&
           2.0 * LT::template k1<R>() + 8.0 * LT::template k2<R>() + 8.0 * LT::template k3<R>() == 1.0;
}
static_assert(k_sum_exact<D3Q15, float>() && k_sum_exact<D3Q15, double>(), "D3Q15 odd-part coefficients");
static_assert(k_sum_exact<D3Q27, float>() && k_sum_exact<D3Q27, double>(), "D3Q27 odd-part coefficients");

// ---- what the exchange needs of a set, for any of the three ----
template <class LT>
__host__ __device__ constexpr bool moves_yz_l(int q)
{
    return LT::cy(q) != 0 || LT::cz(q) != 0;
}
template <class LT>
__host__ __device__ constexpr int nyz()  // directions that move between columns of a plane
{
    int k = 0;
    for (int q = 0; q < LT::Q; ++q) k += moves_yz_l<LT>(q) ? 1 : 0;
    return k;
}
template <class LT>
__host__ __device__ constexpr int yz_index_l(int q)
{
    int k = 0;
    for (int p = 0; p < q; ++p) k += moves_yz_l<LT>(p) ? 1 : 0;
    return k;
}
template <class LT>
__host__ __device__ constexpr int nxp()  // directions with c_x = +1
{
    int k = 0;
    for (int q = 0; q < LT::Q; ++q) k += LT::cx(q) == 1 ? 1 : 0;
    return k;
}
template <class LT>
__host__ __device__ constexpr int xp_index_l(int q)
{
    int k = 0;
    for (int p = 0; p < q; ++p) k += LT::cx(p) == 1 ? 1 : 0;
    return k;
}
static_assert(nyz<D3Q19>() == 16 && nxp<D3Q19>() == 5 && nyz<D3Q15>() == 12 && nxp<D3Q15>() == 5 &&
                  nyz<D3Q27>() == 24 && nxp<D3Q27>() == 9,
              "exchange sizes");

// moving-wall term 6 w_q (c_q . u_w) of a population entering along c_q (as wall_term)
template <class LT, int q, class R>
__device__ __forceinline__ R wall_term_l(R uwx, R uwy, R uwz)
{
    R cu = R(0);
    if constexpr (LT::cx(q) != 0) cu += R(LT::cx(q)) * uwx;
    if constexpr (LT::cy(q) != 0) cu += R(LT::cy(q)) * uwy;
    if constexpr (LT::cz(q) != 0) cu += R(LT::cz(q)) * uwz;
    constexpr R w6 = R(6) * LT::template w<R>(q);
    return w6 * cu;
}

template <class LT, class R>
__device__ __forceinline__ void wall_terms_to_l(R* tab, int lane, R uwx, R uwy, R uwz)
{
    sfor<0, LT::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        if (lane == q) tab[q] = (q == 0) ? R(0) : wall_term_l<LT, q>(uwx, uwy, uwz);
    });
}

// moving_wall_out of d3q19.hpp for any set: the x-only directions are 1 and 1 + H
template <class LT, class R>
__device__ __forceinline__ void moving_wall_out_l(R& vxm, R& vxp, R* X, int stride, int slot, uint32_t rmask,
                                                  const R* tab)
{
    if (!__any(rmask != 0u)) return;
    const volatile R* t = tab;
    sfor<1, LT::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int qo = LT::opp(q);
        const bool hit = (rmask >> q) & 1u;
        if constexpr (moves_yz_l<LT>(qo)) {
            const R x = X[yz_index_l<LT>(qo) * stride + slot];
            X[yz_index_l<LT>(qo) * stride + slot] = hit ? x + t[q] : x;
        } else if constexpr (qo == 1) {
            vxm = hit ? vxm + t[q] : vxm;
        } else {
            vxp = hit ? vxp + t[q] : vxp;
        }
    });
}

}  // namespace lbm
