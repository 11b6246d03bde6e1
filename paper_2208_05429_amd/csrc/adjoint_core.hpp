// adjoint_core.hpp -- per-cell transposed Jacobian of the BGK collision with
// Guo forcing (the "collide^T" of the discrete adjoint), shared by the
// one-step and the two-step adjoint kernels.
//
// With mu the adjoint arriving at the cell (after the transposed stream),
// A = sum_q mu_q w_q, B = sum_q mu_q w_q c_q, C = sum_q mu_q w_q c_q c_q,
// omega = 1/tau and k = 1 - omega/2:
//   g_rho = omega [A (1 - 3/2 u.u) + 3 B.u + 9/2 u.C.u]
//   g_u   = omega rho [3 B + 9 C u - 3 A u] + k [9 C F - 3 A F]
//   lambda_j = (1 - omega) mu_j + g_rho + g_u . (c_j - u) / rho
//   dL/dF += k [3 B - 3 A u + 9 C u] + g_u / (2 rho)
// where rho and u = (sum c f + F/2)/rho are the moments of the state the
// forward collision saw.  The sums run over the velocity set LT (D3Q19,
// D3Q15 or D3Q27: every velocity component is -1, 0 or 1, so c_a c_a = |c_a|).
#pragma once

#include <type_traits>

#include "lattices.hpp"

namespace lbm {

template <class R, bool FORCE, class LT = D3Q19>
__device__ __forceinline__ void collide_adjoint_m(R rho, R ux, R uy, R uz, const R (&mu)[LT::Q], R omega, R Fx, R Fy,
                                                  R Fz, R (&lam)[LT::Q], R& gFx, R& gFy, R& gFz)
{
    R A = R(0), Bx = R(0), By = R(0), Bz = R(0);
    R Cxx = R(0), Cyy = R(0), Czz = R(0), Cxy = R(0), Cxz = R(0), Cyz = R(0);
    sfor<0, LT::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int cx = LT::cx(q), cy = LT::cy(q), cz = LT::cz(q);
        const R mw = mu[q] * LT::template w<R>(q);
        A += mw;
        if constexpr (cx != 0) Bx += R(cx) * mw;
        if constexpr (cy != 0) By += R(cy) * mw;
        if constexpr (cz != 0) Bz += R(cz) * mw;
        if constexpr (cx != 0) Cxx += mw;
        if constexpr (cy != 0) Cyy += mw;
        if constexpr (cz != 0) Czz += mw;
        if constexpr (cx * cy != 0) Cxy += R(cx * cy) * mw;
        if constexpr (cx * cz != 0) Cxz += R(cx * cz) * mw;
        if constexpr (cy * cz != 0) Cyz += R(cy * cz) * mw;
    });
    const R Cux = Cxx * ux + Cxy * uy + Cxz * uz;
    const R Cuy = Cxy * ux + Cyy * uy + Cyz * uz;
    const R Cuz = Cxz * ux + Cyz * uy + Czz * uz;
    const R usq = ux * ux + uy * uy + uz * uz;
    const R g_rho = omega * (A * (R(1) - R(1.5) * usq) + R(3) * (Bx * ux + By * uy + Bz * uz) +
                             R(4.5) * (ux * Cux + uy * Cuy + uz * Cuz));
    const R orho = omega * rho;
    R gux = orho * (R(3) * Bx + R(9) * Cux - R(3) * A * ux);
    R guy = orho * (R(3) * By + R(9) * Cuy - R(3) * A * uy);
    R guz = orho * (R(3) * Bz + R(9) * Cuz - R(3) * A * uz);
    const R kF = R(1) - R(0.5) * omega;
    if constexpr (FORCE) {
        gux += kF * (R(9) * (Cxx * Fx + Cxy * Fy + Cxz * Fz) - R(3) * A * Fx);
        guy += kF * (R(9) * (Cxy * Fx + Cyy * Fy + Cyz * Fz) - R(3) * A * Fy);
        guz += kF * (R(9) * (Cxz * Fx + Cyz * Fy + Czz * Fz) - R(3) * A * Fz);
    }
    const R inv = R(1) / rho;
    const R gdu = (gux * ux + guy * uy + guz * uz) * inv;
    const R omw = R(1) - omega;
    sfor<0, LT::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        R cg = R(0);
        if constexpr (LT::cx(q) != 0) cg += R(LT::cx(q)) * gux;
        if constexpr (LT::cy(q) != 0) cg += R(LT::cy(q)) * guy;
        if constexpr (LT::cz(q) != 0) cg += R(LT::cz(q)) * guz;
        lam[q] = omw * mu[q] + g_rho + (cg * inv - gdu);
    });
    const R i2 = R(0.5) * inv;
    gFx = kF * (R(3) * Bx - R(3) * A * ux + R(9) * Cux) + gux * i2;
    gFy = kF * (R(3) * By - R(3) * A * uy + R(9) * Cuy) + guy * i2;
    gFz = kF * (R(3) * Bz - R(3) * A * uz + R(9) * Cuz) + guz * i2;
}

// Moments of a cell of set LT from its offsets g = f - w: D3Q19 takes the
// pairwise sums of d3q19.hpp, the other sets the plain sums.
template <class R, bool FORCE, class LT = D3Q19>
__device__ __forceinline__ Moments<R> moments_l(const R (&g)[LT::Q], R Fx, R Fy, R Fz)
{
    if constexpr (std::is_same<LT, D3Q19>::value) {
        return moments<R, FORCE>(g, Fx, Fy, Fz);
    } else {
        Moments<R> m;
        m.drho = g[0];
        m.jx = m.jy = m.jz = R(0);
        sfor<1, LT::Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            m.drho += g[q];
            if constexpr (LT::cx(q) != 0) m.jx = LT::cx(q) > 0 ? m.jx + g[q] : m.jx - g[q];
            if constexpr (LT::cy(q) != 0) m.jy = LT::cy(q) > 0 ? m.jy + g[q] : m.jy - g[q];
            if constexpr (LT::cz(q) != 0) m.jz = LT::cz(q) > 0 ? m.jz + g[q] : m.jz - g[q];
        });
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
}

// the same from the cell's distributions (offset form)
template <class R, bool FORCE, class LT = D3Q19>
__device__ __forceinline__ void collide_adjoint(const R (&g)[LT::Q], const R (&mu)[LT::Q], R omega, R Fx, R Fy, R Fz,
                                                R (&lam)[LT::Q], R& gFx, R& gFy, R& gFz)
{
    const Moments<R> m = moments_l<R, FORCE, LT>(g, Fx, Fy, Fz);
    collide_adjoint_m<R, FORCE, LT>(m.rho, m.ux, m.uy, m.uz, mu, omega, Fx, Fy, Fz, lam, gFx, gFy, gFz);
}

}  // namespace lbm
