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
// forward collision saw.
#pragma once

#include "d3q19.hpp"

namespace lbm {

template <class R, bool FORCE>
__device__ __forceinline__ void collide_adjoint_m(R rho, R ux, R uy, R uz, const R (&mu)[Q], R omega, R Fx, R Fy,
                                                  R Fz, R (&lam)[Q], R& gFx, R& gFy, R& gFz)
{
    R A = R(0), Bx = R(0), By = R(0), Bz = R(0);
    R Cxx = R(0), Cyy = R(0), Czz = R(0), Cxy = R(0), Cxz = R(0), Cyz = R(0);
    sfor<0, Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const R mw = mu[q] * wq<R>(q);
        A += mw;
        if constexpr (cxq(q) != 0) Bx += R(cxq(q)) * mw;
        if constexpr (cyq(q) != 0) By += R(cyq(q)) * mw;
        if constexpr (czq(q) != 0) Bz += R(czq(q)) * mw;
        if constexpr (cxq(q) != 0) Cxx += mw;
        if constexpr (cyq(q) != 0) Cyy += mw;
        if constexpr (czq(q) != 0) Czz += mw;
        if constexpr (cxq(q) * cyq(q) != 0) Cxy += R(cxq(q) * cyq(q)) * mw;
        if constexpr (cxq(q) * czq(q) != 0) Cxz += R(cxq(q) * czq(q)) * mw;
        if constexpr (cyq(q) * czq(q) != 0) Cyz += R(cyq(q) * czq(q)) * mw;
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
    sfor<0, Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        R cg = R(0);
        if constexpr (cxq(q) != 0) cg += R(cxq(q)) * gux;
        if constexpr (cyq(q) != 0) cg += R(cyq(q)) * guy;
        if constexpr (czq(q) != 0) cg += R(czq(q)) * guz;
        lam[q] = omw * mu[q] + g_rho + (cg * inv - gdu);
    });
    const R i2 = R(0.5) * inv;
    gFx = kF * (R(3) * Bx - R(3) * A * ux + R(9) * Cux) + gux * i2;
    gFy = kF * (R(3) * By - R(3) * A * uy + R(9) * Cuy) + guy * i2;
    gFz = kF * (R(3) * Bz - R(3) * A * uz + R(9) * Cuz) + guz * i2;
}

// the same from the cell's distributions (offset form)
template <class R, bool FORCE>
__device__ __forceinline__ void collide_adjoint(const R (&g)[Q], const R (&mu)[Q], R omega, R Fx, R Fy, R Fz,
                                                R (&lam)[Q], R& gFx, R& gFy, R& gFz)
{
    const Moments<R> m = moments<R, FORCE>(g, Fx, Fy, Fz);
    collide_adjoint_m<R, FORCE>(m.rho, m.ux, m.uy, m.uz, mu, omega, Fx, Fy, Fz, lam, gFx, gFy, gFz);
}

}  // namespace lbm
