// k_adjoint.hip -- discrete adjoint of the D3Q19 BGK step, one step per
// launch: the seed dL/df of a loss of the final velocity field, and
// lambda_t = C_t^T S^T lambda_{t+1} with the force gradient (the transposed
// collision is in adjoint_core.hpp; the two-step merged form in
// k_adjoint2.hip).
//
// One forward step is f_{t+1} = S(C(f_t; F)) with S the push streaming with
// bounce-back (a permutation plus a constant wall term) and C the per-cell
// collision.  S^T gathers mu_q(x) = lambda_q(x + c_q), or lambda_opp(q)(x)
// when the link leaves through a wall.
#include "adjoint_core.hpp"
#include "lbm_internal.hpp"

namespace lbm {

// lambda := dL/df from dL/du of the state f; gradF += dL/du / (2 rho)
template <int S, bool FORCE, class LT = D3Q19>
__global__ __launch_bounds__(256) void k_macro_adjoint(Geom g, const typename Codec<S>::T* __restrict__ f,
                                                       const typename Codec<S>::R* __restrict__ F,
                                                       const typename Codec<S>::R* __restrict__ gu,
                                                       typename Codec<S>::R* __restrict__ lam,
                                                       typename Codec<S>::R* __restrict__ gF)
{
    using Cd = Codec<S>;
    using R = typename Cd::R;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= g.N) return;
    constexpr int QL = LT::Q;
    R v[QL];
#pragma unroll
    for (int q = 0; q < QL; ++q) v[q] = Cd::dec(f[q * g.N + i]);
    R Fx = R(0), Fy = R(0), Fz = R(0);
    if constexpr (FORCE) {
        Fx = F[i];
        Fy = F[g.N + i];
        Fz = F[2 * g.N + i];
    }
    const Moments<R> m = moments_l<R, FORCE, LT>(v, Fx, Fy, Fz);
    const R inv = R(1) / m.rho;
    const R gx = gu[i], gy = gu[g.N + i], gz = gu[2 * g.N + i];
    const R gdu = gx * m.ux + gy * m.uy + gz * m.uz;
    sfor<0, QL>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        R cg = R(0);
        if constexpr (LT::cx(q) != 0) cg += R(LT::cx(q)) * gx;
        if constexpr (LT::cy(q) != 0) cg += R(LT::cy(q)) * gy;
        if constexpr (LT::cz(q) != 0) cg += R(LT::cz(q)) * gz;
        lam[q * g.N + i] = (cg - gdu) * inv;
    });
    if (gF) {
        const R h = R(0.5) * inv;
        gF[i] += gx * h;
        gF[g.N + i] += gy * h;
        gF[2 * g.N + i] += gz * h;
    }
}

// mu_q(x): lambda_q at the target of the link (x, q), or lambda_opp(q)(x) when
// the link leaves through a wall face
template <class R, bool WALLS, class LT = D3Q19>
__device__ __forceinline__ void stream_adjoint_gather(const Geom& g, const R* __restrict__ lin, int x, int y, int z,
                                                      long long i, R (&mu)[LT::Q])
{
    const int n[3] = {g.nx, g.ny, g.nz};
    sfor<0, LT::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const int c[3] = {LT::cx(q), LT::cy(q), LT::cz(q)};
        int p[3] = {x + c[0], y + c[1], z + c[2]};
        bool out = false;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            if (c[ax] == 0 || (p[ax] >= 0 && p[ax] < n[ax])) continue;
            if (WALLS && g.wall[ax])
                out = true;
            else
                p[ax] = p[ax] < 0 ? p[ax] + n[ax] : p[ax] - n[ax];
        }
        if (WALLS && out)
            mu[q] = lin[LT::opp(q) * g.N + i];
        else
            mu[q] = lin[q * g.N + ((long long)p[0] * g.ny + p[1]) * g.nz + p[2]];
    });
}

// one reverse step: lam_out = adjoint of one step at f_t applied to lam_in
template <int S, bool WALLS, bool FORCE, class LT = D3Q19>
__global__ __launch_bounds__(256) void k_adjoint1(Geom g, const typename Codec<S>::T* __restrict__ ft,
                                                  const typename Codec<S>::R* __restrict__ F,
                                                  const typename Codec<S>::R* __restrict__ lin,
                                                  typename Codec<S>::R* __restrict__ lout,
                                                  typename Codec<S>::R* __restrict__ gF)
{
    using Cd = Codec<S>;
    using R = typename Cd::R;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= g.N) return;
    const int z = int(i % g.nz);
    const long long r = i / g.nz;
    const int y = int(r % g.ny), x = int(r / g.ny);
    constexpr int QL = LT::Q;
    R mu[QL], v[QL], lam[QL];
    stream_adjoint_gather<R, WALLS, LT>(g, lin, x, y, z, i, mu);
#pragma unroll
    for (int q = 0; q < QL; ++q) v[q] = Cd::dec(ft[q * g.N + i]);
    R Fx = R(0), Fy = R(0), Fz = R(0);
    if constexpr (FORCE) {
        Fx = F[i];
        Fy = F[g.N + i];
        Fz = F[2 * g.N + i];
    }
    R gx, gy, gz;
    collide_adjoint<R, FORCE, LT>(v, mu, R(g.omega), Fx, Fy, Fz, lam, gx, gy, gz);
#pragma unroll
    for (int q = 0; q < QL; ++q) lout[q * g.N + i] = lam[q];
    if (FORCE && gF) {
        gF[i] += gx;
        gF[g.N + i] += gy;
        gF[2 * g.N + i] += gz;
    }
}

template <int S, bool FORCE, class LT = D3Q19>
static hipError_t macro_adjoint_s(const Geom& g, const void* f, const void* F, const void* gu, void* lam, void* gF,
                                  hipStream_t s)
{
    using Cd = Codec<S>;
    using R = typename Cd::R;
    hipLaunchKernelGGL((k_macro_adjoint<S, FORCE, LT>), dim3(unsigned((g.N + 255) / 256)), dim3(256), 0, s, g,
                       static_cast<const typename Cd::T*>(f), static_cast<const R*>(F), static_cast<const R*>(gu),
                       static_cast<R*>(lam), static_cast<R*>(gF));
    return hipGetLastError();
}

template <class LT>
static hipError_t macro_adjoint_set(int storage, bool force, const Geom& g, const void* f, const void* F,
                                    const void* grad_u, void* lambda, void* grad_force, hipStream_t s)
{
    switch (storage) {
    case ST_F64:
        return force ? macro_adjoint_s<ST_F64, true, LT>(g, f, F, grad_u, lambda, grad_force, s)
                     : macro_adjoint_s<ST_F64, false, LT>(g, f, F, grad_u, lambda, grad_force, s);
    case ST_F32:
        return force ? macro_adjoint_s<ST_F32, true, LT>(g, f, F, grad_u, lambda, grad_force, s)
                     : macro_adjoint_s<ST_F32, false, LT>(g, f, F, grad_u, lambda, grad_force, s);
    case ST_F16:
        return force ? macro_adjoint_s<ST_F16, true, LT>(g, f, F, grad_u, lambda, grad_force, s)
                     : macro_adjoint_s<ST_F16, false, LT>(g, f, F, grad_u, lambda, grad_force, s);
    case ST_BF16:
        return force ? macro_adjoint_s<ST_BF16, true, LT>(g, f, F, grad_u, lambda, grad_force, s)
                     : macro_adjoint_s<ST_BF16, false, LT>(g, f, F, grad_u, lambda, grad_force, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_macro_adjoint(int storage, bool force, const Geom& g, const void* f, const void* F,
                                const void* grad_u, void* lambda, void* grad_force, hipStream_t s)
{
    if (g.lat == 15) return macro_adjoint_set<D3Q15>(storage, force, g, f, F, grad_u, lambda, grad_force, s);
    if (g.lat == 27) return macro_adjoint_set<D3Q27>(storage, force, g, f, F, grad_u, lambda, grad_force, s);
    switch (storage) {
    case ST_F64:
        return force ? macro_adjoint_s<ST_F64, true>(g, f, F, grad_u, lambda, grad_force, s)
                     : macro_adjoint_s<ST_F64, false>(g, f, F, grad_u, lambda, grad_force, s);
    case ST_F32:
        return force ? macro_adjoint_s<ST_F32, true>(g, f, F, grad_u, lambda, grad_force, s)
                     : macro_adjoint_s<ST_F32, false>(g, f, F, grad_u, lambda, grad_force, s);
    case ST_F16:
        return force ? macro_adjoint_s<ST_F16, true>(g, f, F, grad_u, lambda, grad_force, s)
                     : macro_adjoint_s<ST_F16, false>(g, f, F, grad_u, lambda, grad_force, s);
    case ST_BF16:
        return force ? macro_adjoint_s<ST_BF16, true>(g, f, F, grad_u, lambda, grad_force, s)
                     : macro_adjoint_s<ST_BF16, false>(g, f, F, grad_u, lambda, grad_force, s);
    }
    return hipErrorInvalidValue;
}

template <int S, bool FORCE, class LT = D3Q19>
static hipError_t adjoint1_s(const Geom& g, const void* ft, const void* F, const void* lin, void* lout, void* gF,
                             hipStream_t s)
{
    using Cd = Codec<S>;
    using R = typename Cd::R;
    const bool walls = g.wall[0] || g.wall[1] || g.wall[2];
    auto fp = static_cast<const typename Cd::T*>(ft);
    auto Fp = static_cast<const R*>(F);
    auto li = static_cast<const R*>(lin);
    auto lo = static_cast<R*>(lout);
    auto gp = static_cast<R*>(gF);
    const dim3 grid(unsigned((g.N + 255) / 256));
    if (walls)
        hipLaunchKernelGGL((k_adjoint1<S, true, FORCE, LT>), grid, dim3(256), 0, s, g, fp, Fp, li, lo, gp);
    else
        hipLaunchKernelGGL((k_adjoint1<S, false, FORCE, LT>), grid, dim3(256), 0, s, g, fp, Fp, li, lo, gp);
    return hipGetLastError();
}

template <class LT>
static hipError_t adjoint1_set(int storage, bool force, const Geom& g, const void* f_t, const void* F,
                               const void* lam_in, void* lam_out, void* grad_force, hipStream_t s)
{
    switch (storage) {
    case ST_F64:
        return force ? adjoint1_s<ST_F64, true, LT>(g, f_t, F, lam_in, lam_out, grad_force, s)
                     : adjoint1_s<ST_F64, false, LT>(g, f_t, F, lam_in, lam_out, grad_force, s);
    case ST_F32:
        return force ? adjoint1_s<ST_F32, true, LT>(g, f_t, F, lam_in, lam_out, grad_force, s)
                     : adjoint1_s<ST_F32, false, LT>(g, f_t, F, lam_in, lam_out, grad_force, s);
    case ST_F16:
        return force ? adjoint1_s<ST_F16, true, LT>(g, f_t, F, lam_in, lam_out, grad_force, s)
                     : adjoint1_s<ST_F16, false, LT>(g, f_t, F, lam_in, lam_out, grad_force, s);
    case ST_BF16:
        return force ? adjoint1_s<ST_BF16, true, LT>(g, f_t, F, lam_in, lam_out, grad_force, s)
                     : adjoint1_s<ST_BF16, false, LT>(g, f_t, F, lam_in, lam_out, grad_force, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_step_adjoint(int storage, bool force, int k, const Geom& g, const void* f_t, const void* F,
                               const void* lam_in, void* lam_out, void* grad_force, hipStream_t s)
{
    if (k == 2) return launch_step_adjoint2(storage, g, f_t, force ? F : nullptr, lam_in, lam_out, grad_force, s);
    if (g.lat != 19) {
        if (k != 1) return hipErrorInvalidValue;
        return g.lat == 15 ? adjoint1_set<D3Q15>(storage, force, g, f_t, F, lam_in, lam_out, grad_force, s)
                           : adjoint1_set<D3Q27>(storage, force, g, f_t, F, lam_in, lam_out, grad_force, s);
    }
    if (k != 1) return hipErrorInvalidValue;
    switch (storage) {
    case ST_F64:
        return force ? adjoint1_s<ST_F64, true>(g, f_t, F, lam_in, lam_out, grad_force, s)
                     : adjoint1_s<ST_F64, false>(g, f_t, F, lam_in, lam_out, grad_force, s);
    case ST_F32:
        return force ? adjoint1_s<ST_F32, true>(g, f_t, F, lam_in, lam_out, grad_force, s)
                     : adjoint1_s<ST_F32, false>(g, f_t, F, lam_in, lam_out, grad_force, s);
    case ST_F16:
        return force ? adjoint1_s<ST_F16, true>(g, f_t, F, lam_in, lam_out, grad_force, s)
                     : adjoint1_s<ST_F16, false>(g, f_t, F, lam_in, lam_out, grad_force, s);
    case ST_BF16:
        return force ? adjoint1_s<ST_BF16, true>(g, f_t, F, lam_in, lam_out, grad_force, s)
                     : adjoint1_s<ST_BF16, false>(g, f_t, F, lam_in, lam_out, grad_force, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lbm
