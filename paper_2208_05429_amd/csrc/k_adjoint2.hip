// k_adjoint2.hip -- the discrete adjoint of two merged time steps in one pass
// over memory: lambda_t from lambda_{t+2}, the state f_t and the force F, with
// the intermediate state f_{t+1} recomputed on chip.
//
// Two forward steps are f_{t+1} = S(C_t f_t), f_{t+2} = S(C_{t+1} f_{t+1}),
// so the adjoint is
//   lambda_{t+1} = C_{t+1}^T S^T lambda_{t+2},   lambda_t = C_t^T S^T lambda_{t+1},
// and dL/dF gains the force terms of both transposed collisions (adjoint_core.hpp).
//
// The transposed stream is itself a stream.  S^T pulls lambda along +c
// (mu_q(x) = lambda_q(x + c_q), or lambda_opp(q)(x) when the link leaves
// through a wall).  Relabelled as nu_p = lambda_opp(p), that is the forward
// push of nu with velocities c_p and the same halfway bounce-back (without a
// moving-wall term, which is constant).  So all three exchanges of a pass --
// the forward recompute f_t -> f_{t+1}, nu of lambda_{t+2} and nu of
// lambda_{t+1} -- run through the same receive machinery as the forward
// march (complete / deposit of march.hpp), three levels deep:
//
//   S1  plane P (front): collide f_t(P) on the tile plus a halo of two cells;
//       its post-collision values and nu(lambda_{t+2}(P)) enter the exchange;
//   S2  plane P-1 on the tile plus one halo cell: f_{t+1}(P-1) and
//       mu(P-1) = S^T lambda_{t+2} are complete; lambda_{t+1}(P-1) =
//       C_{t+1}^T mu enters the third exchange;
//   S3  plane P-2 on the tile: mu = S^T lambda_{t+1} is complete, and
//       lambda_t(P-2) = C_t^T mu (moments of f_t(P-2) kept from S1) is
//       written out, together with the force gradient of both steps.
//
// The output is a separate buffer, so workgroups are independent: any number
// of them, no co-residency and no progress counters.  Each owns a y-z tile
// and an x segment and starts two planes early to fill its pipeline.
// Bytes per cell and pass: f_t (19 s), lambda_{t+2} and lambda_t (2 x 19 x r),
// F (3 r) and the read-modify-write of dL/dF (6 r); 132 B per lattice update
// at FP32.
#include <atomic>

#include "adjoint_core.hpp"
#include "march.hpp"

namespace lbm {

// nu_p = v_opp(p): the relabelling between lambda and a forward-moving field
template <class LT, class R>
__device__ __forceinline__ void opp_relabel(const R (&src)[LT::Q], R (&dst)[LT::Q])
{
    sfor<0, LT::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        dst[q] = src[LT::opp(q)];
    });
}

template <int TY, int TZ>
struct Adj2Shape {
    static constexpr int WZ2 = TZ + 4, NC2 = (TY + 4) * WZ2;  // frame: tile plus two halo cells
    static constexpr int WZ1 = TZ + 2, NC1 = (TY + 2) * WZ1;  // tile plus one halo cell
};

template <int S, int TY, int TZ, int NT, bool WALLS, bool FORCE, class LT = D3Q19>
__global__ __launch_bounds__(NT) void k_adjoint2(Adj2Args a)
{
    using Cd = Codec<S>;
    using T = typename Cd::T;
    using R = typename Cd::R;
    using Sh = Adj2Shape<TY, TZ>;
    constexpr int WZ2 = Sh::WZ2, NC2 = Sh::NC2, WZ1 = Sh::WZ1, NC1 = Sh::NC1;
    static_assert(NC2 <= NT, "one frame column per thread");
    constexpr int QL = LT::Q;         // velocities
    constexpr int NYZ = nyz<LT>();    // those exchanged through LDS
    constexpr int NXP = nxp<LT>();    // those with c_x = +1, carried to the next plane
    constexpr int XP = LT::H + 1;     // the x-only direction (+1, 0, 0); (-1, 0, 0) is 1
    constexpr uint32_t CXP = mask_cx<LT>(1), CXM = mask_cx<LT>(-1);

    __shared__ R XF[NYZ * NC2];  // forward recompute: post-collision f_t
    __shared__ R XA[NYZ * NC2];  // nu of lambda_{t+2}
    __shared__ R XC[NYZ * NC1];  // nu of lambda_{t+1}
    __shared__ R WT[WALLS ? QL : 1];

    const Geom& g = a.g;
    const int tid = threadIdx.x;
    // Workgroup b runs on XCD b % 8; consecutive work items (z, then y
    // neighbours) go to the same XCD, so that a tile's halo and the parts of
    // the cache lines its frame rows share with the next tile are read from
    // that XCD's L2 rather than again from memory.
    const int per = gridDim.x >> 3;
    const int wid = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (wid >= a.items) return;  // padding of the grid
    const int tz = wid % a.ntz, ty = (wid / a.ntz) % a.nty, seg = wid / (a.ntz * a.nty);
    const int s = seg * a.seg_len, e = min(s + a.seg_len, g.nx);
    const int TYe = min(TY, g.ny - ty * TY), TZe = min(TZ, g.nz - tz * TZ);
    const bool wallx = g.wall[0] != 0;
    const R omega = R(g.omega);
    const long long N = g.N, PL = g.PL;
    if constexpr (WALLS) wall_terms_to_l<LT>(WT, tid, R(g.uw[0]), R(g.uw[1]), R(g.uw[2]));

    // ---- this thread's column of the frame ----
    const int c = tid;
    int gofs = -1, rad = 3, ci1 = 0;
    uint32_t byz = 0, myz = 0;
    if (c < NC2) {
        const int ly = c / WZ2, lz = c - (c / WZ2) * WZ2;
        if (ly < TYe + 4 && lz < TZe + 4) {
            const int dy = ly < 2 ? 2 - ly : (ly >= 2 + TYe ? ly - (2 + TYe) + 1 : 0);
            const int dz = lz < 2 ? 2 - lz : (lz >= 2 + TZe ? lz - (2 + TZe) + 1 : 0);
            int y = ty * TY - 2 + ly, z = tz * TZ - 2 + lz;
            bool inside = true;
            if (g.wall[1]) inside = inside && y >= 0 && y < g.ny;
            else y = wrapi(y, g.ny);
            if (g.wall[2]) inside = inside && z >= 0 && z < g.nz;
            else z = wrapi(z, g.nz);
            if (inside) {
                gofs = y * g.nz + z;
                rad = dy > dz ? dy : dz;
                ci1 = (ly - 1) * WZ1 + (lz - 1);
                if constexpr (WALLS) {
                    sfor<1, QL>([&](auto qc) {
                        constexpr int q = decltype(qc)::value;
                        if constexpr (moves_yz_l<LT>(q)) {
                            const int ys = y - LT::cy(q), zs = z - LT::cz(q);
                            int f1 = -1, f2 = -1;
                            if (g.wall[1] && ys < 0) f1 = 2;
                            if (g.wall[1] && ys >= g.ny) f1 = 3;
                            if (g.wall[2] && zs < 0) f2 = 4;
                            if (g.wall[2] && zs >= g.nz) f2 = 5;
                            if (f1 >= 0 || f2 >= 0) byz |= 1u << q;
                            if (g.moving_face >= 0 && (f1 == g.moving_face || f2 == g.moving_face)) myz |= 1u << q;
                        }
                    });
                }
            }
        }
    }
    const bool loads = rad <= 2 && gofs >= 0;
    const uint32_t loffT = loads ? uint32_t(gofs) * uint32_t(sizeof(T)) : kOffNone;
    const uint32_t loffR = loads ? uint32_t(gofs) * uint32_t(sizeof(R)) : kOffNone;
    const uint32_t ooffR = (rad == 0 && gofs >= 0) ? uint32_t(gofs) * uint32_t(sizeof(R)) : kOffNone;

    auto xb = [&](int p) -> uint32_t {
        if (!wallx) return 0u;
        return (p == 0 ? CXP : 0u) | (p == g.nx - 1 ? CXM : 0u);
    };
    auto xm = [&](int p) -> uint32_t {
        if (!wallx) return 0u;
        return ((p == 0 && g.moving_face == 0) ? CXP : 0u) | ((p == g.nx - 1 && g.moving_face == 1) ? CXM : 0u);
    };
    auto present = [&](int p) -> bool { return !wallx || (p >= 0 && p < g.nx); };

    // ---- registers of the three exchange levels and the histories ----
    T Lf[QL];  // raw f_t of the next plane
    R La[QL];  // lambda_{t+2} of the next plane
    R Fl[3] = {R(0), R(0), R(0)}, gFl[3] = {R(0), R(0), R(0)};
    R accA[QL], accB[QL], accC[QL], nxtA[NXP], nxtB[NXP], nxtC[NXP];
    R oA[3], oB[3], oC[3];
    R Fh1[3], Fh2[3], mh1[4], mh2[4], gFp[3];
#pragma unroll
    for (int q = 0; q < QL; ++q) {
        Lf[q] = T(0);
        La[q] = accA[q] = accB[q] = accC[q] = R(0);
    }
#pragma unroll
    for (int j = 0; j < NXP; ++j) nxtA[j] = nxtB[j] = nxtC[j] = R(0);
#pragma unroll
    for (int j = 0; j < 3; ++j) oA[j] = oB[j] = oC[j] = Fh1[j] = Fh2[j] = gFp[j] = R(0);
#pragma unroll
    for (int j = 0; j < 4; ++j) mh1[j] = mh2[j] = (j == 0 ? R(1) : R(0));

    const T* __restrict__ ft = static_cast<const T*>(a.ft);
    const R* __restrict__ F = static_cast<const R*>(a.F);
    const R* __restrict__ lin = static_cast<const R*>(a.lin);
    R* __restrict__ lout = static_cast<R*>(a.lout);
    R* __restrict__ gF = static_cast<R*>(a.gF);
    const uint32_t planeT = uint32_t(PL) * uint32_t(sizeof(T)), planeR = uint32_t(PL) * uint32_t(sizeof(R));

    // Loads of plane xp: f_t (issue_f), and lambda_{t+2}, F and the old dL/dF
    // of plane xp - 2, the plane the iteration that consumes them writes
    // (issue_l); issued unconditionally with an empty range where nothing is
    // wanted.  With two waves per SIMD the pass waits on memory, so each group
    // goes out as soon as its registers are free: lambda's once the current
    // plane's lambda has entered its exchange, before the collision (7 %
    // faster at 256^3 than issuing both after it).
    auto issue_f = [&](int xp, bool wanted) {
        const bool live = wanted && present(xp);
        const int px = wrapi(xp, g.nx);
        const T* bf = ft + (long long)px * PL;
#pragma unroll
        for (int q = 0; q < QL; ++q) {
            Lf[q] = Buf<T>::ld(make_rsrc(bf, live ? planeT : 0u), loffT);
            bf += N;
        }
    };
    auto issue_l = [&](int xp, bool wanted) {
        const bool live = wanted && present(xp);
        const int px = wrapi(xp, g.nx);
        const R* bl = lin + (long long)px * PL;
#pragma unroll
        for (int q = 0; q < QL; ++q) {
            La[q] = Buf<R>::ld(make_rsrc(bl, live ? planeR : 0u), loffR);
            bl += N;
        }
        if constexpr (FORCE) {
            const R* bF = F + (long long)px * PL;
            const int xo = xp - 2;
            const bool lo = wanted && gF != nullptr && xo >= s && xo < e && present(xo);
            const R* bG = gF + (long long)wrapi(xo, g.nx) * PL;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                Fl[k] = Buf<R>::ld(make_rsrc(bF, live ? planeR : 0u), loffR);
                gFl[k] = Buf<R>::ld(make_rsrc(bG, lo ? planeR : 0u), ooffR);
                bF += N;
                bG += N;
            }
        }
    };

    if constexpr (WALLS) __syncthreads();  // the wall-term table is complete
    const int total = (e - s) + 4;
    issue_f(s - 2, true);
    issue_l(s - 2, true);
    for (int i = 0; i < total; ++i) {
        const int P = s - 2 + i;

        // ---- S1: plane P enters the two outer exchanges ----
        R Fc[3], gFo[3], mc[4] = {R(1), R(0), R(0), R(0)};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            Fc[k] = Fl[k];
            gFo[k] = gFl[k];
        }
        const bool s1 = present(P) && loads;
        R v[QL];
        if (s1) {
#pragma unroll
            for (int q = 0; q < QL; ++q) v[q] = Cd::dec(Lf[q]);
            R nu[QL];
            opp_relabel<LT>(La, nu);
            sfor<0, QL>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                if constexpr (moves_yz_l<LT>(q)) XA[yz_index_l<LT>(q) * NC2 + c] = nu[q];
            });
            oB[0] = nu[0];
            oB[1] = nu[1];
            oB[2] = nu[XP];
        }
        issue_l(P + 1, i + 1 < total);
        if (s1) {
            const Moments<R> m = moments_l<R, FORCE, LT>(v, Fc[0], Fc[1], Fc[2]);
            mc[0] = m.rho;
            mc[1] = m.ux;
            mc[2] = m.uy;
            mc[3] = m.uz;
            LT::template collide<R, FORCE>(v, omega, Fc[0], Fc[1], Fc[2]);
            sfor<0, QL>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                if constexpr (moves_yz_l<LT>(q)) XF[yz_index_l<LT>(q) * NC2 + c] = v[q];
            });
            if constexpr (WALLS) moving_wall_out_l<LT>(v[1], v[XP], XF, NC2, c, myz | xm(P), WT);
            oA[0] = v[0];
            oA[1] = v[1];
            oA[2] = v[XP];
        }
        issue_f(P + 1, i + 1 < total);
        __syncthreads();

        // ---- S2: plane P-1 on the tile plus one cell: f_{t+1}, lambda_{t+1} ----
        R gFa[3] = {R(0), R(0), R(0)};
        if (rad <= 1 && gofs >= 0) {
            const uint32_t bd = byz | xb(P - 1), bn = byz | xb(P);
            complete<R, WALLS, LT>(accA, XF, NC2, c, WZ2, oA[1], bd);
            complete<R, WALLS, LT>(accB, XA, NC2, c, WZ2, oB[1], bd);
            if (present(P - 1)) {
                R mu[QL], lam[QL], nu[QL];
                opp_relabel<LT>(accB, mu);
                collide_adjoint<R, FORCE, LT>(accA, mu, omega, Fh1[0], Fh1[1], Fh1[2], lam, gFa[0], gFa[1], gFa[2]);
                opp_relabel<LT>(lam, nu);
                sfor<0, QL>([&](auto qc) {
                    constexpr int q = decltype(qc)::value;
                    if constexpr (moves_yz_l<LT>(q)) XC[yz_index_l<LT>(q) * NC1 + ci1] = nu[q];
                });
                oC[0] = nu[0];
                oC[1] = nu[1];
                oC[2] = nu[XP];
            }
            deposit<R, WALLS, LT>(accA, nxtA, XF, NC2, c, WZ2, oA[0], oA[1], oA[2], bn);
            deposit<R, WALLS, LT>(accB, nxtB, XA, NC2, c, WZ2, oB[0], oB[1], oB[2], bn);
        }
        __syncthreads();

        // ---- S3: plane P-2 on the tile: lambda_t and dL/dF ----
        const int po = P - 2;
        const bool out = po >= s && po < e && present(po);
        R lam0[QL], go[3];
#pragma unroll
        for (int q = 0; q < QL; ++q) lam0[q] = R(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) go[k] = R(0);
        if (rad == 0 && gofs >= 0) {
            complete<R, WALLS, LT>(accC, XC, NC1, ci1, WZ1, oC[1], byz | xb(po));
            if (out) {
                R mu[QL], gx, gy, gz;
                opp_relabel<LT>(accC, mu);
                collide_adjoint_m<R, FORCE, LT>(mh2[0], mh2[1], mh2[2], mh2[3], mu, omega, Fh2[0], Fh2[1], Fh2[2],
                                                lam0, gx, gy, gz);
                go[0] = gFo[0] + (gFp[0] + gx);
                go[1] = gFo[1] + (gFp[1] + gy);
                go[2] = gFo[2] + (gFp[2] + gz);
            }
            deposit<R, WALLS, LT>(accC, nxtC, XC, NC1, ci1, WZ1, oC[0], oC[1], oC[2], byz | xb(P - 1));
        }
        {
            const R* bq = lout + (long long)wrapi(po, g.nx) * PL;
#pragma unroll
            for (int q = 0; q < QL; ++q) {
                Buf<R>::st(lam0[q], make_rsrc(bq, out ? planeR : 0u), ooffR);
                bq += N;
            }
            if constexpr (FORCE) {
                const bool og = out && gF != nullptr;
                const R* bG = gF + (long long)wrapi(po, g.nx) * PL;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    Buf<R>::st(go[k], make_rsrc(bG, og ? planeR : 0u), ooffR);
                    bG += N;
                }
            }
        }

        // ---- histories move one plane ----
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            gFp[k] = gFa[k];
            Fh2[k] = Fh1[k];
            Fh1[k] = Fc[k];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            mh2[j] = mh1[j];
            mh1[j] = mc[j];
        }
    }
}

template <int S, int TY, int TZ, int NT, class LT = D3Q19>
static hipError_t adjoint2_shape(const Geom& g, const void* ft, const void* F, const void* lin, void* lout, void* gF,
                                 hipStream_t st)
{
    Adj2Args a;
    a.g = g;
    a.ft = ft;
    a.F = F;
    a.lin = lin;
    a.lout = lout;
    a.gF = gF;
    a.nty = (g.ny + TY - 1) / TY;
    a.ntz = (g.nz + TZ - 1) / TZ;
    const bool walls = g.wall[0] || g.wall[1] || g.wall[2];
    const bool force = F != nullptr;
    // Work items (tile, x segment) run in waves of `resident` workgroups, and
    // one item costs its segment length plus the 4 planes that fill its
    // pipeline.  Take the segment count that minimises waves x (length + 4).
    // The count is looked up once per device and kernel variant (walls,
    // force) and kept; concurrent first calls compute the same value.
    constexpr int kDevices = 64;
    static std::atomic<int> resident_of[kDevices][4];  // static storage: zero until looked up
    const int variant = (walls ? 2 : 0) + (force ? 1 : 0);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDevices) dev = -1;
    int resident = dev >= 0 ? resident_of[dev][variant].load(std::memory_order_relaxed) : 0;
    if (resident == 0) {
        int cus = 0, per = 0;
        auto k = walls ? (force ? k_adjoint2<S, TY, TZ, NT, true, true, LT> : k_adjoint2<S, TY, TZ, NT, true, false, LT>)
                       : (force ? k_adjoint2<S, TY, TZ, NT, false, true, LT> : k_adjoint2<S, TY, TZ, NT, false, false, LT>);
        if (dev >= 0 && hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, NT, 0) == hipSuccess && cus * per > 0)
            resident = cus * per;
        else
            resident = 256;
        if (dev >= 0) resident_of[dev][variant].store(resident, std::memory_order_relaxed);
    }
    const long long tiles = (long long)a.nty * a.ntz;
    long long best = -1;
    a.nseg = 1;
    a.seg_len = g.nx;
    for (int ns = 1; ns <= g.nx; ++ns) {
        const int len = (g.nx + ns - 1) / ns, n = (g.nx + len - 1) / len;
        if (n != ns) continue;  // the same split as a smaller count
        const long long cost = ((tiles * n + resident - 1) / resident) * (len + 4);
        if (best < 0 || cost < best) {
            best = cost;
            a.nseg = n;
            a.seg_len = len;
        }
    }
    a.items = int(tiles * a.nseg);
    const dim3 grid(unsigned((a.items + 7) / 8 * 8));
    if (walls) {
        if (force)
            hipLaunchKernelGGL((k_adjoint2<S, TY, TZ, NT, true, true, LT>), grid, dim3(NT), 0, st, a);
        else
            hipLaunchKernelGGL((k_adjoint2<S, TY, TZ, NT, true, false, LT>), grid, dim3(NT), 0, st, a);
    } else {
        if (force)
            hipLaunchKernelGGL((k_adjoint2<S, TY, TZ, NT, false, true, LT>), grid, dim3(NT), 0, st, a);
        else
            hipLaunchKernelGGL((k_adjoint2<S, TY, TZ, NT, false, false, LT>), grid, dim3(NT), 0, st, a);
    }
    return hipGetLastError();
}

// FP32 arithmetic (32- and 16-bit storage).  Each tile is one 512-thread
// workgroup per plane, so the plane takes the tiling with the fewest tiles of
// 12 x 28 (its 16 x 32 frame of tile plus two halo cells fills the workgroup
// exactly), 10 x 32 (a 14 x 36 frame; rows of 32 cells store whole cache
// lines) and 16 x 16, preferring them in that order on a tie.  Measured, per
// two-step call with walls and a force: 128 x 64 x 64 takes 14 tiles of
// 10 x 32 against 16 of 16 x 16 (0.080 against 0.095 ms); 256^2 planes 208 of
// 10 x 32 against 220 of 12 x 28 (level, 2.07 and 2.09 ms); 512^2 planes 817
// of 12 x 28 against 832 of 10 x 32 (16.3 against 18.4 ms).  The choice
// depends on the lattice only, so every storage takes the same tiles.
template <int S, class LT>
static hipError_t adjoint2_r32(const Geom& g, const void* f_t, const void* F, const void* lam_in, void* lam_out,
                               void* grad_force, hipStream_t s)
{
    const long long t1228 = (long long)((g.ny + 11) / 12) * ((g.nz + 27) / 28);
    const long long t1032 = (long long)((g.ny + 9) / 10) * ((g.nz + 31) / 32);
    const long long t1616 = (long long)((g.ny + 15) / 16) * ((g.nz + 15) / 16);
    if (t1228 <= t1032 && t1228 <= t1616)
        return adjoint2_shape<S, 12, 28, 512, LT>(g, f_t, F, lam_in, lam_out, grad_force, s);
    if (t1032 <= t1616) return adjoint2_shape<S, 10, 32, 512, LT>(g, f_t, F, lam_in, lam_out, grad_force, s);
    return adjoint2_shape<S, 16, 16, 512, LT>(g, f_t, F, lam_in, lam_out, grad_force, s);
}

template <class LT>
static hipError_t adjoint2_set(int storage, const Geom& g, const void* f_t, const void* F, const void* lam_in,
                               void* lam_out, void* grad_force, hipStream_t s)
{
    switch (storage) {
    // FP64 holds more than 256 registers per lane (one wave per SIMD), so a
    // workgroup is 256 threads; 8 x 16 tiles (a 12 x 20 frame, rows of 16
    // doubles: one cache line) did a two-step call 1.5-1.7x faster than 8 x 8
    // (128 x 64 x 64: 0.144 against 0.212 ms; 256^3: 4.80 against 8.10 ms;
    // 12 x 12: 0.170 and 5.10 ms).
    case ST_F64: return adjoint2_shape<ST_F64, 8, 16, 256, LT>(g, f_t, F, lam_in, lam_out, grad_force, s);
    case ST_F32: return adjoint2_r32<ST_F32, LT>(g, f_t, F, lam_in, lam_out, grad_force, s);
    case ST_F16: return adjoint2_r32<ST_F16, LT>(g, f_t, F, lam_in, lam_out, grad_force, s);
    case ST_BF16: return adjoint2_r32<ST_BF16, LT>(g, f_t, F, lam_in, lam_out, grad_force, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_step_adjoint2(int storage, const Geom& g, const void* f_t, const void* F, const void* lam_in,
                                void* lam_out, void* grad_force, hipStream_t s)
{
    if (g.lat == 15) return adjoint2_set<D3Q15>(storage, g, f_t, F, lam_in, lam_out, grad_force, s);
    if (g.lat == 27) return adjoint2_set<D3Q27>(storage, g, f_t, F, lam_in, lam_out, grad_force, s);
    return adjoint2_set<D3Q19>(storage, g, f_t, F, lam_in, lam_out, grad_force, s);
}

}  // namespace lbm
