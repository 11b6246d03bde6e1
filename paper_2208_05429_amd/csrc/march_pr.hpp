// march_pr.hpp -- the marching in-place update of march.hpp laid out for
// 32-bit arithmetic on CDNA4: every thread owns one pair of z-adjacent
// interior columns of its tile and at most one column of the halo ring.
//
// Why this layout.  The interior of a TY x TZ tile is exactly TY*TZ/2 pairs, so
// the interior loads and the in-place stores of a direction are 8-byte-per-
// lane accesses that cover whole cache lines (a wave reads or writes two
// rows of 64 floats), and a thread issues 19 pair loads + 19 ring loads + 19
// pair stores per plane: fewer than the 63 vector-memory operations a wave
// may have in flight, so no store ever waits for the prefetch (with a body
// force, 18 force loads come on top).  Ring columns
// (halo of width M) are never stored and never receive the last step, so
// they carry no last-step pipeline registers.
//
// Pipeline of one iteration (load front at plane xl), as in march.hpp:
//   A  step-1 collide of plane xl (pair and ring), each column's loads of
//      plane xl+1 issued right after its collide;
//   |  barrier, publish the load front;
//   E  (M = 2) step-1 receive (completes plane xl-1 at t+1) and step-2
//      collide of that plane on the tile plus one halo cell;  | barrier;
//   D  receive of the last step: completes plane xl-M (time t+M) for the
//      pair; each wave checks the neighbours' progress counters (read at the
//      start of the iteration) and stores the pair in place.
// The hazard protocol, the side planes of the segment ends and the boundary
// rules are those of march.hpp.
#pragma once

#include "march.hpp"

namespace lbm {

// Two z-adjacent values of one direction, moved as one access: 8 bytes for
// 32-bit storage, 4 bytes for 16-bit storage.  P is how a loaded pair waits in
// registers until it is decoded: two floats, or both 16-bit codes packed in
// one register (half the registers for a plane of loads in flight).
template <class T>
struct Buf2;
template <>
struct Buf2<float> {
    struct P {
        float a, b;
    };
    static __device__ __forceinline__ P ld(__amdgpu_buffer_rsrc_t r, uint32_t off)
    {
        auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
        return P{__uint_as_float(v[0]), __uint_as_float(v[1])};
    }
    static __device__ __forceinline__ P zero() { return P{0.0f, 0.0f}; }
    template <int K>
    static __device__ __forceinline__ float get(P p)
    {
        return K == 0 ? p.a : p.b;
    }
    // AUX: the store's cache policy (0, or 2 for non-temporal)
    template <int AUX = 0>
    static __device__ __forceinline__ void st(float a, float b, __amdgpu_buffer_rsrc_t r, uint32_t off)
    {
        typedef unsigned int u2 __attribute__((ext_vector_type(2)));
        u2 w;
        w[0] = __float_as_uint(a);
        w[1] = __float_as_uint(b);
        __builtin_amdgcn_raw_buffer_store_b64(w, r, off, 0, AUX);
    }
};
template <>
struct Buf2<uint16_t> {
    typedef uint32_t P;
    static __device__ __forceinline__ P ld(__amdgpu_buffer_rsrc_t r, uint32_t off)
    {
        return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
    }
    static __device__ __forceinline__ P zero() { return 0u; }
    template <int K>
    static __device__ __forceinline__ uint16_t get(P p)
    {
        return K == 0 ? uint16_t(p & 0xffffu) : uint16_t(p >> 16);
    }
    // both codes already packed (Codec::enc2)
    template <int AUX = 0>
    static __device__ __forceinline__ void st(uint32_t w, __amdgpu_buffer_rsrc_t r, uint32_t off)
    {
        __builtin_amdgcn_raw_buffer_store_b32(w, r, off, 0, AUX);
    }
};

// Exchange buffers are split by column parity: column c of a row-major grid
// with an even row length lives at (c & 1) * (size / 2) + (c >> 1), so the
// lanes of a wave, which own consecutive pairs, touch consecutive words
// (a plain row-major buffer would give stride-2 bank conflicts).  PAR is the
// parity of the column when known at compile time (pair columns), -1 else.
template <int PAR, int HALF>
__device__ __forceinline__ int split_at(int c, int d)
{
    if constexpr (PAR >= 0) {
        const int t = PAR + d;  // d is a compile-time constant at every call site
        return ((t & 1) ? HALF : 0) + (c >> 1) + (t >> 1);
    } else {
        const int cc = c + d;
        return ((cc & 1) ? HALF : 0) + (cc >> 1);
    }
}

// complete() / deposit() of march.hpp on a parity-split buffer of 16 rows of
// STRIDE columns with row pitch WZL, with walls handled through ghost slots.
//
// Walls in y and z.  A population whose source lies beyond a y/z wall is the
// receiving cell's own reversed post-collision value (plus the moving-wall
// term).  The receiver itself writes that value into the exchange slot it is
// about to pull from: the slot of an out-of-domain position, which no other
// cell reads or writes.  The pulls are then the periodic ones, unchanged:
//   c_x = 0   ghost written right after the collision (ghost_out);
//   c_x = +1  the pending value in nxt[] is replaced right after the
//             collision (ghost_out);
//   c_x = -1  pulled one iteration later from the next plane's exchange:
//             ghost written at deposit time, into the buffer that plane will
//             use (Xg), where it survives because collisions write only slots
//             of cells inside the domain.
// Lanes without such a link write to a sink at the end of the buffer
// instead of branching.
// Walls in x are uniform over a plane (xw: the receiving directions of this
// plane whose source plane is beyond an x wall): deposit puts the reversed
// values in place and complete keeps them.
// A copy of v the compiler cannot see through: keeps a computation that
// depends on it inside the loop instead of hoisted (and kept live) outside.
__device__ __forceinline__ int opaque(int v)
{
    asm volatile("" : "+v"(v));
    return v;
}

template <class R, bool WALLS, int PAR, int STRIDE, int WZL, class LT = D3Q19>
__device__ __forceinline__ void complete_s(R (&acc)[LT::Q], const R* __restrict__ X, int ci, R o1, uint32_t xw)
{
    constexpr int HALF = STRIDE / 2;
    // next to an x wall (uniform over the plane) every c_x = -1 population was
    // put in place by deposit_s, and there is nothing to receive
    if (WALLS && (xw & mask_cx<LT>(-1)) != 0u) return;
    sfor<0, LT::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        if constexpr (LT::cx(q) == -1) {
            if constexpr (moves_yz_l<LT>(q))
                acc[q] = X[yz_index_l<LT>(q) * STRIDE + split_at<PAR, HALF>(ci, -LT::cy(q) * WZL - LT::cz(q))];
            else
                acc[q] = o1;
        }
    });
}

// own reversed post-collision value of direction q (its opposite's slot)
template <class R, int PAR, int STRIDE, int q, class LT = D3Q19>
__device__ __forceinline__ R own_reversed(const R* __restrict__ X, int ci, R o1, R o10)
{
    constexpr int qo = LT::opp(q);
    if constexpr (moves_yz_l<LT>(qo))
        return X[yz_index_l<LT>(qo) * STRIDE + split_at<PAR, STRIDE / 2>(ci, 0)];
    else
        return (qo == 1) ? o1 : o10;
}

template <class R, bool WALLS, int PAR, int STRIDE, int WZL, class LT = D3Q19>
__device__ __forceinline__ void deposit_s(R (&acc)[LT::Q], R (&nxt)[nxp<LT>()], R* __restrict__ X, int ci, R o0, R o1, R o10,
                                          uint32_t xw, uint32_t byz, uint32_t mv, const R* WT, R* Xg, int lane)
{
    constexpr int HALF = STRIDE / 2;
    sfor<0, LT::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        if constexpr (LT::cx(q) == 0) {
            if constexpr (q == 0)
                acc[q] = o0;
            else
                acc[q] = X[yz_index_l<LT>(q) * STRIDE + split_at<PAR, HALF>(ci, -LT::cy(q) * WZL - LT::cz(q))];
        } else if constexpr (LT::cx(q) == 1) {
            constexpr int j = xp_index_l<LT>(q);
            acc[q] = nxt[j];
            if constexpr (moves_yz_l<LT>(q))
                nxt[j] = X[yz_index_l<LT>(q) * STRIDE + split_at<PAR, HALF>(ci, -LT::cy(q) * WZL - LT::cz(q))];
            else
                nxt[j] = o10;
        }
    });
    if constexpr (WALLS) {
        if (xw != 0u) {  // a plane next to an x wall (uniform)
            const int cio = opaque(ci);
            sfor<1, LT::Q>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                if constexpr (LT::cx(q) != 0) {
                    if ((xw >> q) & 1u) {
                        const R own = own_reversed<R, PAR, STRIDE, q, LT>(X, cio, o1, o10);
                        acc[q] = ((mv >> q) & 1u) ? own + WT[opaque(q)] : own;
                    }
                }
            });
        }
        if (__any(byz != 0u)) {  // c_x = -1 ghosts for the next plane's completion
            const int cio = opaque(ci), sk = opaque(nyz<LT>() * STRIDE + lane);
            sfor<1, LT::Q>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                if constexpr (LT::cx(q) == -1 && moves_yz_l<LT>(q)) {
                    const bool hit = (byz >> q) & 1u;
                    const R own = own_reversed<R, PAR, STRIDE, q, LT>(X, cio, o1, o10);
                    const int gi = yz_index_l<LT>(q) * STRIDE + split_at<PAR, HALF>(cio, -LT::cy(q) * WZL - LT::cz(q));
                    Xg[hit ? gi : sk] = ((mv >> q) & 1u) ? own + WT[opaque(q)] : own;
                }
            });
        }
    }
}

// Right after a receiving cell's collision (v: its post-collision values,
// already written to its own slots): c_x = 0 ghosts and c_x = +1 replacements.
template <class R, int PAR, int STRIDE, int WZL, class LT = D3Q19>
__device__ __forceinline__ void ghost_out(const R (&v)[LT::Q], R (&nxt)[nxp<LT>()], R* __restrict__ X, int ci, uint32_t byz,
                                          uint32_t myz, const R* WT, int lane)
{
    constexpr int HALF = STRIDE / 2;
    if (!__any(byz != 0u)) return;
    const int cio = opaque(ci), sk = opaque(nyz<LT>() * STRIDE + lane);
    sfor<1, LT::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        if constexpr (moves_yz_l<LT>(q) && LT::cx(q) >= 0) {
            const bool hit = (byz >> q) & 1u;
            const R val = ((myz >> q) & 1u) ? v[LT::opp(q)] + WT[opaque(q)] : v[LT::opp(q)];
            if constexpr (LT::cx(q) == 0) {
                const int gi = yz_index_l<LT>(q) * STRIDE + split_at<PAR, HALF>(cio, -LT::cy(q) * WZL - LT::cz(q));
                X[hit ? gi : sk] = val;
            } else {
                nxt[xp_index_l<LT>(q)] = hit ? val : nxt[xp_index_l<LT>(q)];
            }
        }
    });
}

template <int M, int TY, int TZ>
struct PairRingShape {
    static constexpr int WY = TY + 2 * M, WZ = TZ + 2 * M, NC = WY * WZ;
    static constexpr int NT = TY * TZ / 2;  // one interior pair per thread
    static constexpr int RING = NC - TY * TZ;
    static constexpr int WZ2 = TZ + 2, NC2 = (TY + 2) * WZ2;
    // The ring in rounds (bands of tile rows): rows below the tile, the side
    // columns and rows above each fill whole waves, so that the source of a
    // wave's ring loads (the lattice or a saved band boundary) is uniform.
    static constexpr int B1 = (M * WZ + 63) / 64 * 64;               // side columns start
    static constexpr int B2 = (B1 + TY * 2 * M + 63) / 64 * 64;      // rows above start
    static constexpr int RINGB = B2 + M * WZ;
    static_assert(TZ % 2 == 0, "pairs need an even tile width");
    static_assert(RING <= NT, "at most one ring column per thread");
    static_assert(RINGB <= NT, "the banded ring layout fits the workgroup");
};

// local (ly, lz) of ring slot r: rows below the tile, side columns, rows
// above, row-major; in rounds each part starts on a wave boundary (slots in
// between are empty: returns false)
template <int M, int TY, int TZ>
__device__ __forceinline__ bool ring_cell(int r, bool banded, int& ly, int& lz)
{
    using Sh = PairRingShape<M, TY, TZ>;
    constexpr int WZ = TZ + 2 * M;
    const int b1 = banded ? Sh::B1 : M * WZ, b2 = banded ? Sh::B2 : M * WZ + TY * 2 * M;
    if (r < M * WZ) {
        ly = r / WZ;
        lz = r - ly * WZ;
        return true;
    }
    if (r >= b1 && r < b1 + TY * 2 * M) {
        const int rr = r - b1;
        ly = M + rr / (2 * M);
        const int k = rr - (rr / (2 * M)) * (2 * M);
        lz = k < M ? k : TZ + k;
        return true;
    }
    if (r >= b2 && r < b2 + M * WZ) {
        const int rr = r - b2;
        ly = M + TY + rr / WZ;
        lz = rr - (rr / WZ) * WZ;
        return true;
    }
    return false;
}

template <int S, int M, int TY, int TZ, bool WALLS, bool FORCE, int PF, class LT = D3Q19>
__global__ __launch_bounds__(TY * TZ / 2) void k_march_pr(MarchArgs a)
{
    constexpr int QL = LT::Q;        // velocities
    constexpr int NYZ = nyz<LT>();   // those exchanged through LDS
    constexpr int NXP = nxp<LT>();   // those with c_x = +1
    constexpr int XP = LT::H + 1;    // the x-only direction (+1, 0, 0)
    using Cd = Codec<S>;
    using T = typename Cd::T;
    using R = typename Cd::R;
    using Sh = PairRingShape<M, TY, TZ>;
    constexpr int WZ = Sh::WZ, NC = Sh::NC, WZ2 = Sh::WZ2, NC2 = Sh::NC2;
    constexpr int NB1 = (M == 1) ? 2 : 1;
    constexpr uint32_t CXP = mask_cx<LT>(1), CXM = mask_cx<LT>(-1);
    static_assert(M == 1 || M == 2, "one or two merged steps");
    static_assert(sizeof(T) == 2 || sizeof(T) == 4, "32-bit arithmetic storages");
    static_assert(PF == 1 || PF == 2, "loads run one or two planes ahead");

    constexpr int SK = WALLS ? 64 : 0;  // each exchange buffer ends in a sink for ghost writes of lanes without a wall link
    __shared__ R X1[NB1][NYZ * NC + SK];
    __shared__ R X2[(M == 2) ? NYZ * NC2 + SK : 1];
    __shared__ R WT[WALLS ? QL : 1];  // moving-wall terms (entry q: received along c_q)

    const Geom& g = a.g;
    const int tid = threadIdx.x;
    int wid = blockIdx.x;
    if (a.xcd_remap) {
        const int per = gridDim.x >> 3;
        wid = (wid & 7) * per + (wid >> 3);
    }
    if (wid >= a.items) return;  // padding of the grid (uniform per workgroup, before any barrier)
    const bool banded = a.nty_band < a.nty;
    int tz, ty, seg;
    tile_of_item<TZ>(wid, a.nty_band, a.ntz, tz, ty, seg);
    ty += a.band_ty0;
    const long long gtile = ((long long)seg * a.nty + ty) * a.ntz + tz;  // progress counter index
    const int s = seg * a.seg_len, e = min(s + a.seg_len, g.nx);
    const int TYe = min(TY, g.ny - ty * TY), TZe = min(TZ, g.nz - tz * TZ);
    const bool wallx = g.wall[0] != 0;
    const bool has_next = !wallx || seg + 1 < a.nseg;
    const int nseg_next = (seg + 1 == a.nseg) ? 0 : seg + 1;
    const R omega = R(g.omega);
    if constexpr (WALLS) wall_terms_to_l<LT>(WT, tid, R(g.uw[0]), R(g.uw[1]), R(g.uw[2]));
    // receiving directions whose source lies beyond the moving face, for a
    // cell next to it (y or z face; an x face is handled per plane by xm)
    uint32_t mface = 0u;
    if constexpr (WALLS) {
        sfor<1, QL>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            const int f = g.moving_face;
            if ((f == 2 && LT::cy(q) == 1) || (f == 3 && LT::cy(q) == -1) || (f == 4 && LT::cz(q) == 1) ||
                (f == 5 && LT::cz(q) == -1))
                mface |= 1u << q;
        });
    }
    // moving-wall links of a column (its bounce mask with the bit-31 flag)
    auto mlinks = [&](uint32_t b) -> uint32_t { return (b >> 31) ? (b & mface) : 0u; };
    const int lane = tid & 63;
    const long long N = g.N, PL = g.PL;

    // ---- the three columns of this thread: 0, 1 = interior pair, 2 = ring ----
    constexpr int K = 3;
    int gofs[K], rad[K], ci[K], ci2[K];
    uint32_t voff[K], byz[K];
    uint32_t shoff = kOffNone;  // ring column in a band boundary copy: (row * nz + z) * sizeof(T)
#pragma unroll
    for (int k = 0; k < K; ++k) {
        gofs[k] = -1;
        rad[k] = M + 1;
        ci[k] = 0;
        ci2[k] = 0;
        voff[k] = kOffNone;
        byz[k] = 0;
        int ly = 0, lz = 0;
        bool have = true;
        if (k < 2) {
            ly = M + tid / (TZ / 2);
            lz = M + 2 * (tid - (tid / (TZ / 2)) * (TZ / 2)) + k;
        } else {
            have = ring_cell<M, TY, TZ>(tid, banded, ly, lz);
        }
        if (!have) continue;
        ci[k] = ly * WZ + lz;
        if (ly >= TYe + 2 * M || lz >= TZe + 2 * M) continue;
        const int dy = ly < M ? M - ly : (ly >= M + TYe ? ly - (M + TYe) + 1 : 0);
        const int dz = lz < M ? M - lz : (lz >= M + TZe ? lz - (M + TZe) + 1 : 0);
        int y = ty * TY - M + ly, z = tz * TZ - M + lz;
        bool inside = true;
        if (g.wall[1]) inside = inside && y >= 0 && y < g.ny;
        else y = wrapi(y, g.ny);
        if (g.wall[2]) inside = inside && z >= 0 && z < g.nz;
        else z = wrapi(z, g.nz);
        if (!inside) continue;
        gofs[k] = y * g.nz + z;
        voff[k] = uint32_t(gofs[k]) * uint32_t(sizeof(T));
        rad[k] = dy > dz ? dy : dz;
        ci2[k] = (ly - 1) * WZ2 + (lz - 1);
        if (k == 2 && (ly < M || ly >= M + TYe)) {
            const int row = ly < M ? ly : ly - (M + TYe);
            shoff = uint32_t(row * g.nz + z) * uint32_t(sizeof(T));
        }
        if constexpr (WALLS) {
            uint32_t b = 0, mv = 0;
            sfor<1, QL>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                if constexpr (moves_yz_l<LT>(q)) {
                    const int ys = y - LT::cy(q), zs = z - LT::cz(q);
                    int f1 = -1, f2 = -1;
                    if (g.wall[1] && ys < 0) f1 = 2;
                    if (g.wall[1] && ys >= g.ny) f1 = 3;
                    if (g.wall[2] && zs < 0) f2 = 4;
                    if (g.wall[2] && zs >= g.nz) f2 = 5;
                    if (f1 >= 0 || f2 >= 0) b |= 1u << q;
                    if (g.moving_face >= 0 && (f1 == g.moving_face || f2 == g.moving_face)) mv |= 1u << q;
                }
            });
            // bit 31: the column touches the moving face; its moving-wall links
            // are then exactly byz & mface (mface below, uniform)
            byz[k] = b | (mv ? 0x80000000u : 0u);
        }
    }
    // Inside the march a column counts as present through rad alone (rad <= M
    // only for columns in the domain), and the second pair column's indices
    // follow from the first: fewer registers live across the march.
    ci[1] = ci[0] + 1;
    ci2[1] = ci2[0] + 1;
    // memory offsets: the pair moves as one access keyed on its first column
    // (a pair starts at an even z of an even-length row, so it never wraps)
    const bool pair_loads = rad[0] <= M && gofs[0] >= 0;
    const uint32_t loffP = pair_loads ? voff[0] : kOffNone;
    const uint32_t soffP = (rad[0] == 0 && gofs[0] >= 0) ? voff[0] : kOffNone;
    // in a round, a wave of ring rows below (above) the band reads the saved
    // boundary rows of the band there when that band was already updated
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const T* shell_w = nullptr;
    if (banded) {  // only the band's first (last) row of tiles borders the band below (above)
        if (wave < Sh::B1 / 64 && ty == a.band_ty0) shell_w = static_cast<const T*>(a.shell_lo);
        else if (wave >= Sh::B2 / 64 && ty == a.band_ty0 + a.nty_band - 1) shell_w = static_cast<const T*>(a.shell_hi);
    }
    const bool ring_loads = rad[2] <= M && gofs[2] >= 0;
    const uint32_t loffG = ring_loads ? voff[2] : kOffNone;              // in the lattice or the side planes
    const uint32_t loffS = (ring_loads && shell_w) ? shoff : kOffNone;  // in a saved band boundary
    const uint32_t loffPR = pair_loads ? uint32_t(gofs[0]) * uint32_t(sizeof(R)) : kOffNone;
    const uint32_t loffGR = (rad[2] <= M && gofs[2] >= 0) ? uint32_t(gofs[2]) * uint32_t(sizeof(R)) : kOffNone;

    auto xb = [&](int p) -> uint32_t {
        if (!wallx) return 0u;
        return (p == 0 ? CXP : 0u) | (p == g.nx - 1 ? CXM : 0u);
    };
    auto xm = [&](int p) -> uint32_t {
        if (!wallx) return 0u;
        return ((p == 0 && g.moving_face == 0) ? CXP : 0u) | ((p == g.nx - 1 && g.moving_face == 1) ? CXM : 0u);
    };
    auto present = [&](int p) -> bool { return !wallx || (p >= 0 && p < g.nx); };

    // ---- pipeline registers ----
    using P2 = typename Buf2<T>::P;
    P2 Lp[PF][QL];  // raw pair loads, PF planes in flight
    T Lg[PF][QL];   // raw ring loads
    R Fl1[PF][K][3];
    R acc1[K][QL], nxt1[K][NXP];  // step 1: pair and ring
    R acc2[2][QL], nxt2[2][NXP];  // last step of M = 2: pair only
    R o1[K][3], o2[K][3];
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int q = 0; q < QL; ++q) {
            acc1[k][q] = R(0);
            if (k < 2) acc2[k][q] = R(0);
        }
#pragma unroll
        for (int j = 0; j < NXP; ++j) {
            nxt1[k][j] = R(0);
            if (k < 2) nxt2[k][j] = R(0);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int b = 0; b < PF; ++b) Fl1[b][k][c] = R(0);
            o1[k][c] = o2[k][c] = R(0);
        }
    }

#pragma unroll
    for (int b = 0; b < PF; ++b)
#pragma unroll
        for (int q = 0; q < QL; ++q) {
            Lp[b][q] = Buf2<T>::zero();
            Lg[b][q] = T(0);
        }

    const T* __restrict__ f = static_cast<const T*>(a.f);
    T* __restrict__ fo = static_cast<T*>(a.fo);
    const T* __restrict__ side = static_cast<const T*>(a.side);
    const R* __restrict__ F = static_cast<const R*>(a.force);
    const uint32_t plane_bytes = uint32_t(PL) * uint32_t(sizeof(T));

    // Loads are issued every iteration, unconditionally (empty range when the
    // plane is absent or past the end), so the outstanding-operation counts
    // the compiler tracks stay exact.
    auto plane_base = [&](int xp, long long& qstride) -> const T* {
        if (a.inplace && xp >= e && has_next) {
            qstride = PL;
            return side + ((long long)(nseg_next * M + (xp - e)) * QL) * PL;
        }
        qstride = N;
        return f + (long long)wrapi(xp, g.nx) * PL;
    };
    auto load_force = [&](int xp, bool live, R (&Fb)[3], uint32_t off) {
        if constexpr (FORCE) {
            const uint32_t rangeR = live ? uint32_t(PL) * uint32_t(sizeof(R)) : 0u;
            const R* bc = F + (long long)wrapi(xp, g.nx) * PL;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Fb[c] = Buf<R>::ld(make_rsrc(bc, rangeR), off);
                bc += N;
            }
        }
    };
    auto load_pair = [&](int xp, bool wanted, P2 (&L)[QL], R (&Fb)[K][3]) {
        const bool live = wanted && present(xp);
        long long qs;
        const T* bq = plane_base(xp, qs);
        const uint32_t range = live ? plane_bytes : 0u;
#pragma unroll
        for (int q = 0; q < QL; ++q) {
            L[q] = Buf2<T>::ld(make_rsrc(bq, range), loffP);
            bq += qs;
        }
        if constexpr (FORCE) {
            load_force(xp, live, Fb[0], loffPR);
            const uint32_t off1 = loffPR == kOffNone ? kOffNone : loffPR + uint32_t(sizeof(R));
            load_force(xp, live, Fb[1], off1);
        }
    };
    auto load_ring = [&](int xp, bool wanted, T (&L)[QL], R (&Fb)[K][3]) {
        const bool live = wanted && present(xp);
        long long qs;
        const T* bq = plane_base(xp, qs);
        uint32_t range = live ? plane_bytes : 0u, off = loffG;
        if (shell_w && !(a.inplace && xp >= e && has_next)) {  // (the side planes hold every row at time t)
            qs = (long long)M * g.nz;
            bq = shell_w + (long long)wrapi(xp, g.nx) * QL * qs;
            range = live ? uint32_t(qs) * uint32_t(sizeof(T)) : 0u;
            off = loffS;
        }
#pragma unroll
        for (int q = 0; q < QL; ++q) {
            L[q] = Buf<T>::ld(make_rsrc(bq, range), off);
            bq += qs;
        }
        load_force(xp, live, Fb[2], loffGR);
    };

    // hazard check (see march.hpp): every wave reads the counters of the
    // neighbouring work items at the start of an iteration and checks them
    // before its stores at the end of it
    const int* flp = a.flags;
    int fkind = 0;
    {
        const int nnz = 2 * a.rz + 1, n1 = (2 * a.ry + 1) * nnz;
        int lane = tid & 63, sg = seg;
        fkind = 1;
        if (lane >= n1) {
            lane -= n1;
            sg = nseg_next;
            fkind = has_next ? 2 : 0;
        }
        int yy = ty + lane / nnz - a.ry, zz = tz + lane % nnz - a.rz;
        if (lane >= n1) fkind = 0;
        if (g.wall[1]) {
            if (yy < 0 || yy >= a.nty) fkind = 0;
        } else {
            yy = wrapi(yy, a.nty);
        }
        if (yy < a.band_ty0 || yy >= a.band_ty0 + a.nty_band) fkind = 0;  // a tile row outside the band being marched
        if (g.wall[2]) {
            if (zz < 0 || zz >= a.ntz) fkind = 0;
        } else {
            zz = wrapi(zz, a.ntz);
        }
        if (!a.inplace) fkind = 0;  // out of place: nothing to guard
        if (fkind) flp = a.flags + (1 + ((long long)sg * a.nty + yy) * a.ntz + zz) * a.fstride;
    }
    // plane r is stored in iteration i = r - s + 2M; a work item whose halo
    // covers it loads it in its iteration r - s' + M
    auto poll_need = [&](int i, int r) -> int {
        if (fkind == 1) return i - M + 1;
        if (fkind == 2 && r >= e - M) return r - e + M + 1;
        return -(1 << 30);
    };
    auto poll_finish = [&](int seen, int i, int r) {
        const int need = poll_need(i, r) + a.need_bias;
        if (__all(seen >= need)) return;
        bool ok = seen >= need;
        for (int spin = 0; spin < a.spin_limit && !__all(ok); ++spin) {
            __builtin_amdgcn_s_sleep(2);
            if (!ok) ok = __hip_atomic_load(flp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need;
        }
        if (!__all(ok) && (tid & 63) == 0) __hip_atomic_fetch_or(a.flags, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };

    // Stores marked non-temporal keep the finished planes, which this pass
    // does not read again, from displacing the halo and force lines other
    // tiles are about to read from L2 (the planner's choice, uniform per launch).
    auto store_pair = [&](const R (&v0)[QL], const R (&v1)[QL], int r, bool live) {
        const T* bq = fo + (long long)(live ? r : 0) * PL;
        const uint32_t range = live ? plane_bytes : 0u;
        auto all = [&](auto auxc) {
            constexpr int AUX = decltype(auxc)::value;
#pragma unroll
            for (int q = 0; q < QL; ++q) {
                if constexpr (sizeof(T) == 2)
                    Buf2<T>::template st<AUX>(Cd::enc2(v0[q], v1[q]), make_rsrc(bq, range), soffP);
                else
                    Buf2<T>::template st<AUX>(v0[q], v1[q], make_rsrc(bq, range), soffP);
                bq += N;
            }
        };
        if (a.nt_store)
            all(std::integral_constant<int, 2>{});
        else
            all(std::integral_constant<int, 0>{});
    };

    // step-1 collide of column k from its raw values (decoded here)
    auto collide1 = [&](auto kc, R* X1w, const P2 (&LP)[QL], const T (&LG)[QL], const R (&Fb)[K][3]) {
        constexpr int k = decltype(kc)::value;
        R v[QL];
#pragma unroll
        for (int q = 0; q < QL; ++q) {
            if constexpr (k < 2)
                v[q] = Cd::dec(Buf2<T>::template get<k>(LP[q]));
            else
                v[q] = Cd::dec(LG[q]);
        }
        LT::template collide<R, FORCE>(v, omega, Fb[k][0], Fb[k][1], Fb[k][2]);
        // (with walls or a force, the slot address is rebuilt per plane rather
        // than kept live across the march: those variants are short of
        // registers, and a spilled address reloads behind the plane's loads)
        int sl = ((ci[k] & 1) ? NC / 2 : 0) + (ci[k] >> 1);
        if constexpr (WALLS || FORCE) sl = opaque(sl);
        sfor<0, QL>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            if constexpr (moves_yz_l<LT>(q)) X1w[yz_index_l<LT>(q) * NC + sl] = v[q];
        });
        if constexpr (WALLS) {
            // level-1 receivers: the tile plus M-1 halo cells
            constexpr int PARk = (k == 0) ? (M & 1) : ((k == 1) ? ((M + 1) & 1) : -1);
            if (rad[k] <= M - 1) ghost_out<R, PARk, NC, WZ, LT>(v, nxt1[k], X1w, ci[k], byz[k], mlinks(byz[k]), WT, lane);
        }
        o1[k][0] = v[0];
        o1[k][1] = v[1];
        o1[k][2] = v[XP];
    };

    if constexpr (WALLS) __syncthreads();  // the wall-term table is complete
    const int total = (e - s) + 2 * M;
    // prologue: the first PF planes; iteration i consumes buffer i % PF and
    // refills it with plane xl + PF
#pragma unroll
    for (int b = 0; b < PF; ++b) {
        load_pair(s - M + b, b < total, Lp[b], Fl1[b]);
        load_ring(s - M + b, b < total, Lg[b], Fl1[b]);
    }
    auto iteration = [&](auto pbc, int i) {
        constexpr int pb = decltype(pbc)::value;
        const int xl = s - M + i;
        if constexpr (WALLS) {
            // The wall masks are loop-invariant; left visible, the compiler
            // hoists every per-direction condition and ghost address out of
            // the march and runs out of registers.  Recomputing them per plane
            // costs a few instructions on the few lanes that need them.
#pragma unroll
            for (int k = 0; k < K; ++k) asm volatile("" : "+v"(byz[k]));
        }
        if constexpr (WALLS && FORCE) {
            // With a force as well, the LDS addresses derived from the column
            // indices are hoisted the same way and spill (reloads that queue
            // behind the plane's loads); rebuilding them per plane is cheaper.
            asm volatile("" : "+v"(ci[0]), "+v"(ci[2]), "+v"(ci2[0]), "+v"(ci2[2]));
            ci[1] = ci[0] + 1;
            ci2[1] = ci2[0] + 1;
        }
        R* X1w = X1[(M == 1) ? (i & 1) : 0];
        const int r_out = xl - M;
        const bool storing = r_out >= s && r_out < e;
        const bool next_wanted = i + PF < total;
        const int seen = __hip_atomic_load(flp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

        // The force of plane xl-1, which the second step collides in E, is
        // read again (it was read two planes ago and sits in L2) rather than
        // kept in registers through two iterations.
        R Fr[K][3];
        if constexpr (FORCE && M == 2) {
            const bool live = i >= M && present(xl - 1);
            load_force(xl - 1, live, Fr[0], loffPR);
            load_force(xl - 1, live, Fr[1], loffPR == kOffNone ? kOffNone : loffPR + uint32_t(sizeof(R)));
            load_force(xl - 1, live, Fr[2], loffGR);
        }

        // ---- A: step-1 collide of plane xl; loads of plane xl+1 follow each column ----
        const bool pres = present(xl);
        if (pres && rad[0] <= M)
            collide1(std::integral_constant<int, 0>{}, X1w, Lp[pb], Lg[pb], Fl1[pb]);
        if (pres && rad[1] <= M)
            collide1(std::integral_constant<int, 1>{}, X1w, Lp[pb], Lg[pb], Fl1[pb]);
        load_pair(xl + PF, next_wanted, Lp[pb], Fl1[pb]);
        if (pres && rad[2] <= M)
            collide1(std::integral_constant<int, 2>{}, X1w, Lp[pb], Lg[pb], Fl1[pb]);
        load_ring(xl + PF, next_wanted, Lg[pb], Fl1[pb]);
        __syncthreads();
        if (tid == 0) __hip_atomic_store(a.flags + (1 + gtile) * a.fstride, i + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

        if constexpr (M == 2) {
            // ---- E: step-1 receive (completes plane xl-1), step-2 collide of it ----
            const uint32_t xbd1 = xb(xl - 1), xbn1 = xb(xl), xmn1 = xm(xl);
            const bool coll2 = i >= M && present(xl - 1);
            sfor<0, K>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                constexpr int PAR = (k == 0) ? (M & 1) : ((k == 1) ? ((M + 1) & 1) : -1);  // parity of ci
                constexpr int PAR2 = (k == 0) ? 1 : ((k == 1) ? 0 : -1);                 // parity of ci2
                if (rad[k] <= 1) {
                    complete_s<R, WALLS, PAR, NC, WZ, LT>(acc1[k], X1w, ci[k], o1[k][1], xbd1);
                    if (coll2) {
                        LT::template collide<R, FORCE>(acc1[k], omega, Fr[k][0], Fr[k][1], Fr[k][2]);
                        int sl2 = split_at<PAR2, NC2 / 2>(ci2[k], 0);
                        if constexpr (WALLS || FORCE) sl2 = opaque(sl2);
                        sfor<0, QL>([&](auto qc) {
                            constexpr int q = decltype(qc)::value;
                            if constexpr (moves_yz_l<LT>(q)) X2[yz_index_l<LT>(q) * NC2 + sl2] = acc1[k][q];
                        });
                        if constexpr (WALLS && k < 2) {  // level-2 receivers: the tile
                            if (rad[k] == 0)
                                ghost_out<R, PAR2, NC2, WZ2, LT>(acc1[k], nxt2[k], X2, ci2[k], byz[k], mlinks(byz[k]), WT, lane);
                        }
                        o2[k][0] = acc1[k][0];
                        o2[k][1] = acc1[k][1];
                        o2[k][2] = acc1[k][XP];
                    }
                    deposit_s<R, WALLS, PAR, NC, WZ, LT>(acc1[k], nxt1[k], X1w, ci[k], o1[k][0], o1[k][1], o1[k][2],
                                                     xbn1, byz[k], mlinks(byz[k]) | xmn1, WT, X1w, lane);
                }
            });
            __syncthreads();
        }

        // ---- D: last-step receive of the pair, hazard check, in-place store ----
        {
            const int p = xl - M + 1;  // plane the last step collided
            const uint32_t xbd = xb(p - 1), xbn = xb(p), xmn = xm(p);
            const bool act = rad[0] == 0;
            if constexpr (M == 2) {
                if (act) {
                    complete_s<R, WALLS, 1, NC2, WZ2, LT>(acc2[0], X2, ci2[0], o2[0][1], xbd);
                    complete_s<R, WALLS, 0, NC2, WZ2, LT>(acc2[1], X2, ci2[1], o2[1][1], xbd);
                }
                if (storing) poll_finish(seen, i, r_out);
                store_pair(acc2[0], acc2[1], r_out, storing);
                if (act) {
                    deposit_s<R, WALLS, 1, NC2, WZ2, LT>(acc2[0], nxt2[0], X2, ci2[0], o2[0][0], o2[0][1], o2[0][2],
                                                     xbn, byz[0], mlinks(byz[0]) | xmn, WT, X2, lane);
                    deposit_s<R, WALLS, 0, NC2, WZ2, LT>(acc2[1], nxt2[1], X2, ci2[1], o2[1][0], o2[1][1], o2[1][2],
                                                     xbn, byz[1], mlinks(byz[1]) | xmn, WT, X2, lane);
                }
            } else {
                if (act) {
                    complete_s<R, WALLS, 1, NC, WZ, LT>(acc1[0], X1w, ci[0], o1[0][1], xbd);
                    complete_s<R, WALLS, 0, NC, WZ, LT>(acc1[1], X1w, ci[1], o1[1][1], xbd);
                }
                if (storing) poll_finish(seen, i, r_out);
                store_pair(acc1[0], acc1[1], r_out, storing);
                if (act) {
                    R* X1n = X1[(M == 1) ? ((i + 1) & 1) : 0];  // the buffer the next plane uses
                    deposit_s<R, WALLS, 1, NC, WZ, LT>(acc1[0], nxt1[0], X1w, ci[0], o1[0][0], o1[0][1], o1[0][2],
                                                   xbn, byz[0], mlinks(byz[0]) | xmn, WT, X1n, lane);
                    deposit_s<R, WALLS, 0, NC, WZ, LT>(acc1[1], nxt1[1], X1w, ci[1], o1[1][0], o1[1][1], o1[1][2],
                                                   xbn, byz[1], mlinks(byz[1]) | xmn, WT, X1n, lane);
                }
            }
        }
    };
    for (int i = 0; i < total; i += PF) {
        iteration(std::integral_constant<int, 0>{}, i);
        if constexpr (PF == 2) {
            if (i + 1 < total) iteration(std::integral_constant<int, 1>{}, i + 1);
        }
    }
}

template <int S, int M, int TY, int TZ, bool WALLS, bool FORCE, int PF, class LT = D3Q19>
hipError_t launch_march_pr_shape(const MarchPlan& p, const MarchArgs& a, hipStream_t st)
{
    auto kern = k_march_pr<S, M, TY, TZ, WALLS, FORCE, PF, LT>;
    MarchArgs arg = a;
    void* params[] = {&arg};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(p.blocks),
                                      dim3(PairRingShape<M, TY, TZ>::NT), params, 0, st);
}

template <int S, int M, int TY, int TZ, bool WALLS, bool FORCE, int PF, class LT = D3Q19>
int max_blocks_pr_shape()
{
    int dev = 0, per_cu = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_march_pr<S, M, TY, TZ, WALLS, FORCE, PF, LT>,
                                                     PairRingShape<M, TY, TZ>::NT, 0) != hipSuccess)
        return 0;
    return per_cu * cus;
}

}  // namespace lbm
