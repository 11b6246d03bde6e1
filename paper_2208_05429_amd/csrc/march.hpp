// march.hpp -- the in-place, single-copy D3Q19 update with M in {1, 2, 3} time
// steps merged per pass over HBM (the paper's Fuse Swap LBM of Sec. 3 /
// Alg. 1 for M = 1, its two-step merging of Sec. 4.1 / Alg. 2 for M = 2, and
// the deeper merging its conclusion (Sec. 6) names as the next step for M = 3),
// designed for CDNA4 rather than transcribed from the CPU algorithms.
//
// Decomposition.  The y-z plane is cut into TY x TZ tiles and the x axis into
// segments; one workgroup owns a (tile, segment) work item and marches along
// x, one plane per iteration.  It loads the time-t plane of its tile plus a
// halo of M cells (all 19 populations, straight from the single copy),
// collides it, and exchanges the populations that move in y or z through LDS;
// populations that move only in x stay in the thread's registers and reach
// their plane one iteration later or earlier.  For M = 2 the second step runs
// one plane behind the first on the tile plus a halo of one cell, so the t+1
// state never leaves the chip (the dependency cone of Sec. 4.1: the second
// computation of a cell follows the first of its later neighbours).  The
// finished t+M plane, M planes behind the load front, is written back in
// place over the time-t plane it replaces: there is no second lattice.
//
// In-place hazards across workgroups (the GPU form of the thread-safety
// argument of Sec. 4.2).  A workgroup may overwrite plane r only after every
// workgroup whose halo covers its tile has loaded plane r.  Each work item
// publishes its load front in a progress counter (agent-scope atomic); before
// a store, one wave polls the counters of the neighbouring tiles (and, for the
// last M planes of a segment, of the next segment, whose first loads reach
// back M planes).  All work items are co-resident (cooperative launch), and
// the one with the smallest load front never waits, so the march cannot
// deadlock; every wait is additionally bounded and reports a timeout.
// The first M planes of every segment are read by the previous segment at
// its end, after they were overwritten; a prepass saves their time-t copies
// (the analogue of the bounding-box pre-processing of Alg. 1's Stage I).
//
// Boundaries.  Periodic axes wrap indices.  A population whose source lies
// beyond a wall is the cell's own reversed post-collision value (halfway
// bounce-back, what the swap algorithm leaves in slots without a partner),
// plus 6 w_q (c_q . u_w) if the moving face is among the faces crossed.
#pragma once

#include "d3q19.hpp"
#include "lattices.hpp"
#include "lbm_internal.hpp"

namespace lbm {

// direction masks: bit q set for every q with c_x = +1 / -1
template <class LT = D3Q19>
__host__ __device__ constexpr uint32_t mask_cx(int sgn)
{
    uint32_t m = 0;
    for (int q = 0; q < LT::Q; ++q)
        if (LT::cx(q) == sgn) m |= 1u << q;
    return m;
}

__device__ __forceinline__ int wrapi(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// Work item -> (tile z, tile row within the band, x segment).  Items of a
// segment go stripe by stripe, each stripe about 512 cells wide in z and
// row-major inside, so that the 32 consecutive items one XCD runs (after the
// XCD remap) form a compact block of tiles whose halos its L2 shares: four
// tile rows of eight 64-wide tiles rather than two rows of a 1024-wide plane.
template <int TZ>
__device__ __forceinline__ void tile_of_item(int item, int nty, int ntz, int& tz, int& ty, int& seg)
{
    constexpr int WANT = (512 / TZ) > 0 ? 512 / TZ : 1;
    const int bz = ntz < WANT ? ntz : WANT;
    const int run = nty * ntz;
    seg = item / run;
    const int r = item - seg * run;
    const int full = ntz / bz, per_stripe = nty * bz;
    const int s = r / per_stripe;
    if (s < full) {
        const int l = r - s * per_stripe;
        ty = l / bz;
        tz = s * bz + (l - (l / bz) * bz);
    } else {  // the narrower last stripe
        const int w = ntz - full * bz, l = r - full * per_stripe;
        ty = l / w;
        tz = full * bz + (l - (l / w) * w);
    }
}

// The two halves of one level's exchange for one column.  The level has just
// collided plane p: the post-collision values of the column-moving
// directions are in X (16 rows of `stride` columns; this column at index ci,
// row pitch wz), the three x-only directions (q = 0, 1, 10) in o0, o1, o10.
//
// complete(): acc[] holds plane p-1 except its c_x = -1 populations, which
// come from plane p; afterwards acc[] is the whole plane p-1 (at the level's
// output time).  bdone: directions of plane p-1 whose source is beyond a wall
// (their value was deposited earlier).
template <class R, bool WALLS, class LT = D3Q19>
__device__ __forceinline__ void complete(R (&acc)[LT::Q], const R* __restrict__ X, int stride, int ci, int wz, R o1,
                                         uint32_t bdone)
{
    sfor<0, LT::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        if constexpr (LT::cx(q) == -1) {
            R rv;
            if constexpr (moves_yz_l<LT>(q))
                rv = X[yz_index_l<LT>(q) * stride + ci - LT::cy(q) * wz - LT::cz(q)];
            else
                rv = o1;
            if constexpr (WALLS)
                acc[q] = ((bdone >> q) & 1u) ? acc[q] : rv;
            else
                acc[q] = rv;
        }
    });
}

// deposit(): after acc[] was consumed, refill it with what is known of plane
// p (c_x = 0 populations, bounce-backs, and the c_x = +1 populations received
// one iteration earlier in nxt[]) and put plane p+1's c_x = +1 populations in
// nxt[].  bnext: directions of plane p whose source is beyond a wall (a
// moving wall's term was already added at the source, see moving_wall_out).
template <class R, bool WALLS, class LT = D3Q19>
__device__ __forceinline__ void deposit(R (&acc)[LT::Q], R (&nxt)[nxp<LT>()], const R* __restrict__ X, int stride, int ci,
                                        int wz, R o0, R o1, R o10, uint32_t bnext)
{
    sfor<0, LT::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int qo = LT::opp(q);
        R bval = R(0);
        if constexpr (WALLS && q != 0) {
            if constexpr (moves_yz_l<LT>(qo))
                bval = X[yz_index_l<LT>(qo) * stride + ci];
            else
                bval = (qo == 1) ? o1 : o10;
        }
        if constexpr (LT::cx(q) == 0) {
            R rv;
            if constexpr (q == 0)
                rv = o0;
            else
                rv = X[yz_index_l<LT>(q) * stride + ci - LT::cy(q) * wz - LT::cz(q)];
            if constexpr (WALLS && q != 0)
                acc[q] = ((bnext >> q) & 1u) ? bval : rv;
            else
                acc[q] = rv;
        } else if constexpr (LT::cx(q) == 1) {
            constexpr int j = xp_index_l<LT>(q);
            if constexpr (WALLS)
                acc[q] = ((bnext >> q) & 1u) ? bval : nxt[j];
            else
                acc[q] = nxt[j];
            if constexpr (moves_yz_l<LT>(q))
                nxt[j] = X[yz_index_l<LT>(q) * stride + ci - LT::cy(q) * wz - LT::cz(q)];
            else
                nxt[j] = o10;
        } else {
            if constexpr (WALLS) acc[q] = bval;
        }
    });
}

template <class LT, int S, int M, int TY, int TZ, int NT, bool WALLS, bool FORCE, bool ROUNDS, int PF = 1>
__global__ __launch_bounds__(NT) void k_march(MarchArgs a)
{
    constexpr int QL = LT::Q;                 // velocities
    constexpr int NYZ = nyz<LT>();            // those that move between columns, exchanged through LDS
    constexpr int NXP = nxp<LT>();            // those with c_x = +1, carried to the next plane
    constexpr int XP = LT::H + 1;             // the x-only direction (+1, 0, 0); (-1, 0, 0) is 1
    using Cd = Codec<S>;
    using T = typename Cd::T;
    using R = typename Cd::R;
    constexpr int WY = TY + 2 * M, WZ = TZ + 2 * M, NC = WY * WZ;
    constexpr int K = (NC + NT - 1) / NT;
    // step 2 runs on the tile plus M-1 halo cells, step 3 (M = 3) on the tile plus one
    constexpr int WZ2 = TZ + 2 * (M - 1), NC2 = (TY + 2 * (M - 1)) * WZ2;
    constexpr int WZ3 = TZ + 2, NC3 = (TY + 2) * WZ3;
    constexpr int K3 = (M == 3) ? K : 1;  // step-3 registers exist for M = 3 only
    constexpr int NB1 = (M == 1) ? 2 : 1;  // a single exchange level is double-buffered
    constexpr uint32_t CXP = mask_cx<LT>(1), CXM = mask_cx<LT>(-1);
    static_assert(M >= 1 && M <= 3, "one to three merged steps");
    static_assert(PF == 1 || PF == 2, "loads run one or two planes ahead");

    __shared__ R X1[NB1][NYZ * NC];
    __shared__ R X2[(M >= 2) ? NYZ * NC2 : 1];
    __shared__ R X3[(M == 3) ? NYZ * NC3 : 1];
    __shared__ R WT[WALLS ? QL : 1];  // moving-wall terms (entry q: received along c_q)

    const Geom& g = a.g;
    const int tid = threadIdx.x;
    int wid = blockIdx.x;
    if (a.xcd_remap) {
        const int per = gridDim.x >> 3;
        wid = (wid & 7) * per + (wid >> 3);
    }
    if (wid >= a.items) return;  // padding of the grid (uniform per workgroup, before any barrier)
    // A round covers the band of tile rows [band_ty0, band_ty0 + nty_band).
    // ROUNDS compiles the band edge code in; the 32- and 16-bit storages
    // launch that build only for planes that run in rounds, since it costs
    // their variants registers.
    const bool banded = a.nty_band < a.nty;
    int tz, ty, seg;
    tile_of_item<TZ>(wid, a.nty_band, a.ntz, tz, ty, seg);
    ty += a.band_ty0;
    const long long gtile = ((long long)seg * a.nty + ty) * a.ntz + tz;  // progress counter index
    const int s = seg * a.seg_len, e = min(s + a.seg_len, g.nx);
    const int TYe = min(TY, g.ny - ty * TY), TZe = min(TZ, g.nz - tz * TZ);
    // Rounds: the band's first (last) row of tiles reads the halo rows below
    // (above) the band from the saved band boundary rows, when the band there
    // was already updated this pass (the host passes those copies only then).
    const T* shell_lo = (banded && ty == a.band_ty0) ? static_cast<const T*>(a.shell_lo) : nullptr;
    const T* shell_hi = (banded && ty == a.band_ty0 + a.nty_band - 1) ? static_cast<const T*>(a.shell_hi) : nullptr;
    const bool wallx = g.wall[0] != 0;
    const bool has_next = !wallx || seg + 1 < a.nseg;
    const int nseg_next = (seg + 1 == a.nseg) ? 0 : seg + 1;
    const R omega = R(g.omega);
    if constexpr (WALLS) wall_terms_to_l<LT>(WT, tid, R(g.uw[0]), R(g.uw[1]), R(g.uw[2]));
    const long long N = g.N, PL = g.PL;

    // ---- columns owned by this thread ----
    int gofs[K], rad[K], ci2[K], ci3[K3];
    uint32_t voff[K];   // byte offset of the column within one direction's plane
    uint32_t loff[K];   // voff for columns that load (tile plus M halo cells), else out of range
    uint32_t loffR[K];  // the same in units of the arithmetic type (force field)
    uint32_t soff[K];   // voff for interior columns (stored), else out of range
    uint32_t byz[K], myz[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        gofs[k] = -1;
        voff[k] = kOffNone;
        rad[k] = M + 1;
        ci2[k] = 0;
        if constexpr (M == 3) ci3[k] = 0;
        byz[k] = 0;
        myz[k] = 0;
        const int c = tid + k * NT;
        if (c < NC) {
            const int ly = c / WZ, lz = c - (c / WZ) * WZ;
            if (ly < TYe + 2 * M && lz < TZe + 2 * M) {
                const int dy = ly < M ? M - ly : (ly >= M + TYe ? ly - (M + TYe) + 1 : 0);
                const int dz = lz < M ? M - lz : (lz >= M + TZe ? lz - (M + TZe) + 1 : 0);
                int y = ty * TY - M + ly, z = tz * TZ - M + lz;
                bool inside = true;
                if (g.wall[1]) inside = inside && y >= 0 && y < g.ny;
                else y = wrapi(y, g.ny);
                if (g.wall[2]) inside = inside && z >= 0 && z < g.nz;
                else z = wrapi(z, g.nz);
                if (inside) {
                    gofs[k] = y * g.nz + z;
                    voff[k] = uint32_t(gofs[k]) * uint32_t(sizeof(T));
                    rad[k] = dy > dz ? dy : dz;
                    ci2[k] = (ly - 1) * WZ2 + (lz - 1);
                    if constexpr (M == 3) ci3[k] = (ly - 2) * WZ3 + (lz - 2);
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
                        byz[k] = b;
                        myz[k] = mv;
                    }
                }
            }
        }
    }

#pragma unroll
    for (int k = 0; k < K; ++k) {
        const bool loads = rad[k] <= M && gofs[k] >= 0;
        loff[k] = loads ? voff[k] : kOffNone;
        loffR[k] = loads ? uint32_t(gofs[k]) * uint32_t(sizeof(R)) : kOffNone;
        soff[k] = (rad[k] == 0 && gofs[k] >= 0) ? voff[k] : kOffNone;
    }

    // x-wall bounce-back and moving-face masks of a plane
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
    T Lr[PF][K][QL];  // raw loads, PF planes in flight
    R Fl1[PF][K][3], Fl2[K][3], Fl3[K3][3];
    R acc1[K][QL], nxt1[K][NXP], acc2[K][QL], nxt2[K][NXP], acc3[K3][QL], nxt3[K3][NXP];
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int q = 0; q < QL; ++q) {
            for (int b = 0; b < PF; ++b) Lr[b][k][q] = T(0);
            acc1[k][q] = R(0);
            acc2[k][q] = R(0);
            if constexpr (M == 3) acc3[k][q] = R(0);
        }
#pragma unroll
        for (int j = 0; j < NXP; ++j) {
            nxt1[k][j] = R(0);
            nxt2[k][j] = R(0);
            if constexpr (M == 3) nxt3[k][j] = R(0);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            for (int b = 0; b < PF; ++b) Fl1[b][k][c] = R(0);
            Fl2[k][c] = R(0);
            if constexpr (M == 3) Fl3[k][c] = R(0);
        }
    }

    const T* __restrict__ f = static_cast<const T*>(a.f);
    T* __restrict__ fo = static_cast<T*>(a.fo);
    const T* __restrict__ side = static_cast<const T*>(a.side);
    const R* __restrict__ F = static_cast<const R*>(a.force);

    // Loads and stores address one direction of one plane through a buffer
    // descriptor built on the scalar unit plus a 32-bit per-lane byte offset;
    // unused slots carry an out-of-range offset and touch no memory.
    const uint32_t plane_bytes = uint32_t(PL) * uint32_t(sizeof(T));
    // Every iteration issues the same loads, unconditionally: a plane that is
    // absent (beyond a wall) or past the end of the march gets an empty buffer
    // range, so the hardware returns zeros without touching memory.  Uniform
    // issue keeps the compiler's count of outstanding memory operations exact.
    auto issue_load_slot = [&](int xp, bool wanted, int k, T (&L)[QL], R (&Fb)[3]) {
        const bool live = wanted && present(xp);
        const bool from_side = a.inplace && xp >= e && has_next;
        const int px = wrapi(xp, g.nx);
        const T* base;
        long long qstride;
        if (from_side) {
            base = side + ((long long)(nseg_next * M + (xp - e)) * QL) * PL;
            qstride = PL;
        } else {
            base = f + (long long)px * PL;
            qstride = N;
        }
        const uint32_t range = live ? plane_bytes : 0u;
        const T* bq = base;  // running pointer: nothing per direction stays live across iterations
        if (!ROUNDS || !(shell_lo || shell_hi) || from_side) {  // (the side planes hold every row at time t)
#pragma unroll
            for (int q = 0; q < QL; ++q) {
                L[q] = Buf<T>::ld(make_rsrc(bq, range), loff[k]);
                bq += qstride;
            }
        } else {
            // A band edge tile: lanes of the rows beyond the band read the
            // saved copy ([x][q][row][z], M rows), the others the lattice.
            // Told apart by the lane's plane offset (row * nz + z) * size: the
            // M rows below the band sit right under its first row; across the
            // periodic seam the rows above are rows 0 .. M-1, whose offsets
            // are those of the copy itself.
            const long long ss = (long long)M * g.nz;
            const uint32_t rowb = uint32_t(g.nz) * uint32_t(sizeof(T));
            const uint32_t lo_first = shell_lo ? uint32_t(a.band_ty0 * TY - M) * rowb : 0u;
            const uint32_t lo_end = shell_lo ? uint32_t(a.band_ty0 * TY) * rowb : 0u;
            const uint32_t hi_end = shell_hi ? uint32_t(M) * rowb : 0u;
            const uint32_t lf = loff[k];
            const bool in_lo = lf != kOffNone && lf >= lo_first && lf < lo_end;
            const bool in_hi = lf != kOffNone && lf < hi_end;
            const uint32_t lofs = (in_lo || in_hi) ? kOffNone : lf;
            const uint32_t olo = in_lo ? lf - lo_first : kOffNone, ohi = in_hi ? lf : kOffNone;
            const uint32_t srange = live ? uint32_t(ss) * uint32_t(sizeof(T)) : 0u;
            const T* blo = shell_lo ? shell_lo + (long long)px * QL * ss : nullptr;
            const T* bhi = shell_hi ? shell_hi + (long long)px * QL * ss : nullptr;
            // Every path issues exactly one load per direction and nothing
            // that reads the loaded values, so the loads stay in flight across
            // the iteration and the compiler's count of outstanding loads is
            // the same on every path (a path that issued more, or picked a
            // value per lane after loading, made the whole march wait for the
            // next plane's loads: rounds 3x slower).  A wave whose lanes all
            // read one source loads through that source's buffer descriptor.
            const bool lat = lf != kOffNone && !in_lo && !in_hi;
            const bool any_lat = __any(lat), any_lo = __any(in_lo), any_hi = __any(in_hi);
            if (!any_lo && !any_hi) {
#pragma unroll
                for (int q = 0; q < QL; ++q) {
                    L[q] = Buf<T>::ld(make_rsrc(bq, range), lf);
                    bq += qstride;
                }
            } else if (!any_lat && !any_hi) {
#pragma unroll
                for (int q = 0; q < QL; ++q) {
                    L[q] = Buf<T>::ld(make_rsrc(blo, srange), olo);
                    blo += ss;
                }
            } else if (!any_lat && !any_lo) {
#pragma unroll
                for (int q = 0; q < QL; ++q) {
                    L[q] = Buf<T>::ld(make_rsrc(bhi, srange), ohi);
                    bhi += ss;
                }
            } else {
                // A wave that mixes sources: one global load per lane and
                // direction from the address of its own source, so the wave
                // issues the same loads as on the other paths.  A lane with
                // nothing to load reads its plane's first value, which it
                // never uses.
                using GT = const T __attribute__((address_space(1)));
                const uintptr_t ulo = reinterpret_cast<uintptr_t>(blo), uhi = reinterpret_cast<uintptr_t>(bhi);
                const uintptr_t ula = reinterpret_cast<uintptr_t>(bq);
                const uintptr_t dlo = uintptr_t(ss) * sizeof(T), dla = uintptr_t(qstride) * sizeof(T);
                const uintptr_t own = in_lo ? ulo + olo : (in_hi ? uhi + ohi : ula + (lf == kOffNone ? 0u : lf));
                const uintptr_t step = (in_lo || in_hi) ? dlo : dla;
#pragma unroll
                for (int q = 0; q < QL; ++q) L[q] = *reinterpret_cast<GT*>(own + uintptr_t(q) * step);
            }
        }
        if constexpr (FORCE) {
            const uint32_t rangeR = live ? uint32_t(PL) * uint32_t(sizeof(R)) : 0u;
            const R* bc = F + (long long)px * PL;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Fb[c] = Buf<R>::ld(make_rsrc(bc, rangeR), loffR[k]);
                bc += N;
            }
        }
    };
    auto issue_load = [&](int xp, bool wanted, T (&L)[K][QL], R (&Fb)[K][3]) {
#pragma unroll
        for (int k = 0; k < K; ++k) issue_load_slot(xp, wanted, k, L[k], Fb[k]);
    };

    // Hazard check.  Every wave watches the progress counters itself, one per
    // lane: lanes [0, n1) the tiles around this one in the same segment, lanes
    // [n1, 2 n1) the same tiles in the next segment, whose first M loads reach
    // back into this one.  The counters are read at the end of an iteration
    // and checked by each wave before its stores in the next one, so no
    // barrier ever waits on memory and only a lagging neighbour costs a spin.
    const int* flp = a.flags;  // lanes without a neighbour read the timeout word
    int fkind = 0;             // 0: none, 1: same segment, 2: next segment
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
    // plane r is stored in iteration i = r - s + 2M + 1; every work item whose
    // halo covers it loads it in its iteration r - s' + M, i.e. has published
    // a load front >= r - s' + M + 1 (with loads two planes ahead, one
    // iteration earlier still: the same bound holds)
    auto poll_need = [&](int i, int r) -> int {
        if (fkind == 1) return i - M;
        if (fkind == 2 && r >= e - M) return r - e + M + 1;
        return -(1 << 30);
    };
    auto poll_issue = [&]() -> int { return __hip_atomic_load(flp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); };
    auto poll_finish = [&](int seen, int i, int r) {
        const int need = poll_need(i, r) + a.need_bias;
        if (__all(seen >= need)) return;
        // bounded wait: a timeout is recorded in flags[0] and the march goes on
        bool ok = seen >= need;
        for (int spin = 0; spin < a.spin_limit && !__all(ok); ++spin) {
            __builtin_amdgcn_s_sleep(2);
            if (!ok) ok = __hip_atomic_load(flp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need;
        }
        if (!__all(ok) && (tid & 63) == 0) __hip_atomic_fetch_or(a.flags, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };

    // Stores, like loads, are issued every iteration by every slot; lanes that
    // do not own a finished interior column carry an out-of-range offset and a
    // plane that is not stored this iteration gets an empty range.  The slots
    // share each direction's buffer descriptor.
    auto store_all = [&](const R (&out)[K][QL], int r, bool live) {
        const T* bq = fo + (long long)(live ? r : 0) * PL;
        const uint32_t range = live ? plane_bytes : 0u;
#pragma unroll
        for (int q = 0; q < QL; ++q) {
            const auto rs = make_rsrc(bq, range);
#pragma unroll
            for (int k = 0; k < K; ++k) Buf<T>::st(Cd::enc(out[k][q]), rs, soff[k]);
            bq += N;
        }
    };

    // Pipeline of one iteration (load front at plane xl):
    //   A  step-1 collide of plane xl on the tile plus M halo cells, then at
    //      once the loads of plane xl+PF for the same column (PF = 2: two
    //      register buffers of loads, used in turn);
    //   D  receive of the last step from the exchange filled one iteration
    //      earlier: completes plane xl-M-1 (time t+M), stored in place after
    //      the hazard check;
    //   |  barrier, publish the load front;
    //   E  (M >= 2) receive of step 1 (completes plane xl-1 at t+1) and step-2
    //      collide of that plane on the tile plus M-1 halo cells;
    //   |  (M >= 2) barrier;
    //   E3 (M = 3) receive of step 2 (completes plane xl-2 at t+2) and step-3
    //      collide of that plane on the tile plus one halo cell;
    //   |  (M = 3) barrier.
    // Each level's exchange is read in the phase after the one that filled it,
    // so every level keeps its own LDS buffer.  Stores leave early and the
    // loads of the next plane have the whole of E (and E3) to arrive: the
    // first wait of the next iteration finds them done.
    R o1[K][3], o1p[K][3], o2[K][3], o3[K3][3];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            o1[k][c] = o1p[k][c] = o2[k][c] = R(0);
            if constexpr (M == 3) o3[k][c] = R(0);
        }
    if constexpr (WALLS) __syncthreads();  // the wall-term table is complete
    const int total = (e - s) + 2 * M + 1;
    // prologue: the first PF planes; iteration i consumes buffer i % PF and
    // refills it with plane xl + PF (planes up to e - 1 + M are wanted)
#pragma unroll
    for (int b = 0; b < PF; ++b) issue_load(s - M + b, s - M + b <= e - 1 + M, Lr[b], Fl1[b]);
    int seen = poll_issue();
    auto iteration = [&](auto pbc, int i) {
        constexpr int pb = decltype(pbc)::value;
        const int xl = s - M + i;
        R* X1w = X1[(M == 1) ? (i & 1) : 0];        // filled by this iteration's step-1 collide
        R* X1r = X1[(M == 1) ? ((i + 1) & 1) : 0];  // (M = 1) filled one iteration earlier
        const int r_out = xl - M - 1;
        const bool storing = r_out >= s && r_out < e;
        const bool next_wanted = xl + PF <= e - 1 + M;

        // ---- A: step-1 collide of plane xl, then the loads of plane xl+PF ----
        R Fs[K][3];
        const bool pres = present(xl);
        const uint32_t xmc = xm(xl);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if constexpr (FORCE) {
#pragma unroll
                for (int c = 0; c < 3; ++c) Fs[k][c] = Fl1[pb][k][c];
            }
            if (pres && rad[k] <= M && gofs[k] >= 0) {
                R v[QL];
#pragma unroll
                for (int q = 0; q < QL; ++q) v[q] = Cd::dec(Lr[pb][k][q]);
                LT::template collide<R, FORCE>(v, omega, Fl1[pb][k][0], Fl1[pb][k][1], Fl1[pb][k][2]);
                const int c = tid + k * NT;
                sfor<0, QL>([&](auto qc) {
                    constexpr int q = decltype(qc)::value;
                    if constexpr (moves_yz_l<LT>(q)) X1w[yz_index_l<LT>(q) * NC + c] = v[q];
                });
                if constexpr (WALLS) moving_wall_out_l<LT>(v[1], v[XP], X1w, NC, c, myz[k] | xmc, WT);
                o1[k][0] = v[0];
                o1[k][1] = v[1];
                o1[k][2] = v[XP];
            }
            issue_load_slot(xl + PF, next_wanted, k, Lr[pb][k], Fl1[pb][k]);
        }

        // ---- D: last-step receive, hazard check, in-place stores ----
        // (complete and deposit only read the exchange, so every slot
        // completes, then all store together, then all deposit)
        if (storing) poll_finish(seen, i, r_out);
        {
            const int p = xl - M;  // plane collided by the last step one iteration ago
            const uint32_t xbd = xb(p - 1), xbn = xb(p);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (rad[k] == 0 && gofs[k] >= 0) {
                    if constexpr (M == 3) {
                        complete<R, WALLS, LT>(acc3[k], X3, NC3, ci3[k], WZ3, o3[k][1], byz[k] | xbd);
                    } else if constexpr (M == 2) {
                        complete<R, WALLS, LT>(acc2[k], X2, NC2, ci2[k], WZ2, o2[k][1], byz[k] | xbd);
                    } else {
                        complete<R, WALLS, LT>(acc1[k], X1r, NC, tid + k * NT, WZ, o1p[k][1], byz[k] | xbd);
                    }
                }
            }
            if constexpr (M == 3)
                store_all(acc3, r_out, storing);
            else if constexpr (M == 2)
                store_all(acc2, r_out, storing);
            else
                store_all(acc1, r_out, storing);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (rad[k] == 0 && gofs[k] >= 0) {
                    if constexpr (M == 3) {
                        deposit<R, WALLS, LT>(acc3[k], nxt3[k], X3, NC3, ci3[k], WZ3, o3[k][0], o3[k][1], o3[k][2],
                                              byz[k] | xbn);
                    } else if constexpr (M == 2) {
                        deposit<R, WALLS, LT>(acc2[k], nxt2[k], X2, NC2, ci2[k], WZ2, o2[k][0], o2[k][1], o2[k][2],
                                              byz[k] | xbn);
                    } else {
                        const int c = tid + k * NT;
                        deposit<R, WALLS, LT>(acc1[k], nxt1[k], X1r, NC, c, WZ, o1p[k][0], o1p[k][1], o1p[k][2],
                                              byz[k] | xbn);
                    }
                }
            }
        }
        if constexpr (M == 1) {
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) o1p[k][c] = o1[k][c];
            seen = poll_issue();
        }
        __syncthreads();
        if (tid == 0) __hip_atomic_store(a.flags + (1 + gtile) * a.fstride, i + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

        if constexpr (M >= 2) {
            // ---- E: step-1 receive (completes plane xl-1), step-2 collide of it ----
            // (step 2 collides planes s-M+1 .. e+M-2: from iteration 2 on)
            const uint32_t xbd1 = xb(xl - 1), xbn1 = xb(xl), xmc2 = xm(xl - 1);
            const bool coll2 = i >= 2 && present(xl - 1);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (rad[k] <= M - 1 && gofs[k] >= 0) {
                    const int c = tid + k * NT;
                    complete<R, WALLS, LT>(acc1[k], X1w, NC, c, WZ, o1[k][1], byz[k] | xbd1);
                    if (coll2) {
                        LT::template collide<R, FORCE>(acc1[k], omega, Fl2[k][0], Fl2[k][1], Fl2[k][2]);
                        sfor<0, QL>([&](auto qc) {
                            constexpr int q = decltype(qc)::value;
                            if constexpr (moves_yz_l<LT>(q)) X2[yz_index_l<LT>(q) * NC2 + ci2[k]] = acc1[k][q];
                        });
                        if constexpr (WALLS)
                            moving_wall_out_l<LT>(acc1[k][1], acc1[k][XP], X2, NC2, ci2[k], myz[k] | xmc2, WT);
                        o2[k][0] = acc1[k][0];
                        o2[k][1] = acc1[k][1];
                        o2[k][2] = acc1[k][XP];
                    }
                    deposit<R, WALLS, LT>(acc1[k], nxt1[k], X1w, NC, c, WZ, o1[k][0], o1[k][1], o1[k][2],
                                      byz[k] | xbn1);
                }
                if constexpr (FORCE && M == 2) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) Fl2[k][c] = Fs[k][c];
                }
            }
            if constexpr (M == 2) seen = poll_issue();
            __syncthreads();
        }
        if constexpr (M == 3) {
            // ---- E3: step-2 receive (completes plane xl-2 at t+2), step-3 collide of it ----
            // (step 3 collides planes s-1 .. e: from iteration 4 on)
            const uint32_t xbd2 = xb(xl - 2), xbn2 = xb(xl - 1), xmc3 = xm(xl - 2);
            const bool coll3 = i >= 4 && present(xl - 2);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (rad[k] <= M - 2 && gofs[k] >= 0) {
                    complete<R, WALLS, LT>(acc2[k], X2, NC2, ci2[k], WZ2, o2[k][1], byz[k] | xbd2);
                    if (coll3) {
                        LT::template collide<R, FORCE>(acc2[k], omega, Fl3[k][0], Fl3[k][1], Fl3[k][2]);
                        sfor<0, QL>([&](auto qc) {
                            constexpr int q = decltype(qc)::value;
                            if constexpr (moves_yz_l<LT>(q)) X3[yz_index_l<LT>(q) * NC3 + ci3[k]] = acc2[k][q];
                        });
                        if constexpr (WALLS)
                            moving_wall_out_l<LT>(acc2[k][1], acc2[k][XP], X3, NC3, ci3[k], myz[k] | xmc3, WT);
                        o3[k][0] = acc2[k][0];
                        o3[k][1] = acc2[k][1];
                        o3[k][2] = acc2[k][XP];
                    }
                    deposit<R, WALLS, LT>(acc2[k], nxt2[k], X2, NC2, ci2[k], WZ2, o2[k][0], o2[k][1], o2[k][2],
                                      byz[k] | xbn2);
                }
                if constexpr (FORCE) {
                    // forces of planes xl-1 and xl move one level down
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        Fl3[k][c] = Fl2[k][c];
                        Fl2[k][c] = Fs[k][c];
                    }
                }
            }
            seen = poll_issue();
            __syncthreads();
        }
    };
    for (int i = 0; i < total; i += PF) {
        iteration(std::integral_constant<int, 0>{}, i);
        if constexpr (PF == 2) {
            if (i + 1 < total) iteration(std::integral_constant<int, 1>{}, i + 1);
        }
    }
}

// Launch of one compiled shape.  Cooperative launch guarantees co-residency
// of all work items (required by the progress-counter protocol).
template <int S, int M, int TY, int TZ, int NT, bool WALLS, bool FORCE, bool ROUNDS, class LT = D3Q19, int PF = 1>
hipError_t launch_march_shape(const MarchPlan& p, const MarchArgs& a, hipStream_t st)
{
    auto kern = k_march<LT, S, M, TY, TZ, NT, WALLS, FORCE, ROUNDS, PF>;
    MarchArgs arg = a;
    void* params[] = {&arg};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(p.blocks), dim3(NT), params, 0, st);
}

template <int S, int M, int TY, int TZ, int NT, bool WALLS, bool FORCE, bool ROUNDS, class LT = D3Q19, int PF = 1>
int max_blocks_shape()
{
    int dev = 0, per_cu = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_march<LT, S, M, TY, TZ, NT, WALLS, FORCE, ROUNDS, PF>, NT,
                                                     0) != hipSuccess)
        return 0;
    return per_cu * cus;
}

}  // namespace lbm
