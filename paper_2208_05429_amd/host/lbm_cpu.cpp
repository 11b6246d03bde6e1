// lbm_cpu.cpp -- the paper's sequential CPU algorithms for the single-copy
// D3Q19 update (include/lbm_cpu.h): the Fuse Swap LBM of Sec. 3 / Alg. 1 and
// the two-step memory-aware LBM of Sec. 4.1 / Alg. 2 with its prism
// traversal.  Host context for the GPU library, one thread, FP64.
//
// The swap algorithm (Sec. 3).  A cell collides, then `reverts' (slot q takes
// the post-collision value of the opposite direction), then swaps slot q+9
// with slot q of its neighbour x + c_q for q = 1..9, the neighbours that
// precede it in the sweep and have already reverted.  Every slot is swapped
// exactly once per step, so after the sweep slot q of cell x holds the value
// streamed into x along c_q.  A slot whose partner lies beyond a wall keeps
// its reverted value: halfway bounce-back.
//
// Two merged steps (Sec. 4.1).  Writing first(x) and second(x) for a cell's
// computation at time t and t+1, second(x) needs (a) first() of the nine
// cells that swap into x (its successors x - c_q), so that x holds its whole
// t+1 state, and (b) second() of the nine predecessors x + c_q it swaps with
// at t+1.  The sweep runs first() in an order where every predecessor comes
// first and, after first(x, y, z), runs second() of the cells that have just
// become ready:
//   (x-1, y-1, z-1)                      the cell one further back on every axis;
//   (x-1, y-1, nz-1) when z = nz-1       the last cell of a row;
//   (x-1, ny-1, z-2) when y = ny-1       the last row of a layer: its
//                                        predecessor (x-1, ny-2, z-1) takes
//                                        its second computation only now;
//   (x-1, ny-1, nz-2), (x-1, ny-1, nz-1) when y = ny-1 and z = nz-1;
// and the top layer x = nx-1 takes its second computations after the sweep.
// These are derived from (a) and (b), each trigger being the last cell of the
// sweep that the target depends on; the checked mode verifies (a) and (b)
// before every computation.
//
// Prism traversal (Sec. 4.1, Fig. 3).  In the skewed coordinates
// Y' = y + dx and Z' = z + y + 2 dx (dx = x minus the first layer of a stride
// of `tile' layers) every predecessor of a cell, and every trigger of the
// rules above, has coordinates no larger than the cell's; the sweep visits
// tile^3 boxes of (x, Y', Z') in lexicographic order, and each box in
// lexicographic order, so dependencies still come first, and a box's cells
// (a prism in (x, y, z): parallelogram slices shifted one cell per row and
// per layer) stay in cache between their two computations.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/lbm_cpu.h"

namespace {

constexpr int Q = 19;
constexpr int CX[Q] = {0, -1, 0, 0, -1, -1, -1, -1, 0, 0, 1, 0, 0, 1, 1, 1, 1, 0, 0};
constexpr int CY[Q] = {0, 0, -1, 0, -1, 1, 0, 0, -1, -1, 0, 1, 0, 1, -1, 0, 0, 1, 1};
constexpr int CZ[Q] = {0, 0, 0, -1, 0, 0, -1, 1, -1, 1, 0, 0, 1, 0, 0, 1, -1, 1, -1};

constexpr double weight(int q)
{
    return q == 0 ? 1.0 / 3.0 : (CX[q] * CX[q] + CY[q] * CY[q] + CZ[q] * CZ[q] == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

struct Lat {
    int n[3];
    long long N;
    double omega;
    bool wall[3];   // axis has walls (else periodic)
    int moving;     // moving face 0..5 or -1
    double term[Q]; // -6 w_q (c_q . u_w): added to a population bounced back after leaving along c_q
    double* g;
    // checked mode: 0 = nothing this sweep, 1 = first done, 2 = second done
    std::vector<signed char> state;
    bool checked = false, bad = false;

    double* cell(int x, int y, int z) const { return g + (((long long)x * n[1] + y) * n[2] + z) * Q; }
    long long id(int x, int y, int z) const { return ((long long)x * n[1] + y) * n[2] + z; }
};

// BGK in offset form: g_q = f_q - w_q, delta rho = sum g, j = sum c g,
// g_q <- g_q - omega (g_q - geq_q), geq_q = w_q [drho + rho (3 cu + 4.5 cu^2 - 1.5 u^2)].
// Each direction q = 1..9 is taken with its opposite q + 9: the equilibrium
// splits into a part even in c (shared) and a part odd in c (sign flipped).
inline void collide(double* c, double omega)
{
    double s[10], d[10];
    for (int q = 1; q <= 9; ++q) {
        s[q] = c[q] + c[q + 9];
        d[q] = c[q] - c[q + 9];
    }
    double drho = c[0], jx = 0.0, jy = 0.0, jz = 0.0;
    for (int q = 1; q <= 9; ++q) {
        drho += s[q];
        jx += CX[q] * d[q];
        jy += CY[q] * d[q];
        jz += CZ[q] * d[q];
    }
    const double rho = 1.0 + drho, inv = 1.0 / rho;
    const double ux = jx * inv, uy = jy * inv, uz = jz * inv;
    const double usq = 1.5 * (ux * ux + uy * uy + uz * uz);
    const double omw = 1.0 - omega;
    c[0] = omw * c[0] + omega * weight(0) * (drho - rho * usq);
    for (int q = 1; q <= 9; ++q) {
        const double w = weight(q);
        const double cu = CX[q] * ux + CY[q] * uy + CZ[q] * uz;
        const double even = omega * w * (drho + rho * (4.5 * cu * cu - usq));
        const double odd = omega * w * rho * 3.0 * cu;
        c[q] = omw * c[q] + even + odd;
        c[q + 9] = omw * c[q + 9] + even - odd;
    }
}

inline void revert(double* c)
{
    for (int q = 1; q <= 9; ++q) std::swap(c[q], c[q + 9]);
}

// The link from (x,y,z) along c_q: false if it leaves through a wall (then
// *mv tells whether the moving face is among the faces crossed), else the
// (wrapped) target.
inline bool link(const Lat& L, int x, int y, int z, int q, int* t, bool* mv)
{
    const int p[3] = {x + CX[q], y + CY[q], z + CZ[q]};
    bool inside = true;
    *mv = false;
    for (int a = 0; a < 3; ++a) {
        int v = p[a];
        if (v < 0 || v >= L.n[a]) {
            const int face = 2 * a + (v < 0 ? 0 : 1);
            if (L.wall[a]) {
                inside = false;
                if (face == L.moving) *mv = true;
            } else {
                v = v < 0 ? v + L.n[a] : v - L.n[a];
            }
        }
        t[a] = v;
    }
    return inside;
}

// Bounce-backs of the slots whose partner would be a later cell beyond a
// wall: slot q (q = 1..9) holds the reverted value leaving along c_{q+9}.
inline void successor_walls(const Lat& L, int x, int y, int z, double* c)
{
    for (int q = 1; q <= 9; ++q) {
        int t[3];
        bool mv;
        if (!link(L, x, y, z, q + 9, t, &mv) && mv) c[q] += L.term[q + 9];
    }
}

// Swaps with the nine predecessors (slot q+9 with their slot q), or the
// bounce-back where a predecessor lies beyond a wall.
inline void predecessor_swaps(const Lat& L, int x, int y, int z, double* c)
{
    for (int q = 1; q <= 9; ++q) {
        int t[3];
        bool mv;
        if (link(L, x, y, z, q, t, &mv))
            std::swap(c[q + 9], L.cell(t[0], t[1], t[2])[q]);
        else if (mv)
            c[q + 9] += L.term[q];
    }
}

// Bulk cell: every partner is inside and precedes it; no boundary checks.
inline void bulk_op(const Lat& L, int x, int y, int z)
{
    double* c = L.cell(x, y, z);
    collide(c, L.omega);
    revert(c);
    const long long sx = (long long)L.n[1] * L.n[2] * Q, sy = (long long)L.n[2] * Q, sz = Q;
    for (int q = 1; q <= 9; ++q) std::swap(c[q + 9], c[CX[q] * sx + CY[q] * sy + CZ[q] * sz + q]);
}

bool on_box(const Lat& L, int x, int y, int z)
{
    return x == 0 || y == 0 || z == 0 || x == L.n[0] - 1 || y == L.n[1] - 1 || z == L.n[2] - 1;
}

// collide + swap_stream of one cell, with the boundary checks only on the
// bounding box (Alg. 2's adaptive_collide_stream)
inline void adaptive_op(const Lat& L, int x, int y, int z)
{
    if (on_box(L, x, y, z)) {
        double* c = L.cell(x, y, z);
        collide(c, L.omega);
        revert(c);
        successor_walls(L, x, y, z, c);
        predecessor_swaps(L, x, y, z, c);
    } else {
        bulk_op(L, x, y, z);
    }
}

// ---- Alg. 1: one step ----
void fuse_swap_step(const Lat& L)
{
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2];
    // Stage I: collide and revert on the bounding box (their swaps wait for
    // Stage III, when every partner, across a periodic wrap too, has reverted)
    for (int x = 0; x < nx; ++x)
        for (int y = 0; y < ny; ++y)
            for (int z = 0; z < nz; ++z) {
                if (!on_box(L, x, y, z)) {
                    z = std::max(z, nz - 2);  // jump over the bulk of the row
                    continue;
                }
                double* c = L.cell(x, y, z);
                collide(c, L.omega);
                revert(c);
                successor_walls(L, x, y, z, c);
            }
    // Stage II: the bulk, collide + swap_stream without boundary checks
    for (int x = 1; x < nx - 1; ++x)
        for (int y = 1; y < ny - 1; ++y)
            for (int z = 1; z < nz - 1; ++z) bulk_op(L, x, y, z);
    // Stage III: swap_stream of the bounding box
    for (int x = 0; x < nx; ++x)
        for (int y = 0; y < ny; ++y)
            for (int z = 0; z < nz; ++z) {
                if (!on_box(L, x, y, z)) {
                    z = std::max(z, nz - 2);
                    continue;
                }
                predecessor_swaps(L, x, y, z, L.cell(x, y, z));
            }
}

// ---- Alg. 2 ----
// checked mode: the states the swap algorithm requires of the partners
bool check_first(Lat& L, int x, int y, int z)
{
    if (L.state[L.id(x, y, z)] != 0) return false;
    for (int q = 1; q <= 9; ++q) {
        int t[3];
        bool mv;
        if (link(L, x, y, z, q, t, &mv) && L.state[L.id(t[0], t[1], t[2])] != 1) return false;
    }
    L.state[L.id(x, y, z)] = 1;
    return true;
}

bool check_second(Lat& L, int x, int y, int z)
{
    if (L.state[L.id(x, y, z)] != 1) return false;
    for (int q = 1; q <= 9; ++q) {
        int t[3];
        bool mv;
        if (link(L, x, y, z, q + 9, t, &mv) && L.state[L.id(t[0], t[1], t[2])] < 1) return false;  // (a)
        if (link(L, x, y, z, q, t, &mv) && L.state[L.id(t[0], t[1], t[2])] != 2) return false;     // (b)
    }
    L.state[L.id(x, y, z)] = 2;
    return true;
}

inline void first(Lat& L, int x, int y, int z)
{
    if (L.checked && !check_first(L, x, y, z)) L.bad = true;
    adaptive_op(L, x, y, z);
}

inline void second(Lat& L, int x, int y, int z)
{
    if (L.checked && !check_second(L, x, y, z)) L.bad = true;
    adaptive_op(L, x, y, z);
}

// first(x, y, z) and the second computations it makes ready
inline void visit(Lat& L, int x, int y, int z)
{
    first(L, x, y, z);
    if (x == 0) return;
    const int ny = L.n[1], nz = L.n[2];
    if (y >= 1 && z >= 1) second(L, x - 1, y - 1, z - 1);
    if (z == nz - 1 && y >= 1) second(L, x - 1, y - 1, nz - 1);
    if (y == ny - 1 && z >= 2) second(L, x - 1, ny - 1, z - 2);
    if (y == ny - 1 && z == nz - 1) {
        if (nz >= 2) second(L, x - 1, ny - 1, nz - 2);
        second(L, x - 1, ny - 1, nz - 1);
    }
}

void two_step_sweep(Lat& L, int tile)
{
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2];
    if (L.checked) std::fill(L.state.begin(), L.state.end(), 0);
    if (tile <= 0) {
        for (int x = 0; x < nx; ++x)
            for (int y = 0; y < ny; ++y)
                for (int z = 0; z < nz; ++z) visit(L, x, y, z);
    } else {
        const int T = tile;
        for (int x0 = 0; x0 < nx; x0 += T) {
            const int x1 = std::min(x0 + T, nx);
            const int ymax = ny - 1 + (T - 1), zmax = nz - 1 + ny - 1 + 2 * (T - 1);
            for (int Yb = 0; Yb <= ymax; Yb += T)
                for (int Zb = 0; Zb <= zmax; Zb += T)
                    for (int x = x0; x < x1; ++x) {
                        const int dx = x - x0;
                        const int ylo = std::max(Yb - dx, 0), yhi = std::min(Yb + T - 1 - dx, ny - 1);
                        for (int y = ylo; y <= yhi; ++y) {
                            const int zlo = std::max(Zb - y - 2 * dx, 0);
                            const int zhi = std::min(Zb + T - 1 - y - 2 * dx, nz - 1);
                            for (int z = zlo; z <= zhi; ++z) visit(L, x, y, z);
                        }
                    }
        }
    }
    // the top layer's second computations
    for (int y = 0; y < ny; ++y)
        for (int z = 0; z < nz; ++z) second(L, nx - 1, y, z);
}

lbm_status setup(const lbm_config* cfg, double* g, Lat* L)
{
    if (!cfg || !g) return LBM_EINVAL;
    if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1) return LBM_EINVAL;
    if (!(cfg->tau > 0.5) || !isfinite(cfg->tau)) return LBM_EINVAL;
    if (cfg->use_force) return LBM_EUNSUPPORTED;
    if (cfg->velocities != 0 && cfg->velocities != 19) return LBM_EUNSUPPORTED;  // D3Q19, as the paper
    int moving = -1;
    for (int a = 0; a < 3; ++a) {
        const int lo = cfg->face[2 * a], hi = cfg->face[2 * a + 1];
        if (lo < LBM_PERIODIC || lo > LBM_MOVING_WALL || hi < LBM_PERIODIC || hi > LBM_MOVING_WALL)
            return LBM_EINVAL;
        if ((lo == LBM_PERIODIC) != (hi == LBM_PERIODIC)) return LBM_EINVAL;
        L->wall[a] = lo != LBM_PERIODIC;
        for (int s = 0; s < 2; ++s)
            if (cfg->face[2 * a + s] == LBM_MOVING_WALL) {
                if (moving >= 0) return LBM_EINVAL;
                moving = 2 * a + s;
            }
    }
    L->n[0] = cfg->nx;
    L->n[1] = cfg->ny;
    L->n[2] = cfg->nz;
    L->N = (long long)cfg->nx * cfg->ny * cfg->nz;
    L->omega = 1.0 / cfg->tau;
    L->moving = moving;
    for (int q = 0; q < Q; ++q)
        L->term[q] = -6.0 * weight(q) * (CX[q] * cfg->wall_u[0] + CY[q] * cfg->wall_u[1] + CZ[q] * cfg->wall_u[2]);
    L->g = g;
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_cpu_init(const lbm_config* cfg, double* g, const double* rho0, const double* u0)
{
    Lat L;
    lbm_status st = setup(cfg, g, &L);
    if (st != LBM_OK) return st;
    for (long long i = 0; i < L.N; ++i) {
        const double rho = rho0 ? rho0[i] : 1.0;
        const double ux = u0 ? u0[i] : 0.0, uy = u0 ? u0[L.N + i] : 0.0, uz = u0 ? u0[2 * L.N + i] : 0.0;
        const double usq = ux * ux + uy * uy + uz * uz;
        for (int q = 0; q < Q; ++q) {
            const double cu = CX[q] * ux + CY[q] * uy + CZ[q] * uz;
            g[i * Q + q] = weight(q) * ((rho - 1.0) + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * usq));
        }
    }
    return LBM_OK;
}

lbm_status lbm_cpu_fuse_swap(const lbm_config* cfg, double* g, int64_t n)
{
    Lat L;
    lbm_status st = setup(cfg, g, &L);
    if (st != LBM_OK) return st;
    if (n < 0) return LBM_EINVAL;
    for (int64_t k = 0; k < n; ++k) fuse_swap_step(L);
    return LBM_OK;
}

lbm_status lbm_cpu_two_step(const lbm_config* cfg, double* g, int64_t n, int32_t tile, int32_t checked)
{
    Lat L;
    lbm_status st = setup(cfg, g, &L);
    if (st != LBM_OK) return st;
    if (n < 0 || tile < 0) return LBM_EINVAL;
    if (!L.wall[0] || !L.wall[1] || !L.wall[2]) return LBM_EUNSUPPORTED;
    if (checked) {
        try {
            L.state.assign(size_t(L.N), 0);
        } catch (const std::bad_alloc&) {
            return LBM_EINVAL;
        }
        L.checked = true;
    }
    for (int64_t k = 0; k < n / 2; ++k) {
        two_step_sweep(L, tile);
        if (L.bad) return LBM_ESTATE;
    }
    if (n & 1) fuse_swap_step(L);
    return LBM_OK;
}

}  // extern "C"
