/*
 * lbm_oracle_q.c -- TEST INFRASTRUCTURE ONLY.
 *
 * The plain FP64 two-array BGK update of lbm_oracle.c written once for the
 * three standard cubic velocity sets, D3Q15, D3Q19 and D3Q27, selected at run
 * time.  Sec. 4.1 of Fu & Song ("Designing a 3D Parallel Memory-Aware Lattice
 * Boltzmann Algorithm on Manycore Systems") states that its two-step merging
 * rule holds for D3Q15, D3Q19, D3Q27 and extended lattices alike; this file
 * is the plain definition the GPU library's D3Q15/D3Q27 kernels are checked
 * against.  Only tests/ may load it.  It shares no code, header, table or
 * helper with the HIP library, and none with lbm_oracle.c either (the D3Q19
 * case of this file is checked against that oracle).
 *
 *   velocity sets  rest c_0 = 0; directions 1..H (H = (Q-1)/2) are the
 *                  neighbours that precede a cell in an x-slowest, z-fastest
 *                  sweep, listed below; c_{q+H} = -c_q.
 *     D3Q15  (-1,0,0) (0,-1,0) (0,0,-1) (-1,-1,-1) (-1,-1,1) (-1,1,-1) (-1,1,1)
 *     D3Q19  (-1,0,0) (0,-1,0) (0,0,-1) (-1,-1,0) (-1,1,0) (-1,0,-1) (-1,0,1)
 *            (0,-1,-1) (0,-1,1)
 *     D3Q27  the nine of D3Q19, then (-1,-1,-1) (-1,-1,1) (-1,1,-1) (-1,1,1)
 *   weights  by |c|^2 = 0, 1, 2, 3:
 *     D3Q15  2/9, 1/9, -, 1/72
 *     D3Q19  1/3, 1/18, 1/36, -
 *     D3Q27  8/27, 2/27, 1/54, 1/216
 *   sound speed cs^2 = 1/3 for all three.
 *   moments, equilibrium, BGK with Guo forcing, push streaming, halfway
 *   bounce-back with the moving-face term: exactly as in lbm_oracle.c, with
 *   the sums taken over the chosen set:
 *     rho = sum f, u = (sum c f + F/2)/rho,
 *     feq_q = w_q rho [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u],
 *     f*_q = f_q - (1/tau)(f_q - feq_q) + (1 - 1/(2 tau)) w_q [3 (c_q - u) + 9 (c_q.u) c_q] . F,
 *     f_q(x + c_q, t+1) = f*_q(x) inside or across periodic faces, and
 *     f_opp(q)(x, t+1) = f*_q(x) - 6 w_q (c_q . u_w) where x + c_q leaves
 *     through a wall face (u_w only if the moving face is among those
 *     crossed).
 *
 * Layout: f[q][x][y][z], z fastest, index q*N + (x*ny + y)*nz + z.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>

#define QMAX 27

typedef struct {
    int32_t nx, ny, nz;
    double tau;
    int32_t face[6];  /* -x,+x,-y,+y,-z,+z: 0 periodic, 1 wall, 2 moving wall */
    double wall_u[3];
    int32_t q;        /* 15, 19 or 27 */
} orq_cfg;

typedef struct {
    int Q;
    int c[QMAX][3];
    double w[QMAX];
    int opp[QMAX];
} lattice_t;

static const int NEG15[7][3] = {{-1, 0, 0}, {0, -1, 0}, {0, 0, -1}, {-1, -1, -1}, {-1, -1, 1}, {-1, 1, -1},
                                {-1, 1, 1}};
static const int NEG19[9][3] = {{-1, 0, 0}, {0, -1, 0}, {0, 0, -1}, {-1, -1, 0}, {-1, 1, 0},
                                {-1, 0, -1}, {-1, 0, 1}, {0, -1, -1}, {0, -1, 1}};
static const int NEG27[13][3] = {{-1, 0, 0}, {0, -1, 0}, {0, 0, -1}, {-1, -1, 0}, {-1, 1, 0},
                                 {-1, 0, -1}, {-1, 0, 1}, {0, -1, -1}, {0, -1, 1}, {-1, -1, -1},
                                 {-1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}};

/* builds the table of velocity set q; 0 on success */
static int make_lattice(int q, lattice_t* L)
{
    const int(*neg)[3];
    double wc[4];
    int H;
    if (q == 15) {
        neg = NEG15;
        H = 7;
        wc[0] = 2.0 / 9.0, wc[1] = 1.0 / 9.0, wc[2] = 0.0, wc[3] = 1.0 / 72.0;
    } else if (q == 19) {
        neg = NEG19;
        H = 9;
        wc[0] = 1.0 / 3.0, wc[1] = 1.0 / 18.0, wc[2] = 1.0 / 36.0, wc[3] = 0.0;
    } else if (q == 27) {
        neg = NEG27;
        H = 13;
        wc[0] = 8.0 / 27.0, wc[1] = 2.0 / 27.0, wc[2] = 1.0 / 54.0, wc[3] = 1.0 / 216.0;
    } else {
        return -1;
    }
    L->Q = 2 * H + 1;
    for (int a = 0; a < 3; ++a) L->c[0][a] = 0;
    for (int k = 0; k < H; ++k)
        for (int a = 0; a < 3; ++a) {
            L->c[1 + k][a] = neg[k][a];
            L->c[1 + H + k][a] = -neg[k][a];
        }
    for (int p = 0; p < L->Q; ++p) {
        int c2 = L->c[p][0] * L->c[p][0] + L->c[p][1] * L->c[p][1] + L->c[p][2] * L->c[p][2];
        L->w[p] = wc[c2];
        L->opp[p] = p == 0 ? 0 : (p <= H ? p + H : p - H);
    }
    return 0;
}

/* Q of set q with its velocities (Qx3), weights and opposites; -1 if unknown */
int32_t orq_tables(int32_t q, int32_t* c_out, double* w_out, int32_t* opp_out)
{
    lattice_t L;
    if (make_lattice(q, &L)) return -1;
    for (int p = 0; p < L.Q; ++p) {
        for (int a = 0; a < 3; ++a) c_out[3 * p + a] = L.c[p][a];
        w_out[p] = L.w[p];
        opp_out[p] = L.opp[p];
    }
    return L.Q;
}

int32_t orq_check(const orq_cfg* g)
{
    lattice_t L;
    if (!g || make_lattice(g->q, &L)) return -1;
    if (g->nx < 1 || g->ny < 1 || g->nz < 1 || !(g->tau > 0.5)) return -1;
    int moving = 0;
    for (int a = 0; a < 3; ++a) {
        int lo = g->face[2 * a], hi = g->face[2 * a + 1];
        if (lo < 0 || lo > 2 || hi < 0 || hi > 2) return -1;
        if ((lo == 0) != (hi == 0)) return -1;
        moving += (lo == 2) + (hi == 2);
    }
    return moving > 1 ? -1 : 0;
}

static size_t ncell(const orq_cfg* g)
{
    return (size_t)g->nx * (size_t)g->ny * (size_t)g->nz;
}

static void equilibrium(const lattice_t* L, double rho, const double* u, double* feq)
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int q = 0; q < L->Q; ++q) {
        double cu = L->c[q][0] * u[0] + L->c[q][1] * u[1] + L->c[q][2] * u[2];
        feq[q] = L->w[q] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

static void moments(const lattice_t* L, const double* f, const double* F, double* rho, double u[3])
{
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < L->Q; ++q) {
        r += f[q];
        for (int a = 0; a < 3; ++a) j[a] += L->c[q][a] * f[q];
    }
    *rho = r;
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + (F ? 0.5 * F[a] : 0.0)) / r;
}

int32_t orq_init(const orq_cfg* g, const double* rho0, const double* u0, double* f)
{
    lattice_t L;
    if (orq_check(g)) return -1;
    make_lattice(g->q, &L);
    size_t N = ncell(g);
    for (size_t i = 0; i < N; ++i) {
        double u[3] = {0.0, 0.0, 0.0}, feq[QMAX];
        if (u0)
            for (int a = 0; a < 3; ++a) u[a] = u0[a * N + i];
        equilibrium(&L, rho0 ? rho0[i] : 1.0, u, feq);
        for (int q = 0; q < L.Q; ++q) f[q * N + i] = feq[q];
    }
    return 0;
}

/* fpost := collision of every cell (F may be NULL) */
int32_t orq_collide(const orq_cfg* g, const double* F, const double* f, double* fpost)
{
    lattice_t L;
    if (orq_check(g)) return -1;
    make_lattice(g->q, &L);
    size_t N = ncell(g);
    double omega = 1.0 / g->tau;
    for (size_t i = 0; i < N; ++i) {
        double fc[QMAX], feq[QMAX], Fc[3] = {0.0, 0.0, 0.0}, rho, u[3];
        for (int q = 0; q < L.Q; ++q) fc[q] = f[q * N + i];
        if (F)
            for (int a = 0; a < 3; ++a) Fc[a] = F[a * N + i];
        moments(&L, fc, F ? Fc : NULL, &rho, u);
        equilibrium(&L, rho, u, feq);
        for (int q = 0; q < L.Q; ++q) {
            double s = 0.0;
            if (F) {
                double cu = L.c[q][0] * u[0] + L.c[q][1] * u[1] + L.c[q][2] * u[2];
                for (int a = 0; a < 3; ++a) s += (3.0 * (L.c[q][a] - u[a]) + 9.0 * cu * L.c[q][a]) * Fc[a];
                s *= (1.0 - 0.5 * omega) * L.w[q];
            }
            fpost[q * N + i] = fc[q] - omega * (fc[q] - feq[q]) + s;
        }
    }
    return 0;
}

/* fout := push streaming of fpost with periodic wrap and bounce-back */
int32_t orq_stream(const orq_cfg* g, const double* fpost, double* fout)
{
    lattice_t L;
    if (orq_check(g)) return -1;
    make_lattice(g->q, &L);
    size_t N = ncell(g);
    int n[3] = {g->nx, g->ny, g->nz};
    for (int x = 0; x < g->nx; ++x)
        for (int y = 0; y < g->ny; ++y)
            for (int z = 0; z < g->nz; ++z) {
                size_t i = ((size_t)x * g->ny + y) * g->nz + z;
                for (int q = 0; q < L.Q; ++q) {
                    int p[3] = {x + L.c[q][0], y + L.c[q][1], z + L.c[q][2]};
                    int inside = 1, moving = 0;
                    for (int a = 0; a < 3; ++a) {
                        if (p[a] >= 0 && p[a] < n[a]) continue;
                        int face = 2 * a + (p[a] >= n[a]);
                        if (g->face[face] == 0) {
                            p[a] = (p[a] + n[a]) % n[a];
                        } else {
                            inside = 0;
                            if (g->face[face] == 2) moving = 1;
                        }
                    }
                    if (inside) {
                        fout[q * N + ((size_t)p[0] * g->ny + p[1]) * g->nz + p[2]] = fpost[q * N + i];
                    } else {
                        double cu = L.c[q][0] * g->wall_u[0] + L.c[q][1] * g->wall_u[1] + L.c[q][2] * g->wall_u[2];
                        fout[L.opp[q] * N + i] = fpost[q * N + i] - (moving ? 6.0 * L.w[q] * cu : 0.0);
                    }
                }
            }
    return 0;
}

int32_t orq_run(const orq_cfg* g, const double* F, double* f, double* tmp, int64_t nsteps)
{
    if (orq_check(g) || nsteps < 0) return -1;
    for (int64_t s = 0; s < nsteps; ++s) {
        orq_collide(g, F, f, tmp);
        orq_stream(g, tmp, f);
    }
    return 0;
}

int32_t orq_macro(const orq_cfg* g, const double* F, const double* f, double* rho, double* u, double* unorm)
{
    lattice_t L;
    if (orq_check(g)) return -1;
    make_lattice(g->q, &L);
    size_t N = ncell(g);
    for (size_t i = 0; i < N; ++i) {
        double fc[QMAX], Fc[3] = {0.0, 0.0, 0.0}, r, uc[3];
        for (int q = 0; q < L.Q; ++q) fc[q] = f[q * N + i];
        if (F)
            for (int a = 0; a < 3; ++a) Fc[a] = F[a * N + i];
        moments(&L, fc, F ? Fc : NULL, &r, uc);
        if (rho) rho[i] = r;
        if (u)
            for (int a = 0; a < 3; ++a) u[a * N + i] = uc[a];
        if (unorm) unorm[i] = sqrt(uc[0] * uc[0] + uc[1] * uc[1] + uc[2] * uc[2]);
    }
    return 0;
}

/* { sum rho, sum j } over the populations, Kahan-compensated */
int32_t orq_sums(const orq_cfg* g, const double* f, double* out)
{
    lattice_t L;
    if (orq_check(g)) return -1;
    make_lattice(g->q, &L);
    size_t N = ncell(g);
    double s[4] = {0, 0, 0, 0}, c[4] = {0, 0, 0, 0};
    for (size_t i = 0; i < N; ++i)
        for (int q = 0; q < L.Q; ++q) {
            double v[4] = {f[q * N + i], L.c[q][0] * f[q * N + i], L.c[q][1] * f[q * N + i], L.c[q][2] * f[q * N + i]};
            for (int k = 0; k < 4; ++k) {
                double y = v[k] - c[k];
                double t = s[k] + y;
                c[k] = (t - s[k]) - y;
                s[k] = t;
            }
        }
    for (int k = 0; k < 4; ++k) out[k] = s[k];
    return 0;
}

/* ---- discrete adjoint of one step f_{t+1} = S(C(f_t; F)) over the set ----
 *
 * For the loss of the final velocity L = sum_x |u(x,T) - u*(x)|^2, written
 * from the chain rule with rho = sum f, u = (sum c f + F/2)/rho, so that
 * d rho / d f_j = 1, d u / d f_j = (c_j - u)/rho and d u / d F = 1/(2 rho):
 *   seed      lambda_q(T) = 2 (u - u*) . (c_q - u)/rho,  dL/dF += (u - u*)/rho
 *   stream^T  the push moves f*_q(x) to x + c_q, or to slot opp(q) of x where
 *             the link leaves through a wall (minus a constant), so
 *             mu_q(x) = lambda_q(x + c_q, t+1) or lambda_opp(q)(x, t+1)
 *   collide^T f*_q = (1 - omega) f_q + omega feq_q(rho, u) + S_q(u, F), with
 *             d feq_q / d rho = feq_q / rho,
 *             d feq_q / d u = w_q rho (3 c_q + 9 (c_q.u) c_q - 3 u),
 *             d S_q / d u  = (1 - omega/2) w_q (9 (c_q.F) c_q - 3 F),
 *             d S_q / d F  = (1 - omega/2) w_q (3 (c_q - u) + 9 (c_q.u) c_q):
 *     a_rho = sum_q mu_q omega feq_q / rho
 *     a_u   = sum_q mu_q [omega d feq_q / d u + d S_q / d u]
 *     lambda_j(t) = (1 - omega) mu_j + a_rho + a_u . (c_j - u)/rho
 *     dL/dF += sum_q mu_q d S_q / d F + a_u / (2 rho)
 */

static void cell_state(const lattice_t* L, const double* f, size_t N, size_t i, const double* F, double* fc,
                       double* Fc, double* rho, double u[3])
{
    for (int q = 0; q < L->Q; ++q) fc[q] = f[q * N + i];
    Fc[0] = Fc[1] = Fc[2] = 0.0;
    if (F)
        for (int a = 0; a < 3; ++a) Fc[a] = F[a * N + i];
    moments(L, fc, F ? Fc : NULL, rho, u);
}

double orq_loss(const orq_cfg* g, const double* F, const double* f, const double* utarget)
{
    lattice_t L;
    if (orq_check(g)) return NAN;
    make_lattice(g->q, &L);
    size_t N = ncell(g);
    double s = 0.0;
    for (size_t i = 0; i < N; ++i) {
        double fc[QMAX], Fc[3], rho, u[3];
        cell_state(&L, f, N, i, F, fc, Fc, &rho, u);
        for (int a = 0; a < 3; ++a) {
            double d = u[a] - utarget[a * N + i];
            s += d * d;
        }
    }
    return s;
}

/* lambda := dL/df of the final state (Q N values); gF += the direct dL/dF */
int32_t orq_loss_seed(const orq_cfg* g, const double* F, const double* f, const double* utarget, double* lambda,
                      double* gF)
{
    lattice_t L;
    if (orq_check(g)) return -1;
    make_lattice(g->q, &L);
    size_t N = ncell(g);
    for (size_t i = 0; i < N; ++i) {
        double fc[QMAX], Fc[3], rho, u[3], d[3];
        cell_state(&L, f, N, i, F, fc, Fc, &rho, u);
        for (int a = 0; a < 3; ++a) d[a] = u[a] - utarget[a * N + i];
        for (int q = 0; q < L.Q; ++q) {
            double s = 0.0;
            for (int a = 0; a < 3; ++a) s += d[a] * (L.c[q][a] - u[a]);
            lambda[q * N + i] = 2.0 * s / rho;
        }
        if (gF)
            for (int a = 0; a < 3; ++a) gF[a * N + i] += d[a] / rho;
    }
    return 0;
}

/* One reverse step: lambda holds lambda_{t+1} on entry and lambda_t on exit;
 * f_t is the state before the forward step; mu is Q N scratch; gF += this
 * step's dL/dF (may be NULL). */
int32_t orq_adjoint_step(const orq_cfg* g, const double* F, const double* f_t, double* lambda, double* mu,
                         double* gF)
{
    lattice_t L;
    if (orq_check(g)) return -1;
    make_lattice(g->q, &L);
    size_t N = ncell(g);
    int n[3] = {g->nx, g->ny, g->nz};
    const double omega = 1.0 / g->tau, kf = 1.0 - 0.5 * omega;
    /* stream^T */
    for (int x = 0; x < g->nx; ++x)
        for (int y = 0; y < g->ny; ++y)
            for (int z = 0; z < g->nz; ++z) {
                size_t i = ((size_t)x * g->ny + y) * g->nz + z;
                for (int q = 0; q < L.Q; ++q) {
                    int p[3] = {x + L.c[q][0], y + L.c[q][1], z + L.c[q][2]};
                    int inside = 1;
                    for (int a = 0; a < 3; ++a) {
                        if (p[a] >= 0 && p[a] < n[a]) continue;
                        if (g->face[2 * a + (p[a] >= n[a])] == 0)
                            p[a] = (p[a] + n[a]) % n[a];
                        else
                            inside = 0;
                    }
                    mu[q * N + i] = inside ? lambda[q * N + ((size_t)p[0] * g->ny + p[1]) * g->nz + p[2]]
                                           : lambda[L.opp[q] * N + i];
                }
            }
    /* collide^T, cell by cell */
    for (size_t i = 0; i < N; ++i) {
        double fc[QMAX], Fc[3], rho, u[3], feq[QMAX];
        cell_state(&L, f_t, N, i, F, fc, Fc, &rho, u);
        equilibrium(&L, rho, u, feq);
        double a_rho = 0.0, a_u[3] = {0.0, 0.0, 0.0}, dF[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < L.Q; ++q) {
            const double m = mu[q * N + i];
            const double cu = L.c[q][0] * u[0] + L.c[q][1] * u[1] + L.c[q][2] * u[2];
            const double cF = L.c[q][0] * Fc[0] + L.c[q][1] * Fc[1] + L.c[q][2] * Fc[2];
            a_rho += m * omega * feq[q] / rho;
            for (int a = 0; a < 3; ++a) {
                const double dfeq = L.w[q] * rho * (3.0 * L.c[q][a] + 9.0 * cu * L.c[q][a] - 3.0 * u[a]);
                const double dS = F ? kf * L.w[q] * (9.0 * cF * L.c[q][a] - 3.0 * Fc[a]) : 0.0;
                a_u[a] += m * (omega * dfeq + dS);
                dF[a] += m * kf * L.w[q] * (3.0 * (L.c[q][a] - u[a]) + 9.0 * cu * L.c[q][a]);
            }
        }
        for (int j = 0; j < L.Q; ++j) {
            double s = 0.0;
            for (int a = 0; a < 3; ++a) s += a_u[a] * (L.c[j][a] - u[a]);
            lambda[j * N + i] = (1.0 - omega) * mu[j * N + i] + a_rho + s / rho;
        }
        if (gF)
            for (int a = 0; a < 3; ++a) gF[a * N + i] += dF[a] + a_u[a] / (2.0 * rho);
    }
    return 0;
}
