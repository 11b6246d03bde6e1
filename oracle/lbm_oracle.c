/*
 * lbm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct FP64 CPU implementation of what the GPU
 * path computes: N time steps of the D3Q19 BGK lattice Boltzmann update, with
 * two arrays and separate collide and stream loops, plus its discrete adjoint.
 * Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may
 * load it.  It shares no code, header, table or helper with the HIP library.
 *
 * Source of the method: Fu & Song, "Designing a 3D Parallel Memory-Aware
 * Lattice Boltzmann Algorithm on Manycore Systems".  Sec. 3 (Fuse Swap LBM,
 * Alg. 1) defines one step as a per-cell `collide' followed by streaming to the
 * neighbours; Sec. 4 merges two such steps per sweep and, in Sec. 5.1, states
 * that the merged in-place algorithms give the same result as the plain
 * single-step solvers.  The paper gives no collision formula, velocity table
 * or boundary formula, so this file writes out the textbook D3Q19 BGK model
 * that the in-place method reaches exactly:
 *
 *   velocities  c_0 = 0; c_1..c_9 = (-1,0,0) (0,-1,0) (0,0,-1) (-1,-1,0)
 *               (-1,1,0) (-1,0,-1) (-1,0,1) (0,-1,-1) (0,-1,1); c_{q+9} = -c_q.
 *               Directions 1..9 point to the neighbours that precede a cell in
 *               an x-slowest, z-fastest sweep, the "half of the neighbours" a
 *               cell swaps with in Sec. 3 (Fig. 1a); direction 9 is the
 *               lower-right Y-Z neighbour named in Sec. 4.1.
 *   weights     w_0 = 1/3, w = 1/18 for |c|^2 = 1, w = 1/36 for |c|^2 = 2.
 *   moments     rho = sum f, j = sum c f, u = (j + F/2)/rho.
 *   equilibrium feq_q = w_q rho [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u].
 *   collide     f*_q = f_q - (1/tau)(f_q - feq_q) + S_q, Guo forcing
 *               S_q = (1 - 1/(2 tau)) w_q [3 (c_q - u) + 9 (c_q.u) c_q] . F.
 *   stream      f_q(x + c_q, t+1) = f*_q(x, t) (push); periodic axes wrap.
 *   walls       halfway bounce-back: a population whose target leaves the box
 *               through a wall face returns to its own cell reversed,
 *               f_opp(q)(x, t+1) = f*_q(x, t) - 6 w_q (c_q . u_w) with the
 *               wall density 1; u_w is the velocity of the moving face and
 *               enters whenever the moving face is among the faces crossed.
 *               With every face a wall, this is exactly what the swap
 *               algorithm of Sec. 3 leaves in the slots that find no partner.
 *
 * Layout (an interface shared with the GPU library by specification only):
 * f[q][x][y][z], z fastest, index q*N + (x*ny + y)*nz + z, N = nx*ny*nz.
 * Vector fields (u, F, gradients) are SoA: a[c*N + cell], c = 0,1,2.
 *
 * Discrete adjoint of one step f_{t+1} = S(C(f_t; F)), for a loss of the
 * final velocity L = sum_x |u(x,T) - u*(x)|^2, written from the chain rule:
 *   seed     lambda_q(T) = 2 (u - u*) . (c_q - u) / rho,  dL/dF += (u - u*)/rho
 *   stream^T mu_q(x) = lambda_q(x + c_q, t+1), or lambda_opp(q)(x, t+1) on a
 *            wall link (the wall term is constant and has no derivative)
 *   collide^T, with omega = 1/tau:
 *            g_rho = sum_q mu_q omega feq_q / rho
 *            g_u   = sum_q mu_q [omega w_q rho (3 c_q + 9 (c_q.u) c_q - 3 u)
 *                                + (1 - omega/2) w_q (9 (c_q.F) c_q - 3 F)]
 *            lambda_j(t) = (1 - omega) mu_j + g_rho + g_u . (c_j - u)/rho
 *            dL/dF += sum_q mu_q (1 - omega/2) w_q [3 (c_q - u) + 9 (c_q.u) c_q]
 *                     + g_u / (2 rho)
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19

typedef struct {
    int32_t nx, ny, nz;
    double tau;
    int32_t face[6];  /* -x,+x,-y,+y,-z,+z: 0 periodic, 1 wall, 2 moving wall */
    double wall_u[3]; /* velocity of the moving-wall face */
} orc_cfg;

static const int CV[Q][3] = {
    {0, 0, 0},
    {-1, 0, 0}, {0, -1, 0}, {0, 0, -1}, {-1, -1, 0}, {-1, 1, 0},
    {-1, 0, -1}, {-1, 0, 1}, {0, -1, -1}, {0, -1, 1},
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, -1, 0},
    {1, 0, 1}, {1, 0, -1}, {0, 1, 1}, {0, 1, -1}};

static double W[Q];
static int OPP[Q];
static int tables_ready = 0;
static int n_threads = 1;

static void tables(void)
{
    if (tables_ready) return;
    for (int q = 0; q < Q; ++q) {
        int c2 = CV[q][0] * CV[q][0] + CV[q][1] * CV[q][1] + CV[q][2] * CV[q][2];
        W[q] = (c2 == 0) ? 1.0 / 3.0 : (c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        for (int p = 0; p < Q; ++p)
            if (CV[p][0] == -CV[q][0] && CV[p][1] == -CV[q][1] && CV[p][2] == -CV[q][2])
                OPP[q] = p;
    }
    tables_ready = 1;
}

/* ---- tables, exported so tests can check them against closed forms ---- */
void orc_tables(int32_t* c_out /* 19x3 */, double* w_out /* 19 */, int32_t* opp_out /* 19 */)
{
    tables();
    for (int q = 0; q < Q; ++q) {
        for (int a = 0; a < 3; ++a) c_out[3 * q + a] = CV[q][a];
        w_out[q] = W[q];
        opp_out[q] = OPP[q];
    }
}

void orc_set_threads(int32_t n)
{
    n_threads = n < 1 ? 1 : n;
}

int32_t orc_threads(void)
{
    return n_threads;
}

/* 0 if the configuration is valid, -1 otherwise. */
int32_t orc_check(const orc_cfg* g)
{
    if (!g || g->nx < 1 || g->ny < 1 || g->nz < 1 || !(g->tau > 0.5)) return -1;
    int moving = 0;
    for (int a = 0; a < 3; ++a) {
        int lo = g->face[2 * a], hi = g->face[2 * a + 1];
        if (lo < 0 || lo > 2 || hi < 0 || hi > 2) return -1;
        if ((lo == 0) != (hi == 0)) return -1;
        moving += (lo == 2) + (hi == 2);
    }
    return moving > 1 ? -1 : 0;
}

/* ---- per-cell physics ---- */

static void moments(const double* f, const double* F, double* rho, double u[3])
{
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < Q; ++q) {
        r += f[q];
        for (int a = 0; a < 3; ++a) j[a] += CV[q][a] * f[q];
    }
    *rho = r;
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + (F ? 0.5 * F[a] : 0.0)) / r;
}

void orc_equilibrium(double rho, const double* u, double* feq)
{
    tables();
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int q = 0; q < Q; ++q) {
        double cu = CV[q][0] * u[0] + CV[q][1] * u[1] + CV[q][2] * u[2];
        feq[q] = W[q] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* BGK collision of one cell with Guo forcing (F may be NULL). */
void orc_collide_cell(const orc_cfg* g, const double* f, const double* F, double* out)
{
    tables();
    double rho, u[3], feq[Q];
    double omega = 1.0 / g->tau;
    moments(f, F, &rho, u);
    orc_equilibrium(rho, u, feq);
    for (int q = 0; q < Q; ++q) {
        double s = 0.0;
        if (F) {
            double cu = CV[q][0] * u[0] + CV[q][1] * u[1] + CV[q][2] * u[2];
            for (int a = 0; a < 3; ++a)
                s += (3.0 * (CV[q][a] - u[a]) + 9.0 * cu * CV[q][a]) * F[a];
            s *= (1.0 - 0.5 * omega) * W[q];
        }
        out[q] = f[q] - omega * (f[q] - feq[q]) + s;
    }
}

/* ---- whole-lattice operations ---- */

#define CELL(g, x, y, z) ((((size_t)(x)) * (size_t)(g)->ny + (size_t)(y)) * (size_t)(g)->nz + (size_t)(z))

static size_t ncell(const orc_cfg* g)
{
    return (size_t)g->nx * (size_t)g->ny * (size_t)g->nz;
}

/* f := feq(rho0, u0); rho0 may be NULL (1), u0 may be NULL (0). */
int32_t orc_init(const orc_cfg* g, const double* rho0, const double* u0, double* f)
{
    if (orc_check(g)) return -1;
    tables();
    size_t N = ncell(g);
    for (size_t i = 0; i < N; ++i) {
        double u[3] = {0.0, 0.0, 0.0}, feq[Q];
        if (u0)
            for (int a = 0; a < 3; ++a) u[a] = u0[a * N + i];
        orc_equilibrium(rho0 ? rho0[i] : 1.0, u, feq);
        for (int q = 0; q < Q; ++q) f[q * N + i] = feq[q];
    }
    return 0;
}

/* fpost := C(f) for every cell. */
int32_t orc_collide(const orc_cfg* g, const double* F, const double* f, double* fpost)
{
    if (orc_check(g)) return -1;
    tables();
    size_t N = ncell(g);
#pragma omp parallel for num_threads(n_threads) schedule(static)
    for (long long i = 0; i < (long long)N; ++i) {
        double fc[Q], out[Q], Fc[3];
        for (int q = 0; q < Q; ++q) fc[q] = f[q * N + i];
        if (F)
            for (int a = 0; a < 3; ++a) Fc[a] = F[a * N + i];
        orc_collide_cell(g, fc, F ? Fc : NULL, out);
        for (int q = 0; q < Q; ++q) fpost[q * N + i] = out[q];
    }
    return 0;
}

/* Target of the link leaving cell (x,y,z) along c_q.  Returns 1 and the target
 * cell index if the link stays in the box (after periodic wrapping); returns
 * 0 if it leaves through one or more wall faces, and then *moving is set if
 * the moving-wall face is among them. */
static int link_target(const orc_cfg* g, int x, int y, int z, int q, size_t* target, int* moving)
{
    int p[3] = {x + CV[q][0], y + CV[q][1], z + CV[q][2]};
    int n[3] = {g->nx, g->ny, g->nz};
    int inside = 1;
    *moving = 0;
    for (int a = 0; a < 3; ++a) {
        if (p[a] >= 0 && p[a] < n[a]) continue;
        int face = 2 * a + (p[a] >= n[a]);
        if (g->face[face] == 0) {
            p[a] = (p[a] + n[a]) % n[a];
        } else {
            inside = 0;
            if (g->face[face] == 2) *moving = 1;
        }
    }
    if (inside) *target = CELL(g, p[0], p[1], p[2]);
    return inside;
}

/* fout := S(fpost), push streaming with periodic wrap and bounce-back. */
int32_t orc_stream(const orc_cfg* g, const double* fpost, double* fout)
{
    if (orc_check(g)) return -1;
    tables();
    size_t N = ncell(g);
#pragma omp parallel for num_threads(n_threads) schedule(static)
    for (int x = 0; x < g->nx; ++x)
        for (int y = 0; y < g->ny; ++y)
            for (int z = 0; z < g->nz; ++z) {
                size_t i = CELL(g, x, y, z);
                for (int q = 0; q < Q; ++q) {
                    size_t t;
                    int moving;
                    if (link_target(g, x, y, z, q, &t, &moving)) {
                        fout[q * N + t] = fpost[q * N + i];
                    } else {
                        double cu = CV[q][0] * g->wall_u[0] + CV[q][1] * g->wall_u[1] +
                                    CV[q][2] * g->wall_u[2];
                        fout[OPP[q] * N + i] = fpost[q * N + i] - (moving ? 6.0 * W[q] * cu : 0.0);
                    }
                }
            }
    return 0;
}

/* nsteps plain steps; the state stays in f, tmp (19N) holds post-collision. */
int32_t orc_run(const orc_cfg* g, const double* F, double* f, double* tmp, int64_t nsteps)
{
    if (orc_check(g) || nsteps < 0) return -1;
    for (int64_t s = 0; s < nsteps; ++s) {
        orc_collide(g, F, f, tmp);
        orc_stream(g, tmp, f);
    }
    return 0;
}

/* rho, u = (j + F/2)/rho and |u| per cell; any output may be NULL. */
int32_t orc_macro(const orc_cfg* g, const double* F, const double* f, double* rho, double* u, double* unorm)
{
    if (orc_check(g)) return -1;
    tables();
    size_t N = ncell(g);
#pragma omp parallel for num_threads(n_threads) schedule(static)
    for (long long i = 0; i < (long long)N; ++i) {
        double fc[Q], Fc[3], r, uc[3];
        for (int q = 0; q < Q; ++q) fc[q] = f[q * N + i];
        if (F)
            for (int a = 0; a < 3; ++a) Fc[a] = F[a * N + i];
        moments(fc, F ? Fc : NULL, &r, uc);
        if (rho) rho[i] = r;
        if (u)
            for (int a = 0; a < 3; ++a) u[a * N + i] = uc[a];
        if (unorm) unorm[i] = sqrt(uc[0] * uc[0] + uc[1] * uc[1] + uc[2] * uc[2]);
    }
    return 0;
}

/* out = { sum rho, sum j_x, sum j_y, sum j_z } with j = sum_q c_q f_q
 * (populations only, no force shift), Kahan-compensated. */
int32_t orc_sums(const orc_cfg* g, const double* f, double* out)
{
    if (orc_check(g)) return -1;
    tables();
    size_t N = ncell(g);
    double s[4] = {0, 0, 0, 0}, c[4] = {0, 0, 0, 0};
    for (size_t i = 0; i < N; ++i)
        for (int q = 0; q < Q; ++q) {
            double v[4] = {f[q * N + i], CV[q][0] * f[q * N + i], CV[q][1] * f[q * N + i],
                           CV[q][2] * f[q * N + i]};
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

/* ---- discrete adjoint ---- */

/* L = sum_x sum_a (u_a(x) - u*_a(x))^2 of the state f. */
double orc_loss(const orc_cfg* g, const double* F, const double* f, const double* utarget)
{
    tables();
    size_t N = ncell(g);
    double L = 0.0;
    for (size_t i = 0; i < N; ++i) {
        double fc[Q], Fc[3], r, uc[3];
        for (int q = 0; q < Q; ++q) fc[q] = f[q * N + i];
        if (F)
            for (int a = 0; a < 3; ++a) Fc[a] = F[a * N + i];
        moments(fc, F ? Fc : NULL, &r, uc);
        for (int a = 0; a < 3; ++a) {
            double d = uc[a] - utarget[a * N + i];
            L += d * d;
        }
    }
    return L;
}

/* lambda := dL/df of the final state; gradF += the direct dL/dF (F may be
 * NULL, then gradF may be NULL too). */
int32_t orc_loss_seed(const orc_cfg* g, const double* F, const double* f, const double* utarget,
                      double* lambda, double* gradF)
{
    if (orc_check(g)) return -1;
    tables();
    size_t N = ncell(g);
#pragma omp parallel for num_threads(n_threads) schedule(static)
    for (long long i = 0; i < (long long)N; ++i) {
        double fc[Q], Fc[3], r, uc[3], d[3];
        for (int q = 0; q < Q; ++q) fc[q] = f[q * N + i];
        if (F)
            for (int a = 0; a < 3; ++a) Fc[a] = F[a * N + i];
        moments(fc, F ? Fc : NULL, &r, uc);
        for (int a = 0; a < 3; ++a) d[a] = uc[a] - utarget[a * N + i];
        for (int q = 0; q < Q; ++q) {
            double s = 0.0;
            for (int a = 0; a < 3; ++a) s += 2.0 * d[a] * (CV[q][a] - uc[a]) / r;
            lambda[q * N + i] = s;
        }
        if (gradF)
            for (int a = 0; a < 3; ++a) gradF[a * N + i] += d[a] / r;
    }
    return 0;
}

/* mu := S^T lambda_next (the transpose of orc_stream's linear part). */
int32_t orc_stream_adjoint(const orc_cfg* g, const double* lambda_next, double* mu)
{
    if (orc_check(g)) return -1;
    tables();
    size_t N = ncell(g);
#pragma omp parallel for num_threads(n_threads) schedule(static)
    for (int x = 0; x < g->nx; ++x)
        for (int y = 0; y < g->ny; ++y)
            for (int z = 0; z < g->nz; ++z) {
                size_t i = CELL(g, x, y, z);
                for (int q = 0; q < Q; ++q) {
                    size_t t;
                    int moving;
                    if (link_target(g, x, y, z, q, &t, &moving))
                        mu[q * N + i] = lambda_next[q * N + t];
                    else
                        mu[q * N + i] = lambda_next[OPP[q] * N + i];
                }
            }
    return 0;
}

/* Adjoint of orc_collide_cell at pre-collision state f: given mu = dL/df*,
 * lam := dL/df and gF += dL/dF (F and gF may be NULL). */
void orc_collide_adjoint_cell(const orc_cfg* g, const double* f, const double* F, const double* mu,
                              double* lam, double* gF)
{
    tables();
    double rho, u[3], feq[Q];
    double omega = 1.0 / g->tau;
    double Fz[3] = {0.0, 0.0, 0.0};
    const double* Fv = F ? F : Fz;
    moments(f, F, &rho, u);
    orc_equilibrium(rho, u, feq);
    double g_rho = 0.0, g_u[3] = {0.0, 0.0, 0.0}, g_F[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < Q; ++q) {
        double cu = CV[q][0] * u[0] + CV[q][1] * u[1] + CV[q][2] * u[2];
        double cF = CV[q][0] * Fv[0] + CV[q][1] * Fv[1] + CV[q][2] * Fv[2];
        g_rho += mu[q] * omega * feq[q] / rho;
        for (int a = 0; a < 3; ++a) {
            double dfeq = W[q] * rho * (3.0 * CV[q][a] + 9.0 * cu * CV[q][a] - 3.0 * u[a]);
            double dS = (1.0 - 0.5 * omega) * W[q] * (9.0 * cF * CV[q][a] - 3.0 * Fv[a]);
            g_u[a] += mu[q] * (omega * dfeq + dS);
            g_F[a] += mu[q] * (1.0 - 0.5 * omega) * W[q] * (3.0 * (CV[q][a] - u[a]) + 9.0 * cu * CV[q][a]);
        }
    }
    for (int j = 0; j < Q; ++j) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a) s += g_u[a] * (CV[j][a] - u[a]) / rho;
        lam[j] = (1.0 - omega) * mu[j] + g_rho + s;
    }
    if (gF)
        for (int a = 0; a < 3; ++a) gF[a] += g_F[a] + g_u[a] / (2.0 * rho);
}

/* One reverse step: lambda holds lambda_{t+1} on entry and lambda_t on exit;
 * f_t is the state before the forward step; tmp is 19N scratch; gradF += . */
int32_t orc_adjoint_step(const orc_cfg* g, const double* F, const double* f_t, double* lambda,
                         double* tmp, double* gradF)
{
    if (orc_check(g)) return -1;
    tables();
    size_t N = ncell(g);
    orc_stream_adjoint(g, lambda, tmp);
#pragma omp parallel for num_threads(n_threads) schedule(static)
    for (long long i = 0; i < (long long)N; ++i) {
        double fc[Q], mu[Q], lam[Q], Fc[3], gF[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < Q; ++q) {
            fc[q] = f_t[q * N + i];
            mu[q] = tmp[q * N + i];
        }
        if (F)
            for (int a = 0; a < 3; ++a) Fc[a] = F[a * N + i];
        orc_collide_adjoint_cell(g, fc, F ? Fc : NULL, mu, lam, gF);
        for (int q = 0; q < Q; ++q) lambda[q * N + i] = lam[q];
        if (gradF)
            for (int a = 0; a < 3; ++a) gradF[a * N + i] += gF[a];
    }
    return 0;
}
