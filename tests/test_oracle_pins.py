"""Pins of the FP64 CPU oracle against facts fixed by the paper and by the
mathematics of the lattice Boltzmann method -- never against the oracle's own
formulas retyped.  Each test names what it pins.

* D3Q19 table: lattice isotropy identities (closed forms) and the paper's
  direction convention (directions 1..9 precede a cell in the sweep, Sec. 3;
  direction 9 is the lower-right Y-Z neighbour, Sec. 4.1).
* Equilibrium: its velocity moments (closed forms of the 2nd-order model).
* Collide + stream: exact invariants (mass, momentum, momentum gain under a
  body force), the uniform-equilibrium fixed point, axis-permutation symmetry.
* Viscosity nu = (tau - 1/2)/3: decay rates of a shear wave and of 2D
  Taylor-Green vortices; the curvature of Poiseuille flow (exact at any tau)
  and the full profile at tau = 1/2 + sqrt(3/16), where halfway bounce-back is
  exact; linear Couette flow under a moving wall.
* Streaming and bounce-back: brute force against the paper's own in-place
  procedure (collide, revert, swap with the nine preceding neighbours; Sec. 3,
  Alg. 1) and against the two-step merged sweep (Sec. 4.1), whose results the
  paper states equal the plain solver's (Sec. 5.1).
* Discrete adjoint: the dot-product identity of the streaming transpose,
  per-cell Jacobians and the whole-run gradient against central differences.
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
from oracle import MOVING_WALL, PERIODIC, WALL, Oracle
from paper_2208_05429_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# D3Q19 table and equilibrium
# --------------------------------------------------------------------------

def test_lattice_isotropy_identities():
    c, w, opp = oracle.tables()
    c = c.astype(np.float64)
    d = np.eye(3)
    assert abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(np.einsum("q,qa->a", w, c), 0.0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("q,qa,qb->ab", w, c, c), d / 3.0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("q,qa,qb,qc->abc", w, c, c, c), 0.0, atol=1e-16)
    four = np.einsum("q,qa,qb,qc,qd->abcd", w, c, c, c, c)
    expect = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9.0
    np.testing.assert_allclose(four, expect, atol=1e-16)
    # 19 distinct velocities with |c|^2 <= 2 and no (+-1,+-1,+-1)
    assert len({tuple(v) for v in c.astype(int)}) == 19
    assert all((v ** 2).sum() <= 2 for v in c)


def test_direction_convention_of_the_paper():
    c, w, opp = oracle.tables()
    for q in range(1, 10):
        np.testing.assert_array_equal(c[q + 9], -c[q])
        assert opp[q] == q + 9 and opp[q + 9] == q
        # a preceding neighbour in an x-slowest, z-fastest sweep (Sec. 3, Fig. 1a)
        assert (c[q][0] * 10000 + c[q][1] * 100 + c[q][2]) < 0
    assert tuple(c[9]) == (0, -1, 1)  # lower-right Y-Z neighbour (Sec. 4.1)
    assert tuple(c[0]) == (0, 0, 0) and opp[0] == 0


def test_equilibrium_moments_closed_form():
    o = Oracle((2, 2, 2), 0.8)
    rng = np.random.default_rng(7)
    c, _, _ = oracle.tables()
    for _ in range(5):
        rho = 1.0 + rng.uniform(-0.1, 0.1)
        u = rng.uniform(-0.1, 0.1, 3)
        feq = np.empty(19)
        oracle.lib().orc_equilibrium(rho, oracle._p(u), oracle._p(feq))
        assert abs(feq.sum() - rho) < 1e-15
        np.testing.assert_allclose(c.T @ feq, rho * u, atol=1e-16)
        np.testing.assert_allclose(np.einsum("qa,qb,q->ab", c, c, feq), rho * (np.outer(u, u) + np.eye(3) / 3),
                                   atol=2e-16)
    assert o.N == 8


# --------------------------------------------------------------------------
# the per-cell velocity norm |u|, the quantity Sec. 5.1 compares across
# algorithms: pinned by states whose norm is known without evaluating it
# --------------------------------------------------------------------------

# velocities with integer-ratio norms (Pythagorean quadruples a^2+b^2+c^2=d^2)
PYTHAGOREAN = [((0.02, 0.03, 0.06), 0.07), ((-0.01, 0.04, -0.08), 0.09), ((0.12, -0.03, 0.04), 0.13),
               ((0.0, -0.06, 0.08), 0.10)]


@pytest.mark.parametrize("u0,norm", PYTHAGOREAN)
def test_velocity_norm_of_uniform_states(u0, norm):
    # a uniform equilibrium (rho0, u0) has velocity u0 and norm |u0| in every cell
    shape = (3, 4, 5)
    o = Oracle(shape, 0.8)
    rho = np.full(shape, 1.07)
    u = np.broadcast_to(np.asarray(u0)[:, None, None, None], (3,) + shape).copy()
    rho_m, u_m, un = o.macro(o.init(rho, u))
    assert np.abs(un - norm).max() <= 1e-15
    for a in range(3):
        assert np.abs(u_m[a] - u0[a]).max() <= 1e-16
    assert np.abs(rho_m - 1.07).max() <= 2e-15


def test_velocity_norm_includes_half_the_force():
    # u = (j + F/2)/rho: an equilibrium of u0 = (0.01, 0.05, 0.03) at rho = 1.25
    # under F = (0.025, 0.025, 0) has u = (0.02, 0.06, 0.03), |u| = 0.07
    shape = (2, 3, 4)
    o = Oracle(shape, 0.8)
    u = np.zeros((3,) + shape)
    u[0], u[1], u[2] = 0.01, 0.05, 0.03
    F = np.zeros((3,) + shape)
    F[0], F[1] = 0.025, 0.025
    _, u_m, un = o.macro(o.init(np.full(shape, 1.25), u), F)
    assert np.abs(un - 0.07).max() <= 1e-15
    np.testing.assert_allclose(u_m[:, 0, 0, 0], (0.02, 0.06, 0.03), atol=1e-16)


def test_velocity_norm_of_taylor_green_2d_is_its_amplitude_field():
    # at t = 0 the 2D vortex u = u0 (sin A cos B, -cos A sin B) has the norm
    # u0 sqrt(sin^2 A cos^2 B + cos^2 A sin^2 B): u0 at (A, B) = (pi/2, 0),
    # zero at (0, 0), and u0 |sin 2A| / sqrt(2) on the diagonal A = B
    shape = (16, 16, 3)
    u0 = 0.04
    o = Oracle(shape, 0.8)
    rho, u = wl.taylor_green_2d(shape, u0, axes=(0, 1))
    _, _, un = o.macro(o.init(rho, u))
    A = 2 * math.pi * np.arange(16) / 16
    amp = u0 * np.sqrt(np.sin(A)[:, None] ** 2 * np.cos(A)[None, :] ** 2 +
                       np.cos(A)[:, None] ** 2 * np.sin(A)[None, :] ** 2)
    assert np.abs(un - amp[:, :, None]).max() <= 1e-15
    assert abs(un[4, 0, 1] - u0) <= 1e-16 and un[0, 0, 2] <= 1e-16
    diag = np.array([un[i, i, 0] for i in range(16)])
    assert np.abs(diag - u0 * np.abs(np.sin(2 * A)) / math.sqrt(2)).max() <= 1e-15


# --------------------------------------------------------------------------
# exact invariants and fixed points
# --------------------------------------------------------------------------

def test_uniform_equilibrium_is_a_fixed_point():
    shape = (5, 4, 6)
    o = Oracle(shape, 0.7)
    rho = np.full(shape, 1.03)
    u = np.zeros((3,) + shape)
    u[0], u[1], u[2] = 0.01, -0.02, 0.005
    f0 = o.init(rho, u)
    f = o.run(f0, 20)
    assert np.abs(f - f0).max() <= 1e-14
    # fluid at rest between static walls on every face
    ow = Oracle(shape, 0.9, faces=(WALL,) * 6)
    g0 = ow.init(np.full(shape, 0.98), None)
    assert np.abs(ow.run(g0, 20) - g0).max() <= 1e-14


def _tgv_noise(shape, seed=11):
    rho, u = wl.taylor_green_3d(shape, 0.03)
    u += wl.uniform_noise(shape, 5e-3, seed)
    return wl.random_density(shape, 0.01, seed + 1), u


@pytest.mark.parametrize("faces,wall_u", [
    ((PERIODIC,) * 6, (0, 0, 0)),
    ((WALL,) * 6, (0, 0, 0)),
    ((WALL, WALL, WALL, MOVING_WALL, WALL, WALL), (0.05, 0.0, 0.0)),
    ((PERIODIC, PERIODIC, WALL, WALL, MOVING_WALL, WALL), (0.03, -0.02, 0.0)),
])
def test_mass_is_conserved(faces, wall_u):
    shape = (7, 6, 5)
    o = Oracle(shape, 0.62, faces=faces, wall_u=wall_u)
    f0 = o.init(*_tgv_noise(shape))
    m0 = o.sums(f0)[0]
    f = o.run(f0, 100)
    assert abs(o.sums(f)[0] - m0) <= 1e-13 * m0


def test_momentum_is_conserved_periodic():
    shape = (7, 6, 5)
    o = Oracle(shape, 0.55)
    f0 = o.init(*_tgv_noise(shape))
    p0 = o.sums(f0)[1:]
    m0 = o.sums(f0)[0]
    f = o.run(f0, 100)
    assert np.abs(o.sums(f)[1:] - p0).max() <= 1e-13 * m0 * 0.03


def test_guo_force_adds_exactly_its_total_momentum():
    # sum_q c_q f*_q = j + F per cell, so P(t) = P(0) + t * sum_x F exactly
    shape = (6, 5, 4)
    o = Oracle(shape, 0.8)
    F = wl.normal_field(shape, 1e-4, 5)
    f0 = o.init(*_tgv_noise(shape))
    p0 = o.sums(f0)[1:]
    t = 50
    f = o.run(f0, t, F)
    expect = p0 + t * F.reshape(3, -1).sum(axis=1)
    assert np.abs(o.sums(f)[1:] - expect).max() <= 1e-13 * np.abs(expect).max() + 1e-15


# --------------------------------------------------------------------------
# viscosity: decay rates and channel flows
# --------------------------------------------------------------------------

def _fit_rate(amps, steps):
    t = np.asarray(steps, np.float64)
    return -np.polyfit(t, np.log(np.asarray(amps)), 1)[0]


def test_shear_wave_decays_at_nu_k2():
    tau = 0.8
    nu = (tau - 0.5) / 3
    for flow, grad, shape in ((0, 1, (2, 32, 2)), (2, 0, (32, 2, 2)), (1, 2, (2, 2, 32))):
        o = Oracle(shape, tau)
        rho, u = wl.shear_wave(shape, 1e-4, flow, grad)
        f = o.init(rho, u)
        k = 2 * math.pi / shape[grad]
        mode = u[flow] / 1e-4
        amps, steps = [], []
        for s in range(0, 101, 10):
            if s:
                f = o.run(f, 10)
            if s >= 10:
                _, uu, _ = o.macro(f)
                amps.append((uu[flow] * mode).sum() / (mode * mode).sum())
                steps.append(s)
        rate = _fit_rate(amps, steps)
        assert abs(rate / (nu * k * k) - 1) < 5e-3


@pytest.mark.parametrize("axes,shape", [((0, 1), (32, 32, 2)), ((1, 2), (2, 32, 32)), ((0, 2), (32, 2, 32))])
def test_taylor_green_2d_decays_at_2_nu_k2(axes, shape):
    tau = 0.8
    nu = (tau - 0.5) / 3
    k = 2 * math.pi / 32
    o = Oracle(shape, tau)
    rho, u = wl.taylor_green_2d(shape, 0.02, axes)
    mode = u / 0.02
    f = o.init(rho, u)
    amps, steps = [], []
    for s in range(0, 101, 10):
        if s:
            f = o.run(f, 10)
        if s >= 10:
            _, uu, _ = o.macro(f)
            amps.append((uu * mode).sum() / (mode * mode).sum())
            steps.append(s)
    rate = _fit_rate(amps, steps)
    assert abs(rate / (2 * nu * k * k) - 1) < 5e-3


def _poiseuille(tau, g, H, steps):
    shape = (2, H, 2)
    o = Oracle(shape, tau, faces=(PERIODIC, PERIODIC, WALL, WALL, PERIODIC, PERIODIC))
    F = np.zeros((3,) + shape)
    F[0] = g
    f = o.run(o.init(), steps, F)
    _, u, _ = o.macro(f, F)
    return u[0, 0, :, 0], o


@pytest.mark.parametrize("tau,steps", [(0.6, 12000), (0.8, 6000), (0.5 + math.sqrt(3.0 / 16.0), 6000)])
def test_poiseuille_curvature_is_exact(tau, steps):
    g, H = 1e-5, 8
    nu = (tau - 0.5) / 3
    prof, _ = _poiseuille(tau, g, H, steps)
    y = np.arange(H, dtype=np.float64)
    a2 = np.polyfit(y, prof, 2)[0]
    assert abs(a2 / (-g / (2 * nu)) - 1) < 1e-9


def test_poiseuille_profile_exact_at_magic_tau():
    # halfway bounce-back puts the wall exactly midway for (tau-1/2)^2 = 3/16
    g, H = 1e-5, 8
    tau = 0.5 + math.sqrt(3.0 / 16.0)
    nu = (tau - 0.5) / 3
    prof, _ = _poiseuille(tau, g, H, 6000)
    y = np.arange(H, dtype=np.float64)
    exact = g / (2 * nu) * (y + 0.5) * (H - 0.5 - y)
    assert np.abs(prof - exact).max() <= 1e-9 * exact.max()


@pytest.mark.parametrize("tau", [0.6, 0.9])
def test_couette_profile_under_moving_wall(tau):
    H, U = 8, 1e-3
    shape = (2, H, 2)
    o = Oracle(shape, tau, faces=(PERIODIC, PERIODIC, WALL, MOVING_WALL, PERIODIC, PERIODIC), wall_u=(U, 0.0, 0.0))
    f = o.run(o.init(), 12000)
    _, u, _ = o.macro(f)
    y = np.arange(H, dtype=np.float64)
    np.testing.assert_allclose(u[0, 0, :, 0], U * (y + 0.5) / H, rtol=0, atol=1e-10 * U)
    assert np.abs(u[1:]).max() < 1e-9 * U


# --------------------------------------------------------------------------
# symmetry
# --------------------------------------------------------------------------

def test_axis_permutation_symmetry():
    shape = (6, 5, 4)
    perm = (1, 2, 0)  # new axis i is old axis perm[i]
    faces = (WALL, MOVING_WALL, PERIODIC, PERIODIC, WALL, WALL)
    wall_u = (0.0, 0.02, -0.01)
    rho, u = _tgv_noise(shape, 3)
    F = wl.normal_field(shape, 1e-4, 9)
    o = Oracle(shape, 0.7, faces=faces, wall_u=wall_u)
    f = o.run(o.init(rho, u), 12, F)
    r1, u1, _ = o.macro(f, F)

    pshape = tuple(shape[p] for p in perm)
    pfaces = sum(((faces[2 * p], faces[2 * p + 1]) for p in perm), ())
    pwall = tuple(wall_u[p] for p in perm)
    prho = np.ascontiguousarray(np.transpose(rho, perm))
    pu = np.ascontiguousarray(np.stack([np.transpose(u[p], perm) for p in perm]))
    pF = np.ascontiguousarray(np.stack([np.transpose(F[p], perm) for p in perm]))
    op = Oracle(pshape, 0.7, faces=pfaces, wall_u=pwall)
    g = op.run(op.init(prho, pu), 12, pF)
    r2, u2, _ = op.macro(g, pF)
    np.testing.assert_allclose(r2, np.transpose(r1, perm), rtol=0, atol=1e-14)
    for i, p in enumerate(perm):
        np.testing.assert_allclose(u2[i], np.transpose(u1[p], perm), rtol=0, atol=1e-15)


# --------------------------------------------------------------------------
# the paper's in-place procedures, brute force
# --------------------------------------------------------------------------

class SwapLattice:
    """The in-place single-copy update of Sec. 3 written from its description:
    per cell, collide, revert (slot q takes the post-collision value of the
    opposite direction) and swap slot q+9 with slot q of the neighbour x+c_q
    for the nine directions that point to already visited cells.  A slot
    whose swap partner is outside a wall keeps its reverted value, i.e. the
    population bounces back; a moving face adds its momentum term there."""

    def __init__(self, o: Oracle, faces, wall_u):
        self.o = o
        self.c, self.w, self.opp = oracle.tables()
        self.shape = o.shape
        self.faces = faces
        self.wall_u = np.asarray(wall_u, np.float64)

    def inside(self, p):
        return all(0 <= p[a] < self.shape[a] for a in range(3))

    def crossed_moving(self, p):
        for a in range(3):
            if p[a] < 0 and self.faces[2 * a] == MOVING_WALL:
                return True
            if p[a] >= self.shape[a] and self.faces[2 * a + 1] == MOVING_WALL:
                return True
        return False

    def collide_revert(self, f, x):
        post = self.o.collide_cell(f[(slice(None),) + x])
        for q in range(19):
            val = post[self.opp[q]]
            src = tuple(x[a] - self.c[q][a] for a in range(3))
            if not self.inside(src) and self.crossed_moving(src):
                val += 6.0 * self.w[q] * float(self.c[q] @ self.wall_u)
            f[(q,) + x] = val

    def swap_stream(self, f, x):
        for q in range(1, 10):
            n = tuple(x[a] + self.c[q][a] for a in range(3))
            if self.inside(n):
                a, b = (q + 9,) + x, (q,) + n
                f[a], f[b] = f[b], f[a]

    def cells(self):
        return list(itertools.product(*[range(n) for n in self.shape]))

    def fuse_swap_step(self, f):
        for x in self.cells():
            self.collide_revert(f, x)
            self.swap_stream(f, x)

    def two_step(self, f):
        """Two merged steps in one sweep: the second computation of a cell runs
        as soon as every neighbour that swaps with it later in the first sweep
        (x - c_q, q = 1..9) has done its first computation; second
        computations keep the sweep order."""
        cells = self.cells()
        index = {x: i for i, x in enumerate(cells)}
        ready = []
        for x in cells:
            r = index[x]
            for q in range(1, 10):
                m = tuple(x[a] - self.c[q][a] for a in range(3))
                if self.inside(m):
                    r = max(r, index[m])
            ready.append(r)
        j = 0
        for i, x in enumerate(cells):
            self.collide_revert(f, x)
            self.swap_stream(f, x)
            while j < len(cells) and ready[j] <= i:
                self.collide_revert(f, cells[j])
                self.swap_stream(f, cells[j])
                j += 1
        while j < len(cells):
            self.collide_revert(f, cells[j])
            self.swap_stream(f, cells[j])
            j += 1


@pytest.mark.parametrize("shape", [(4, 4, 4), (5, 6, 7), (8, 4, 4)])
@pytest.mark.parametrize("lid", [False, True])
def test_swap_algorithm_equals_two_array_oracle(shape, lid):
    faces = (WALL, MOVING_WALL, WALL, WALL, WALL, WALL) if lid else (WALL,) * 6
    wall_u = (0.0, 0.04, -0.03) if lid else (0.0, 0.0, 0.0)
    o = Oracle(shape, 0.65, faces=faces, wall_u=wall_u)
    f0 = o.init(*_tgv_noise(shape, 21))
    s = SwapLattice(o, faces, wall_u)
    f1 = f0.copy()
    s.fuse_swap_step(f1)
    s.fuse_swap_step(f1)
    ref = o.run(f0, 2)
    assert np.abs(f1 - ref).max() <= 1e-15
    f2 = f0.copy()
    s.two_step(f2)
    assert np.abs(f2 - ref).max() <= 1e-15


# --------------------------------------------------------------------------
# discrete adjoint
# --------------------------------------------------------------------------

def test_stream_transpose_dot_product():
    shape = (5, 4, 6)
    o = Oracle(shape, 0.7, faces=(PERIODIC, PERIODIC, WALL, WALL, WALL, WALL))
    rng = np.random.default_rng(3)
    v = rng.normal(size=(19,) + shape)
    w = rng.normal(size=(19,) + shape)
    lhs = (o.stream(v) * w).sum()
    rhs = (v * o.stream_adjoint(w)).sum()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_collide_adjoint_cell_matches_central_differences():
    o = Oracle((2, 2, 2), 0.77)
    rng = np.random.default_rng(4)
    feq = np.empty(19)
    oracle.lib().orc_equilibrium(1.02, oracle._p(np.array([0.03, -0.02, 0.01])), oracle._p(feq))
    f = feq + rng.normal(scale=1e-3, size=19)
    F = rng.normal(scale=1e-3, size=3)
    mu = rng.normal(size=19)
    lam, gF = o.collide_adjoint_cell(f, mu, F)
    h = 1e-6
    for j in range(19):
        e = np.zeros(19)
        e[j] = h
        fd = (mu @ o.collide_cell(f + e, F) - mu @ o.collide_cell(f - e, F)) / (2 * h)
        assert abs(fd - lam[j]) <= 1e-8 * max(1.0, abs(lam).max())
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd = (mu @ o.collide_cell(f, F + e) - mu @ o.collide_cell(f, F - e)) / (2 * h)
        assert abs(fd - gF[a]) <= 1e-8 * max(1.0, abs(gF).max())


def test_loss_seed_matches_central_differences():
    shape = (3, 3, 2)
    o = Oracle(shape, 0.8)
    f = o.init(*_tgv_noise(shape, 5))
    F = wl.normal_field(shape, 1e-3, 6)
    ut = wl.normal_field(shape, 1e-2, 7)
    lam, gF = o.loss_seed(f, ut, F)
    h = 1e-6
    rng = np.random.default_rng(8)
    for _ in range(10):
        q, x, y, z = rng.integers(19), rng.integers(3), rng.integers(3), rng.integers(2)
        fp, fm = f.copy(), f.copy()
        fp[q, x, y, z] += h
        fm[q, x, y, z] -= h
        fd = (o.loss(fp, ut, F) - o.loss(fm, ut, F)) / (2 * h)
        assert abs(fd - lam[q, x, y, z]) <= 1e-7 * np.abs(lam).max()
    for a in range(3):
        Fp, Fm = F.copy(), F.copy()
        Fp[a, 1, 2, 1] += h
        Fm[a, 1, 2, 1] -= h
        fd = (o.loss(f, ut, Fp) - o.loss(f, ut, Fm)) / (2 * h)
        assert abs(fd - gF[a, 1, 2, 1]) <= 1e-7 * np.abs(gF).max()


def test_adjoint_gradient_matches_central_differences():
    # a small channel like the adjoint workload: periodic x, walls in y and z
    shape = (6, 5, 5)
    faces = (PERIODIC, PERIODIC, WALL, WALL, WALL, WALL)
    o = Oracle(shape, 0.8, faces=faces)
    T = 8
    f0 = o.init(*_tgv_noise(shape, 31))
    F = wl.normal_field(shape, 1e-4, 1)
    hidden = wl.normal_field(shape, 1e-4, 2)
    _, ut, _ = o.macro(o.run(f0, T, hidden), hidden)
    L, gF = o.loss_and_grad(f0, F, ut, T)
    assert L > 0
    # the loss is not exactly quadratic in F: central differences carry an
    # eps^2 truncation term (measured 3e-9 relative at eps=1e-4, 3e-11 at 1e-5)
    eps = 1e-5
    for (x, y, z) in wl.sample_cells(shape, 6, 3):
        for a in range(3):
            Fp, Fm = F.copy(), F.copy()
            Fp[a, x, y, z] += eps
            Fm[a, x, y, z] -= eps
            Lp = o.loss(o.run(f0, T, Fp), ut, Fp)
            Lm = o.loss(o.run(f0, T, Fm), ut, Fm)
            fd = (Lp - Lm) / (2 * eps)
            assert abs(fd - gF[a, x, y, z]) <= 1e-6 * np.abs(gF).max()


# --------------------------------------------------------------------------
# regression fixture (written by tests/golden/make_golden.py from the oracle)
# --------------------------------------------------------------------------

def test_oracle_matches_committed_cavity_fixture():
    from tests.golden.make_golden import cavity_case, load_fixture
    rho, unorm = cavity_case()
    ref = load_fixture(os.path.join(GOLDEN, "cavity_5x6x7_lid.txt"))
    np.testing.assert_allclose(rho.ravel(), ref[:, 0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(unorm.ravel(), ref[:, 1], rtol=0, atol=1e-16)
