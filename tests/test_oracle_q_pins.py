"""Pins of the generic-lattice oracle (oracle/lbm_oracle_q.c: D3Q15, D3Q19,
D3Q27) against facts fixed by the mathematics of the lattice Boltzmann
method, before any GPU kernel for those velocity sets is trusted.  Sec. 4.1
of the paper states that its two-step rule holds for D3Q15, D3Q19 and D3Q27.

* Tables: weights and velocities satisfy the isotropy identities up to fourth
  order (closed forms; what makes each set reproduce Navier-Stokes with
  cs^2 = 1/3), the sets have the stated sizes and speeds, directions 1..H
  precede a cell in the sweep (Sec. 3) and c_{q+H} = -c_q.
* D3Q19: the generic code agrees with the separate D3Q19 oracle (an
  independent implementation) on a walled, lid-driven, forced lattice.
* Per set: uniform equilibrium is a fixed point; mass is conserved with
  walls and a tangential lid; momentum is conserved on a periodic lattice;
  the Guo force adds exactly its total momentum; a shear wave decays at
  nu k^2 with nu = (tau - 1/2)/3 along every axis; Poiseuille flow has the
  exact curvature -g/(2 nu), and the exact halfway profile at
  tau = 1/2 + sqrt(3/16); Couette flow under a moving wall is linear.
* Discrete adjoint, per set: the seed is the gradient of the loss and one
  reverse step the gradient of <lambda, step(f, F)> in f and in F (central
  differences of the forward oracle, on walls, a lid and periodic faces), and
  several steps end to end match differences of the whole run; the D3Q19
  case equals the separate D3Q19 oracle's adjoint.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import MOVING_WALL, PERIODIC, WALL, Oracle, OracleQ
from paper_2208_05429_amd import workloads as wl

SETS = [15, 19, 27]
SIZES = {15: (7, {0: 1, 1: 6, 3: 8}), 19: (9, {0: 1, 1: 6, 2: 12}), 27: (13, {0: 1, 1: 6, 2: 12, 3: 8})}


@pytest.mark.parametrize("q", SETS)
def test_isotropy_identities(q):
    c, w, opp = oracle.tables_q(q)
    assert len(c) == q and len({tuple(v) for v in c}) == q
    c = c.astype(np.float64)
    d = np.eye(3)
    assert abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(np.einsum("q,qa->a", w, c), 0.0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("q,qa,qb->ab", w, c, c), d / 3.0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("q,qa,qb,qc->abc", w, c, c, c), 0.0, atol=1e-16)
    four = np.einsum("q,qa,qb,qc,qd->abcd", w, c, c, c, c)
    expect = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9.0
    np.testing.assert_allclose(four, expect, atol=1e-16)
    # the speeds of the set: counts by |c|^2
    speeds = {}
    for v in c.astype(int):
        s = int((v ** 2).sum())
        speeds[s] = speeds.get(s, 0) + 1
    assert speeds == SIZES[q][1]


@pytest.mark.parametrize("q", SETS)
def test_direction_convention(q):
    c, w, opp = oracle.tables_q(q)
    H = SIZES[q][0]
    assert tuple(c[0]) == (0, 0, 0) and opp[0] == 0 and tuple(c[1]) == (-1, 0, 0)
    for k in range(1, H + 1):
        np.testing.assert_array_equal(c[k + H], -c[k])
        assert opp[k] == k + H and opp[k + H] == k
        assert (c[k][0] * 10000 + c[k][1] * 100 + c[k][2]) < 0  # precedes in the x-slowest sweep
    c19, _, _ = oracle.tables()
    np.testing.assert_array_equal(oracle.tables_q(19)[0], c19)  # the same numbering as the D3Q19 oracle
    if q == 27:
        np.testing.assert_array_equal(c[1:10], c19[1:10])


def _state(shape, seed):
    _, u = wl.taylor_green_3d(shape, 0.03)
    u = u + wl.uniform_noise(shape, 5e-3, seed)
    return wl.random_density(shape, 0.01, seed + 1), u


def test_d3q19_agrees_with_the_d3q19_oracle():
    shape = (6, 7, 5)
    faces = (WALL, WALL, WALL, MOVING_WALL, PERIODIC, PERIODIC)
    rho, u = _state(shape, 3)
    F = wl.normal_field(shape, 1e-4, 4)
    a = Oracle(shape, 0.7, faces=faces, wall_u=(0.04, 0.0, 0.01))
    b = OracleQ(shape, 0.7, 19, faces=faces, wall_u=(0.04, 0.0, 0.01))
    fa = a.run(a.init(rho, u), 12, F)
    fb = b.run(b.init(rho, u), 12, F)
    assert np.abs(fa - fb).max() <= 1e-15 * np.abs(fa).max() * 10


@pytest.mark.parametrize("q", SETS)
def test_uniform_equilibrium_is_a_fixed_point(q):
    shape = (5, 4, 6)
    o = OracleQ(shape, 0.7, q)
    u = np.zeros((3,) + shape)
    u[0], u[1], u[2] = 0.01, -0.02, 0.005
    f0 = o.init(np.full(shape, 1.03), u)
    assert np.abs(o.run(f0, 20) - f0).max() <= 1e-14
    ow = OracleQ(shape, 0.9, q, faces=(WALL,) * 6)
    g0 = ow.init(np.full(shape, 0.98), None)
    assert np.abs(ow.run(g0, 20) - g0).max() <= 1e-14


@pytest.mark.parametrize("q", SETS)
@pytest.mark.parametrize("faces,wall_u", [
    ((WALL, WALL, WALL, MOVING_WALL, WALL, WALL), (0.05, 0.0, 0.0)),
    ((PERIODIC, PERIODIC, WALL, WALL, MOVING_WALL, WALL), (0.03, -0.02, 0.0)),
])
def test_mass_is_conserved(q, faces, wall_u):
    shape = (7, 6, 5)
    o = OracleQ(shape, 0.62, q, faces=faces, wall_u=wall_u)
    f0 = o.init(*_state(shape, 11))
    m0 = o.sums(f0)[0]
    assert abs(o.sums(o.run(f0, 100))[0] - m0) <= 1e-13 * m0


@pytest.mark.parametrize("q", SETS)
def test_momentum_is_conserved_and_the_force_adds_its_total(q):
    shape = (7, 6, 5)
    o = OracleQ(shape, 0.55, q)
    f0 = o.init(*_state(shape, 12))
    s0 = o.sums(f0)
    assert np.abs(o.sums(o.run(f0, 100))[1:] - s0[1:]).max() <= 1e-13 * s0[0] * 0.03
    F = wl.normal_field(shape, 1e-4, 13)
    expect = s0[1:] + 50 * F.reshape(3, -1).sum(axis=1)
    assert np.abs(o.sums(o.run(f0, 50, F))[1:] - expect).max() <= 1e-13 * np.abs(expect).max() + 1e-15


@pytest.mark.parametrize("q", SETS)
def test_shear_wave_decays_at_nu_k2(q):
    tau = 0.8
    nu = (tau - 0.5) / 3
    for flow, grad, shape in ((0, 1, (2, 32, 2)), (2, 0, (32, 2, 2)), (1, 2, (2, 2, 32))):
        o = OracleQ(shape, tau, q)
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
        rate = -np.polyfit(np.asarray(steps, float), np.log(np.asarray(amps)), 1)[0]
        assert abs(rate / (nu * k * k) - 1) < 5e-3, (q, flow, grad, rate / (nu * k * k))


@pytest.mark.parametrize("q", SETS)
@pytest.mark.parametrize("tau,steps", [(0.6, 12000), (0.5 + math.sqrt(3.0 / 16.0), 6000)])
def test_poiseuille_curvature_is_exact(q, tau, steps):
    g, H = 1e-5, 8
    nu = (tau - 0.5) / 3
    shape = (2, H, 2)
    o = OracleQ(shape, tau, q, faces=(PERIODIC, PERIODIC, WALL, WALL, PERIODIC, PERIODIC))
    F = np.zeros((3,) + shape)
    F[0] = g
    _, u, _ = o.macro(o.run(o.init(), steps, F), F)
    prof = u[0, 0, :, 0]
    a2 = np.polyfit(np.arange(H, dtype=np.float64), prof, 2)[0]
    assert abs(a2 / (-g / (2 * nu)) - 1) < 1e-9


@pytest.mark.parametrize("q", SETS)
def test_couette_profile_under_moving_wall(q):
    H, U, tau = 8, 1e-3, 0.7
    shape = (2, H, 2)
    o = OracleQ(shape, tau, q, faces=(PERIODIC, PERIODIC, WALL, MOVING_WALL, PERIODIC, PERIODIC), wall_u=(U, 0, 0))
    _, u, _ = o.macro(o.run(o.init(), 12000))
    y = np.arange(H, dtype=np.float64)
    np.testing.assert_allclose(u[0, 0, :, 0], U * (y + 0.5) / H, rtol=0, atol=1e-10 * U)
    assert np.abs(u[1:]).max() < 1e-9 * U


@pytest.mark.parametrize("q", SETS)
def test_poiseuille_profile_exact_at_magic_tau(q):
    # halfway bounce-back puts the walls exactly midway for (tau - 1/2)^2 = 3/16
    g, H = 1e-5, 8
    tau = 0.5 + math.sqrt(3.0 / 16.0)
    nu = (tau - 0.5) / 3
    shape = (2, H, 2)
    o = OracleQ(shape, tau, q, faces=(PERIODIC, PERIODIC, WALL, WALL, PERIODIC, PERIODIC))
    F = np.zeros((3,) + shape)
    F[0] = g
    _, u, _ = o.macro(o.run(o.init(), 6000, F), F)
    y = np.arange(H, dtype=np.float64)
    exact = g / (2 * nu) * (y + 0.5) * (H - 0.5 - y)
    assert np.abs(u[0, 0, :, 0] - exact).max() <= 1e-9 * exact.max()


# ---------------------------------------------------------------------------
# discrete adjoint, pinned by central differences of the forward oracle

ADJ_FACES = (WALL, MOVING_WALL, PERIODIC, PERIODIC, WALL, WALL)
ADJ_WALL_U = (0.0, 0.02, 0.01)


def _adj_problem(q, shape=(5, 6, 7), seed=900):
    rho0, u0 = wl.taylor_green_3d(shape, 0.03)
    u0 = u0 + wl.uniform_noise(shape, 5e-3, seed)
    o = OracleQ(shape, 0.7, q, faces=ADJ_FACES, wall_u=ADJ_WALL_U)
    f = o.init(wl.random_density(shape, 0.01, seed + 1), u0)
    F = wl.normal_field(shape, 1e-3, seed + 2)
    return o, f, F


def _entries(rng, shape, n):
    # random entries, and the cells next to each wall face and the lid
    idx = [tuple(int(rng.integers(0, s)) for s in shape) for _ in range(n)]
    idx += [(0, 2, 0), (shape[0] - 1, 3, shape[2] - 1), (2, 0, 3), (1, shape[1] - 1, 0)]
    return idx


@pytest.mark.parametrize("q", SETS)
def test_adjoint_seed_is_the_gradient_of_the_loss(q):
    o, f, F = _adj_problem(q)
    ut = wl.normal_field(o.shape, 1e-2, 910)
    lam, gF = o.loss_seed(f, ut, F)
    rng = np.random.default_rng(911)
    eps = 1e-6
    for x, y, z in _entries(rng, o.shape, 8):
        p = int(rng.integers(0, q))
        fp, fm = f.copy(), f.copy()
        fp[p, x, y, z] += eps
        fm[p, x, y, z] -= eps
        fd = (o.loss(fp, ut, F) - o.loss(fm, ut, F)) / (2 * eps)
        assert abs(fd - lam[p, x, y, z]) <= 1e-7 * max(1.0, abs(fd)), (p, x, y, z, fd, lam[p, x, y, z])
        a = int(rng.integers(0, 3))
        Fp, Fm = F.copy(), F.copy()
        Fp[a, x, y, z] += eps
        Fm[a, x, y, z] -= eps
        fd = (o.loss(f, ut, Fp) - o.loss(f, ut, Fm)) / (2 * eps)
        assert abs(fd - gF[a, x, y, z]) <= 1e-7 * max(1.0, abs(fd)), (a, x, y, z, fd, gF[a, x, y, z])


@pytest.mark.parametrize("q", SETS)
def test_adjoint_step_is_the_gradient_of_one_step(q):
    o, f, F = _adj_problem(q)
    lam_next = wl.normal_field(o.shape, 1.0, 920, comps=q)
    lam, gF = o.adjoint_step(f, lam_next, F)

    def phi(ff, FF):
        return float(np.sum(lam_next * o.run(ff, 1, FF)))

    rng = np.random.default_rng(921)
    eps = 1e-6
    for x, y, z in _entries(rng, o.shape, 10):
        p = int(rng.integers(0, q))
        fp, fm = f.copy(), f.copy()
        fp[p, x, y, z] += eps
        fm[p, x, y, z] -= eps
        fd = (phi(fp, F) - phi(fm, F)) / (2 * eps)
        assert abs(fd - lam[p, x, y, z]) <= 1e-7 * max(1.0, abs(fd)), (p, x, y, z, fd, lam[p, x, y, z])
        a = int(rng.integers(0, 3))
        Fp, Fm = F.copy(), F.copy()
        Fp[a, x, y, z] += eps
        Fm[a, x, y, z] -= eps
        fd = (phi(f, Fp) - phi(f, Fm)) / (2 * eps)
        assert abs(fd - gF[a, x, y, z]) <= 1e-7 * max(1.0, abs(fd)), (a, x, y, z, fd, gF[a, x, y, z])


@pytest.mark.parametrize("q", [15, 27])
def test_adjoint_over_several_steps_matches_differences_of_the_run(q):
    o, f, F = _adj_problem(q, shape=(4, 5, 6), seed=930)
    ut = wl.normal_field(o.shape, 1e-2, 931)
    steps = 4
    L, g = o.loss_and_grad(f, F, ut, steps)
    rng = np.random.default_rng(932)
    eps = 1e-6
    for _ in range(8):
        a, x, y, z = (int(rng.integers(0, n)) for n in (3,) + o.shape)
        Fp, Fm = F.copy(), F.copy()
        Fp[a, x, y, z] += eps
        Fm[a, x, y, z] -= eps
        fd = (o.loss(o.run(f, steps, Fp), ut, Fp) - o.loss(o.run(f, steps, Fm), ut, Fm)) / (2 * eps)
        assert abs(fd - g[a, x, y, z]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (a, x, y, z, fd, g[a, x, y, z])


def test_d3q19_adjoint_equals_the_d3q19_oracle_adjoint():
    o, f, F = _adj_problem(19)
    ref = Oracle(o.shape, 0.7, faces=ADJ_FACES, wall_u=ADJ_WALL_U)
    lam_next = wl.normal_field(o.shape, 1.0, 940, comps=19)
    ut = wl.normal_field(o.shape, 1e-2, 941)
    a, ga = o.adjoint_step(f, lam_next, F)
    b, gb = ref.adjoint_step(f, lam_next, F)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-13 * np.abs(b).max())
    np.testing.assert_allclose(ga, gb, rtol=0, atol=1e-13 * np.abs(gb).max())
    a, ga = o.loss_seed(f, ut, F)
    b, gb = ref.loss_seed(f, ut, F)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-14 * np.abs(b).max())
    np.testing.assert_allclose(ga, gb, rtol=0, atol=1e-14 * np.abs(gb).max())
