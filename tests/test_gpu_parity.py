"""GPU parity of the HIP library (called through the C ABI) against the FP64
CPU oracle on the same seeded inputs.

Error metric (per field, as for the Taylor-Green workload): max |X_gpu - X_ref|
/ max |X_ref| with u taken as one vector field.  Bars: FP64 <= 1e-12, FP32
<= 2e-6 after 100 steps; 16-bit storage over many steps is reported against
loose bounds (its pin is the half-ulp bound of one store, test_gpu_precision.py).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import MOVING_WALL, PERIODIC, WALL, Oracle
from paper_2208_05429_amd import capi
from paper_2208_05429_amd import workloads as wl
from paper_2208_05429_amd.lattice import Lattice, real_dtype

pytestmark = pytest.mark.gpu

FACE_NAMES = {PERIODIC: "periodic", WALL: "wall", MOVING_WALL: "moving"}


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def gpu_run(shape, tau, storage, scheme, faces=(PERIODIC,) * 6, wall_u=(0, 0, 0), rho0=None, u0=None, F=None,
            steps=0, variant=0):
    print(f"[gpu] {storage} {scheme} shape={shape} steps={steps} faces={faces}", flush=True)
    force = None if F is None else torch.as_tensor(F, dtype=real_dtype(storage))
    lat = Lattice(shape, tau, storage, scheme, [FACE_NAMES[f] for f in faces], wall_u, force,
                  None if rho0 is None else torch.as_tensor(rho0), None if u0 is None else torch.as_tensor(u0),
                  variant=variant)
    lat.step(steps)
    rho, u, un, sums = lat.macroscopic(sums=True)
    torch.cuda.synchronize()
    lat.unorm = un.cpu().numpy()  # |u| per cell, the quantity Sec. 5.1 compares
    return lat, rho.cpu().numpy(), u.cpu().numpy(), sums


SCHEMES = ["two_array", "swap1", "swap2"]


# --------------------------------------------------------------------------
# the 32^3 Taylor-Green workload, 100 steps
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def tgv32_ref():
    cfg = wl.TGV_32
    rho0, u0 = wl.taylor_green_3d(cfg["shape"], cfg["u0"])
    o = Oracle(cfg["shape"], cfg["tau"])
    f = o.run(o.init(rho0, u0), cfg["steps"])
    rho, u, un = o.macro(f)
    return rho0, u0, rho, u, o.sums(f), un


@pytest.mark.parametrize("scheme", SCHEMES)
def test_tgv32_fp64_matches_oracle(tgv32_ref, scheme):
    cfg = wl.TGV_32
    rho0, u0, rho_ref, u_ref, sums_ref, un_ref = tgv32_ref
    lat, rho, u, sums = gpu_run(cfg["shape"], cfg["tau"], "f64", scheme, rho0=rho0, u0=u0, steps=cfg["steps"])
    assert rel(rho, rho_ref) <= 1e-12
    assert rel(u, u_ref) <= 1e-12
    assert rel(lat.unorm, un_ref) <= 1e-12
    assert abs(sums[0] - sums_ref[0]) <= 1e-12 * sums_ref[0]


@pytest.mark.parametrize("scheme", SCHEMES)
def test_tgv32_fp32_matches_oracle(tgv32_ref, scheme):
    cfg = wl.TGV_32
    rho0, u0, rho_ref, u_ref, _, un_ref = tgv32_ref
    lat, rho, u, _ = gpu_run(cfg["shape"], cfg["tau"], "f32", scheme, rho0=rho0, u0=u0, steps=cfg["steps"])
    eu, er, en = rel(u, u_ref), rel(rho, rho_ref), rel(lat.unorm, un_ref)
    print(f"fp32 {scheme}: rho err {er:.3e}  u err {eu:.3e}  |u| err {en:.3e}")
    assert er <= 2e-6 and eu <= 2e-6 and en <= 2e-6


def test_cavity_fp32_100_steps_matches_oracle():
    # the lid-driven cavity of the 256^3 workload at 40 x 48 x 56 (several
    # tiles, ragged last ones): tau 0.52, five static walls, +y lid moving at
    # 0.05 along x, rest state, 100 steps; every field within 2e-6 of the oracle
    shape = (40, 48, 56)
    faces = (WALL, WALL, WALL, MOVING_WALL, WALL, WALL)
    wall_u = (wl.CAVITY_256["lid_u"], 0.0, 0.0)
    tau = wl.CAVITY_256["tau"]
    o = Oracle(shape, tau, faces=faces, wall_u=wall_u)
    ref = o.run(o.init(), 100)
    rho_ref, u_ref, un_ref = o.macro(ref)
    sums_ref = o.sums(ref)
    for scheme in SCHEMES:
        lat, rho, u, sums = gpu_run(shape, tau, "f32", scheme, faces, wall_u, steps=100)
        ef, er, eu, en = rel(lat.distributions(), ref), rel(rho, rho_ref), rel(u, u_ref), rel(lat.unorm, un_ref)
        print(f"cavity fp32 {scheme}: f {ef:.3e} rho {er:.3e} u {eu:.3e} |u| {en:.3e}")
        assert max(ef, er, eu, en) <= 2e-6, scheme
        assert abs(sums[0] - sums_ref[0]) <= 1e-9 * sums_ref[0]


@pytest.mark.parametrize("storage,bound", [("f16", 2e-3), ("bf16", 2e-2)])
def test_tgv32_16bit_storage_error_is_bounded(tgv32_ref, storage, bound):
    # 100 steps of 16-bit rounding of f - w: a loose bound on the accumulated error
    cfg = wl.TGV_32
    rho0, u0, rho_ref, u_ref, _, _ = tgv32_ref
    for scheme in ("swap1", "swap2"):
        _, rho, u, _ = gpu_run(cfg["shape"], cfg["tau"], storage, scheme, rho0=rho0, u0=u0, steps=cfg["steps"])
        eu, er = rel(u, u_ref), rel(rho, rho_ref)
        print(f"{storage} {scheme}: rho err {er:.3e}  u err {eu:.3e}")
        assert er <= bound and eu <= 10 * bound


# --------------------------------------------------------------------------
# ragged lattices spanning several tiles, walls, moving lid, odd step counts
# --------------------------------------------------------------------------

CASES = [
    # shape, faces, wall_u  (odd nz runs the plain-slot kernels, even nz the pair-and-ring ones)
    ((20, 37, 45), (WALL, WALL, WALL, MOVING_WALL, WALL, WALL), (0.05, 0.0, -0.02)),
    ((23, 30, 61), (PERIODIC, PERIODIC, WALL, WALL, MOVING_WALL, WALL), (0.03, -0.02, 0.0)),
    ((17, 41, 33), (PERIODIC,) * 6, (0.0, 0.0, 0.0)),
    ((26, 13, 70), (MOVING_WALL, WALL, PERIODIC, PERIODIC, WALL, WALL), (0.0, 0.04, 0.01)),
    ((20, 37, 68), (WALL, WALL, WALL, MOVING_WALL, WALL, WALL), (0.05, 0.0, -0.02)),
    ((19, 35, 130), (PERIODIC,) * 6, (0.0, 0.0, 0.0)),
    ((21, 18, 66), (PERIODIC, PERIODIC, WALL, WALL, MOVING_WALL, WALL), (0.03, -0.02, 0.0)),
]
VARIANTS = [0, 1, 2, 3, 4]  # 32-bit storages: 16x64 pair-ring, 16x64 slots, 32x32 pair-ring, 32x32 slots,
# 16x64 pair-ring with loads two planes ahead


def _noisy_init(shape, seed):
    rho0, u0 = wl.taylor_green_3d(shape, 0.03)
    u0 = u0 + wl.uniform_noise(shape, 5e-3, seed)
    return wl.random_density(shape, 0.01, seed + 1), u0


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("steps", [1, 2, 9])
def test_ragged_fp64_full_state(case, steps):
    shape, faces, wall_u = CASES[case]
    rho0, u0 = _noisy_init(shape, 100 + case)
    o = Oracle(shape, 0.7, faces=faces, wall_u=wall_u)
    ref = o.run(o.init(rho0, u0), steps)
    rho_ref, u_ref, un_ref = o.macro(ref)
    for scheme in SCHEMES:
        lat, rho, u, _ = gpu_run(shape, 0.7, "f64", scheme, faces, wall_u, rho0, u0, steps=steps)
        f = lat.distributions()
        assert rel(f, ref) <= 1e-12, scheme
        assert rel(rho, rho_ref) <= 1e-12 and rel(u, u_ref) <= 1e-12 and rel(lat.unorm, un_ref) <= 1e-12, scheme


@pytest.mark.parametrize("case", range(len(CASES)))
def test_ragged_fp32_schemes_agree(case):
    shape, faces, wall_u = CASES[case]
    rho0, u0 = _noisy_init(shape, 200 + case)
    o = Oracle(shape, 0.6, faces=faces, wall_u=wall_u)
    steps = 7
    ref = o.run(o.init(rho0, u0), steps)
    _, u_ref, un_ref = o.macro(ref)
    lat, _, u, _ = gpu_run(shape, 0.6, "f32", "two_array", faces, wall_u, rho0, u0, steps=steps)
    a = lat.f.cpu().numpy()
    assert rel(lat.distributions(), ref) <= 2e-6
    assert rel(u, u_ref) <= 2e-6 and rel(lat.unorm, un_ref) <= 2e-6
    # every in-place kernel shape runs the same per-cell arithmetic as the plain
    # scheme: any difference is a race or an indexing slip
    for variant in VARIANTS:
        for scheme in ("swap1", "swap2"):
            lat, _, _, _ = gpu_run(shape, 0.6, "f32", scheme, faces, wall_u, rho0, u0, steps=steps, variant=variant)
            assert np.array_equal(lat.f.cpu().numpy().view(np.uint32), a.view(np.uint32)), (scheme, variant)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("case,force", [(0, False), (4, False), (5, False), (0, True), (4, True)])
def test_ragged_16bit_kernel_shapes_agree(storage, case, force):
    # 16-bit storage rounds every stored value, so shapes agree bitwise only if
    # each runs the same per-cell arithmetic on the same inputs
    shape, faces, wall_u = CASES[case]
    rho0, u0 = _noisy_init(shape, 250 + case)
    F = wl.normal_field(shape, 1e-4, 260 + case) if force else None
    for scheme in ("swap1", "swap2"):
        states = []
        for variant in VARIANTS:
            lat, _, _, _ = gpu_run(shape, 0.6, storage, scheme, faces, wall_u, rho0, u0, F=F, steps=5,
                                   variant=variant)
            states.append(lat.f.view(torch.int16).cpu().numpy().copy())
        for v, st in zip(VARIANTS[1:], states[1:]):
            assert np.array_equal(st, states[0]), (scheme, v)


def test_force_channel_fp64_and_fp32():
    shape = (24, 20, 18)
    faces = (PERIODIC, PERIODIC, WALL, WALL, WALL, WALL)
    rho0, u0 = _noisy_init(shape, 300)
    F = wl.normal_field(shape, 1e-4, 301)
    o = Oracle(shape, 0.8, faces=faces)
    ref = o.run(o.init(rho0, u0), 9, F)
    u_ref = o.macro(ref, F)[1]
    for scheme in SCHEMES:
        lat, rho, u, _ = gpu_run(shape, 0.8, "f64", scheme, faces, rho0=rho0, u0=u0, F=F, steps=9)
        assert rel(lat.distributions(), ref) <= 1e-12, scheme
        assert rel(u, u_ref) <= 1e-12
        lat, rho, u, _ = gpu_run(shape, 0.8, "f32", scheme, faces, rho0=rho0, u0=u0, F=F, steps=9)
        assert rel(lat.distributions(), ref) <= 2e-6, scheme


def test_force_periodic_pair_layout():
    # a body force on a periodic lattice with even nz: the pair-and-ring FP32
    # kernel (several tiles in y and z, a ragged last tile in each)
    shape = (14, 36, 70)
    faces = (PERIODIC,) * 6
    rho0, u0 = _noisy_init(shape, 310)
    F = wl.normal_field(shape, 1e-4, 311)
    o = Oracle(shape, 0.7, faces=faces)
    ref = o.run(o.init(rho0, u0), 9, F)
    for scheme in SCHEMES:
        lat, _, _, _ = gpu_run(shape, 0.7, "f32", scheme, faces, rho0=rho0, u0=u0, F=F, steps=9)
        assert rel(lat.distributions(), ref) <= 2e-6, scheme


@pytest.mark.parametrize("faces,wall_u", [
    ((PERIODIC, PERIODIC, WALL, WALL, WALL, WALL), (0.0, 0.0, 0.0)),
    ((PERIODIC, PERIODIC, WALL, MOVING_WALL, WALL, WALL), (0.04, 0.0, -0.01)),
])
def test_walls_and_force_pair_layout_match_two_array_bitwise(faces, wall_u):
    # walls in y and z with a body force on the pair-and-ring FP32 kernels
    # (16 x 64 and 32 x 32 tiles, one and two merged steps): three tile rows and
    # three tile columns with ragged last ones, against the two-array kernel;
    # the oracle fixes the two-array result
    shape = (10, 40, 150)
    rho0, u0 = _noisy_init(shape, 320)
    F = wl.normal_field(shape, 1e-4, 321)
    o = Oracle(shape, 0.8, faces=faces, wall_u=wall_u)
    ref = o.run(o.init(rho0, u0), 5, F)
    lat, _, _, _ = gpu_run(shape, 0.8, "f32", "two_array", faces, wall_u, rho0, u0, F=F, steps=5)
    assert rel(lat.distributions(), ref) <= 2e-6
    a = lat.f.cpu().numpy().view(np.uint32)
    for variant in (0, 2):
        for scheme in ("swap1", "swap2"):
            lat, _, _, _ = gpu_run(shape, 0.8, "f32", scheme, faces, wall_u, rho0, u0, F=F, steps=5, variant=variant)
            assert np.array_equal(lat.f.cpu().numpy().view(np.uint32), a), (scheme, variant)


def test_conservation_sums_match_oracle():
    shape = (20, 37, 45)
    faces, wall_u = CASES[0][1], CASES[0][2]
    rho0, u0 = _noisy_init(shape, 400)
    o = Oracle(shape, 0.7, faces=faces, wall_u=wall_u)
    ref = o.sums(o.run(o.init(rho0, u0), 6))
    _, _, _, sums = gpu_run(shape, 0.7, "f64", "swap2", faces, wall_u, rho0, u0, steps=6)
    assert abs(sums[0] - ref[0]) <= 1e-12 * ref[0]
    assert np.abs(sums[1:] - ref[1:]).max() <= 1e-12 * ref[0]


def test_repeat_runs_are_bitwise_identical():
    shape = (40, 70, 45)
    rho0, u0 = _noisy_init(shape, 500)
    out = []
    for _ in range(2):
        lat, _, _, _ = gpu_run(shape, 0.6, "f32", "swap2", rho0=rho0, u0=u0, steps=6)
        out.append(lat.f.cpu().numpy().copy())
    assert np.array_equal(out[0].view(np.uint32), out[1].view(np.uint32))


def test_resume_from_state_equals_one_run():
    shape = (40, 70, 45)
    rho0, u0 = _noisy_init(shape, 600)
    a, _, _, _ = gpu_run(shape, 0.6, "f32", "swap2", rho0=rho0, u0=u0, steps=8)
    b, _, _, _ = gpu_run(shape, 0.6, "f32", "swap2", rho0=rho0, u0=u0, steps=4)
    c = Lattice(shape, 0.6, "f32", "swap2", f=b.f.clone())
    c.step(4)
    torch.cuda.synchronize()
    assert np.array_equal(a.f.cpu().numpy().view(np.uint32), c.f.cpu().numpy().view(np.uint32))


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("case", [0, 4, 5])
def test_step_into_matches_in_place(storage, case):
    # the out-of-place pass runs the same per-cell arithmetic: bitwise equal
    # to the in-place update, and the source stays untouched
    shape, faces, wall_u = CASES[case]
    rho0, u0 = _noisy_init(shape, 300 + case)
    print(f"[gpu] step_into {storage} {shape}", flush=True)
    for scheme in SCHEMES:
        lat, _, _, _ = gpu_run(shape, 0.6, storage, scheme, faces, wall_u, rho0, u0, steps=3)
        src = lat.f.clone()
        for k in (1, 2):
            dst = torch.empty_like(src)
            lat.step_into(src, dst, k)
            ref = lat.f.clone()
            lat.step(k)
            torch.cuda.synchronize()
            assert torch.equal(lat.f.view(torch.int8), dst.view(torch.int8)), (scheme, k)
            lat.f.copy_(ref)
        assert torch.equal(src.view(torch.int8), lat.f.view(torch.int8))


# degenerate lattices: single cells, axes of length 1 and 2 (periodic axes
# shorter than the halo wrap onto the tile itself), odd z (plain layout)
DEGENERATE = [
    ((1, 1, 1), (PERIODIC,) * 6, (0.0, 0.0, 0.0)),
    ((2, 2, 2), (PERIODIC,) * 6, (0.0, 0.0, 0.0)),
    ((1, 5, 6), (PERIODIC, PERIODIC, WALL, WALL, WALL, MOVING_WALL), (0.02, 0.01, 0.0)),
    ((3, 1, 4), (WALL, WALL, PERIODIC, PERIODIC, WALL, WALL), (0.0, 0.0, 0.0)),
    ((5, 3, 1), (WALL, MOVING_WALL, WALL, WALL, PERIODIC, PERIODIC), (0.0, 0.03, 0.0)),
    ((4, 2, 7), (WALL,) * 6, (0.0, 0.0, 0.0)),
    ((9, 1, 2), (PERIODIC,) * 6, (0.0, 0.0, 0.0)),
]


@pytest.mark.parametrize("case", range(len(DEGENERATE)))
def test_degenerate_lattices_match_oracle(case):
    shape, faces, wall_u = DEGENERATE[case]
    rho0, u0 = _noisy_init(shape, 500 + case)
    o = Oracle(shape, 0.7, faces=faces, wall_u=wall_u)
    for steps in (0, 1, 2, 5):
        ref = o.run(o.init(rho0, u0), steps)
        for scheme in SCHEMES:
            lat, _, _, _ = gpu_run(shape, 0.7, "f64", scheme, faces, wall_u, rho0, u0, steps=steps)
            assert rel(lat.distributions(), ref) <= 1e-12, (scheme, steps)
            lat32, _, _, _ = gpu_run(shape, 0.7, "f32", scheme, faces, wall_u, rho0, u0, steps=steps)
            assert rel(lat32.distributions(), ref) <= 2e-6, (scheme, steps)


@pytest.mark.parametrize("shape", [(40, 70, 46), (40, 70, 45)])  # pair-and-ring and plain layouts
def test_a_wait_that_gives_up_is_reported_and_stays_reported(shape):
    # failure path of the in-place hazard wait, forced from the host: every
    # wait requires unreachable progress and gives up after a few polls; the
    # passes still complete (accesses stay in bounds) and the time-out shows
    # in lbm_macroscopic, also after later, normal passes
    lat = Lattice(shape, 0.6, "f32", "swap2")
    lat.step(2)
    assert np.isfinite(lat.sums()).all()  # a normal pass reports nothing
    capi.lbm_test_force_wait_timeout(lat.ctx, True)
    print("[gpu] forced hazard-wait time-outs", flush=True)
    lat.step(4)
    with pytest.raises(capi.LbmError) as ei:
        lat.sums()
    assert ei.value.status == capi.LBM_EDEVICE and "timed out" in str(ei.value)
    capi.lbm_test_force_wait_timeout(lat.ctx, False)
    lat.step(2)
    with pytest.raises(capi.LbmError):
        lat.sums()
    lat.close()
    # a new context starts with a clear report
    lat = Lattice(shape, 0.6, "f32", "swap2")
    lat.step(2)
    assert np.isfinite(lat.sums()).all()
    lat.close()
