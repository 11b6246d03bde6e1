"""D3Q15 and D3Q27 (lbm_config.velocities; Sec. 4.1 names both as velocity
sets the two-step rule holds for) through the C ABI against the FP64 oracle
of the same set (oracle/lbm_oracle_q.c, pinned on the CPU): every scheme,
FP64 within 1e-12 and FP32 within 2e-6 of the oracle per field, and the
in-place single-copy schemes equal to the two-array kernel to the bit (the
same per-cell arithmetic).  Ragged tiles, walls, a moving lid, a body force,
odd step counts; FP32 over 100 steps on the 32^3 Taylor-Green vortex; planes
in rounds; FP16/BF16 storage pinned by the half-ulp bound of one store.  (The
sets' adjoint is tested in test_gpu_adjoint.py.)"""
import numpy as np
import pytest
import torch

from oracle import MOVING_WALL, PERIODIC, WALL, OracleQ
from paper_2208_05429_amd import capi
from paper_2208_05429_amd import workloads as wl
from paper_2208_05429_amd.lattice import Lattice, real_dtype

pytestmark = pytest.mark.gpu

NAMES = {PERIODIC: "periodic", WALL: "wall", MOVING_WALL: "moving"}
CASES = [
    ((20, 37, 45), (WALL, WALL, WALL, MOVING_WALL, WALL, WALL), (0.05, 0.0, -0.02)),
    ((23, 30, 61), (PERIODIC, PERIODIC, WALL, WALL, MOVING_WALL, WALL), (0.03, -0.02, 0.0)),
    ((17, 41, 33), (PERIODIC,) * 6, (0.0, 0.0, 0.0)),
    ((26, 13, 70), (MOVING_WALL, WALL, PERIODIC, PERIODIC, WALL, WALL), (0.0, 0.04, 0.01)),
    ((6, 5, 7), (PERIODIC,) * 6, (0.0, 0.0, 0.0)),  # one tile smaller than the halo frame
    # even nz: D3Q15 in FP32 takes the pair-and-ring layout
    ((19, 35, 130), (PERIODIC,) * 6, (0.0, 0.0, 0.0)),
    ((20, 37, 68), (WALL, WALL, WALL, MOVING_WALL, WALL, WALL), (0.05, 0.0, -0.02)),
    ((12, 18, 6), (PERIODIC, PERIODIC, WALL, WALL, MOVING_WALL, WALL), (0.03, -0.02, 0.0)),
]


def rel(a, b):
    return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-300))


def _init(shape, seed):
    _, u0 = wl.taylor_green_3d(shape, 0.03)
    return wl.random_density(shape, 0.01, seed + 1), u0 + wl.uniform_noise(shape, 5e-3, seed)


def _run(q, shape, tau, storage, scheme, faces, wall_u, rho0, u0, steps, F=None):
    print(f"[gpu] D3Q{q} {storage} {scheme} {shape} {steps} steps faces={faces}", flush=True)
    force = None if F is None else torch.as_tensor(F, dtype=real_dtype(storage))
    lat = Lattice(shape, tau, storage, scheme, [NAMES[f] for f in faces], wall_u, force, torch.as_tensor(rho0),
                  torch.as_tensor(u0), velocities=q)
    lat.step(steps)
    rho, u, un, sums = lat.macroscopic(sums=True)
    torch.cuda.synchronize()
    out = (lat.distributions(), rho.cpu().numpy(), u.cpu().numpy(), un.cpu().numpy(), sums, lat.f.clone())
    lat.close()
    return out


@pytest.mark.parametrize("q", [15, 27])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 2e-6)])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_sets_match_the_oracle_and_schemes_agree(q, storage, tol, case):
    shape, faces, wall_u = CASES[case]
    rho0, u0 = _init(shape, 600 + case)
    steps = 9
    o = OracleQ(shape, 0.7, q, faces=faces, wall_u=wall_u)
    ref = o.run(o.init(rho0, u0), steps)
    r_ref, u_ref, un_ref = o.macro(ref)
    s_ref = o.sums(ref)
    base = None
    for scheme in ("two_array", "swap1", "swap2"):
        f, rho, u, un, sums, raw = _run(q, shape, 0.7, storage, scheme, faces, wall_u, rho0, u0, steps)
        assert rel(f, ref) <= tol and rel(rho, r_ref) <= tol and rel(u, u_ref) <= tol and rel(un, un_ref) <= tol
        assert abs(sums[0] - s_ref[0]) <= 1e-12 * s_ref[0] * (1 if storage == "f64" else 1e4)
        view = torch.int64 if storage == "f64" else torch.int32
        if base is None:
            base = raw.view(view)
        else:
            assert torch.equal(raw.view(view), base), scheme


@pytest.mark.parametrize("q", [15, 27])
def test_sets_with_a_body_force(q):
    shape = (24, 20, 18)  # even nz: the pair-and-ring layout for D3Q15
    faces = (PERIODIC, PERIODIC, WALL, WALL, WALL, WALL)
    rho0, u0 = _init(shape, 700)
    F = wl.normal_field(shape, 1e-4, 701)
    o = OracleQ(shape, 0.8, q, faces=faces)
    ref = o.run(o.init(rho0, u0), 7, F)
    _, u_ref, _ = o.macro(ref, F)
    for storage, tol in (("f64", 1e-12), ("f32", 2e-6)):
        base = None
        for scheme in ("two_array", "swap2"):
            f, _, u, _, _, raw = _run(q, shape, 0.8, storage, scheme, faces, (0, 0, 0), rho0, u0, 7, F)
            assert rel(f, ref) <= tol
            view = torch.int64 if storage == "f64" else torch.int32
            if base is None:
                base = raw.view(view)
            else:
                assert torch.equal(raw.view(view), base), (storage, scheme)


@pytest.mark.parametrize("q", [15, 27])
def test_sets_fp32_taylor_green_100_steps(q):
    cfg = wl.TGV_32
    rho0, u0 = wl.taylor_green_3d(cfg["shape"], cfg["u0"])
    o = OracleQ(cfg["shape"], cfg["tau"], q)
    ref = o.run(o.init(rho0, u0), cfg["steps"])
    r_ref, u_ref, un_ref = o.macro(ref)
    for scheme in ("two_array", "swap2"):
        _, rho, u, un, _, _ = _run(q, cfg["shape"], cfg["tau"], "f32", scheme, (PERIODIC,) * 6, (0, 0, 0), rho0, u0,
                                   cfg["steps"])
        e = (rel(rho, r_ref), rel(u, u_ref), rel(un, un_ref))
        print(f"D3Q{q} FP32 {scheme} TGV 32^3 100 steps: rho {e[0]:.2e} u {e[1]:.2e} |u| {e[2]:.2e}")
        assert max(e) <= 2e-6


# planes of more tiles than co-resident workgroups: rounds over bands of tile
# rows, each band's boundary rows saved first (all Q directions)
BANDED = [
    ((6, 272, 1024), (PERIODIC,) * 6, (0.0, 0.0, 0.0)),                               # whole tile rows
    ((5, 282, 999), (WALL, WALL, WALL, MOVING_WALL, WALL, WALL), (0.05, 0.0, 0.01)),  # odd nz, ragged, lid on +y
    ((4, 296, 1024), (PERIODIC,) * 6, (0.0, 0.0, 0.0)),                               # periodic y, ragged last row
    # a short last band marching in x segments of its own (32-bit D3Q15: 16
    # tiles, D3Q27: 32 tiles, 6 segments each)
    ((24, 272, 1024), (PERIODIC,) * 6, (0.0, 0.0, 0.0)),
]


@pytest.mark.parametrize("q", [15, 27])
@pytest.mark.parametrize("storage", ["f32", "f64"])
@pytest.mark.parametrize("case", range(len(BANDED)))
def test_sets_in_rounds_match_two_array_bitwise(q, storage, case):
    shape, faces, wall_u = BANDED[case]
    rho0, u0 = _init(shape, 720 + case)
    view = torch.int64 if storage == "f64" else torch.int32
    base = None
    for scheme in ("two_array", "swap1", "swap2"):
        print(f"[gpu] rounds D3Q{q} {storage} {scheme} {shape}", flush=True)
        lat = Lattice(shape, 0.7, storage, scheme, [NAMES[f] for f in faces], wall_u, rho0=torch.as_tensor(rho0),
                      u0=torch.as_tensor(u0), velocities=q)
        lat.step(3)
        s = lat.sums()  # waits; reports a hazard wait that gave up
        assert np.isfinite(s).all()
        raw = lat.f.view(view).clone()
        lat.close()
        if base is None:
            base = raw
        else:
            assert torch.equal(raw, base), scheme


# ---------------------------------------------------------------------------
# FP16/BF16 offset storage.  From a state whose stored offsets are exact
# 16-bit values, one pass computes in FP32 and rounds each offset once, so every
# stored value lies within half a 16-bit ulp of the oracle of the set run from
# the same decoded state (plus the FP32 arithmetic error).

def _half_ulp(x, storage):
    a = np.abs(x)
    if storage == "f16":
        return 0.5 * 2.0 ** (np.floor(np.log2(np.maximum(a, 2.0 ** -14))) - 10)
    return 0.5 * 2.0 ** (np.floor(np.log2(np.maximum(a, 2.0 ** -126))) - 7)


@pytest.mark.parametrize("q", [15, 27])
@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("scheme,steps", [("swap1", 1), ("swap2", 2), ("two_array", 1)])
@pytest.mark.parametrize("force", [False, True])
def test_sets_16bit_store_is_within_half_an_ulp_of_the_oracle(q, storage, scheme, steps, force):
    from paper_2208_05429_amd.lattice import lattice_weights
    shape = (12, 20, 70)  # even nz: D3Q15 takes the pair-and-ring layout
    faces = (WALL, WALL, WALL, MOVING_WALL, WALL, WALL)
    wall_u = (0.05, 0.0, 0.01)
    rho0, u0 = _init(shape, 740)
    F = wl.normal_field(shape, 1e-3, 741).astype(np.float32).astype(np.float64) if force else None
    print(f"[gpu] D3Q{q} one {storage} store, {scheme}, force {force}", flush=True)
    lat = Lattice(shape, 0.7, storage, scheme, [NAMES[f] for f in faces], wall_u,
                  None if F is None else torch.as_tensor(F), torch.as_tensor(rho0), torch.as_tensor(u0), velocities=q)
    f0 = lat.distributions()  # the decoded 16-bit state: exact in FP64
    lat.step(steps)
    torch.cuda.synchronize()
    w = lattice_weights(q)[:, None, None, None]
    g_gpu = lat.distributions() - w
    lat.close()
    o = OracleQ(shape, 0.7, q, faces=faces, wall_u=wall_u)
    g_ref = o.run(np.ascontiguousarray(f0), steps, F) - w
    err = np.abs(g_gpu - g_ref)
    bound = _half_ulp(np.maximum(np.abs(g_ref), np.abs(g_gpu)), storage) * (1 + 1e-3) + 2e-7
    worst = float((err / bound).max())
    print(f"D3Q{q} {storage} {scheme} force {force}: max err/bound = {worst:.3f}")
    assert worst <= 1.0, worst


@pytest.mark.parametrize("q", [15, 27])
@pytest.mark.parametrize("storage,case", [("f16", 0), ("f16", 1), ("bf16", 2), ("bf16", 3)])
def test_sets_16bit_in_rounds_in_place_matches_out_of_place(q, storage, case):
    # the merged pass rounds to 16 bits once per two steps, so the reference is
    # the same pass out of place (its band edges read the untouched source)
    shape, faces, wall_u = BANDED[case]
    rho0, u0 = _init(shape, 750 + case)
    print(f"[gpu] rounds D3Q{q} {storage} {shape}", flush=True)
    lat = Lattice(shape, 0.6, storage, "swap2", [NAMES[f] for f in faces], wall_u, rho0=torch.as_tensor(rho0),
                  u0=torch.as_tensor(u0), velocities=q)
    a, b = torch.empty_like(lat.f), torch.empty_like(lat.f)
    lat.step_into(lat.f, a, 2)
    lat.step_into(a, b, 2)
    lat.step(4)
    s = lat.sums()
    assert np.isfinite(s).all()
    assert torch.equal(lat.f.view(torch.int16), b.view(torch.int16))
    lat.close()


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_d3q15_16bit_layouts_agree_bitwise(storage):
    # the pair-and-ring and the plain 16 x 64 layouts run the same per-cell
    # arithmetic on the same inputs: their 16-bit stores agree to the bit
    shape, faces, wall_u = CASES[6]
    rho0, u0 = _init(shape, 760)
    states = []
    for variant in (0, 1):
        lat = Lattice(shape, 0.6, storage, "swap2", [NAMES[f] for f in faces], wall_u, rho0=torch.as_tensor(rho0),
                      u0=torch.as_tensor(u0), variant=variant, velocities=15)
        lat.step(5)
        torch.cuda.synchronize()
        states.append(lat.f.view(torch.int16).clone())
        lat.close()
    assert torch.equal(states[0], states[1])


def test_sets_run_without_allocation_too():
    # the allocation-free entry point takes the same configurations
    shape = (20, 24, 30)
    rho0, u0 = _init(shape, 710)
    lat = Lattice(shape, 0.7, "f32", "swap2", ["wall"] * 3 + ["moving"] + ["wall"] * 2, (0.04, 0, 0),
                  rho0=torch.as_tensor(rho0), u0=torch.as_tensor(u0), velocities=27)
    f2 = lat.f.clone()
    lat.step(5)
    capi.lbm_step_static(lat.cfg, f2.data_ptr(), None, 5, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(lat.f.view(torch.int32), f2.view(torch.int32))
    lat.close()


@pytest.mark.parametrize("q,variant", [(15, 1), (15, 2), (15, 3), (27, 1)])
@pytest.mark.parametrize("case", [0, 1, 5, 6])
def test_set_tile_variants_equal_two_array_bitwise(q, variant, case):
    # the larger FP32 tiles (two or three columns per thread)
    shape, faces, wall_u = CASES[case]
    rho0, u0 = _init(shape, 720 + case)
    names = [NAMES[f] for f in faces]
    ref = Lattice(shape, 0.7, "f32", "two_array", names, wall_u, None, torch.as_tensor(rho0), torch.as_tensor(u0),
                  velocities=q)
    print(f"[gpu] D3Q{q} variant {variant} {shape}", flush=True)
    for scheme in ("swap2", "swap1"):
        lat = Lattice(shape, 0.7, "f32", scheme, names, wall_u, None, torch.as_tensor(rho0), torch.as_tensor(u0),
                      variant=variant, velocities=q)
        lat.f.copy_(ref.f)
        r = Lattice(shape, 0.7, "f32", "two_array", names, wall_u, f=ref.f.clone(), velocities=q)
        lat.step(5)
        r.step(5)
        torch.cuda.synchronize()
        assert torch.equal(lat.f.view(torch.int32), r.f.view(torch.int32)), (scheme, variant)
        lat.close()
        r.close()
    ref.close()


@pytest.mark.parametrize("q", [15, 27])
@pytest.mark.parametrize("case", [0, 1, 2, 3, 4, 5])
def test_fp64_tile_variants_equal_two_array_bitwise(q, case):
    # FP64, both tiles of each set (D3Q15 variant 0: 10 x 32, variant 1:
    # 12 x 28; D3Q27 variant 0: 8 x 32, variant 1: 8 x 24), on ragged and
    # walled lattices and, for case 5, a plane that runs in rounds (264 x 1000:
    # D3Q15 10 x 32 in bands of 8, 8, 8 and 3 tile rows, the last in 2 x
    # segments of its own, 12 x 28 in bands of 7, 7, 7 and 1, the last in 6
    # segments; D3Q27 8 x 32 in bands of 8 ending on one row in 6 segments)
    shape, faces, wall_u = (CASES[case] if case < 5 else ((24, 264, 1000), (PERIODIC,) * 6, (0.0, 0.0, 0.0)))
    rho0, u0 = _init(shape, 760 + case)
    names = [NAMES[f] for f in faces]
    ref = Lattice(shape, 0.7, "f64", "two_array", names, wall_u, None, torch.as_tensor(rho0), torch.as_tensor(u0),
                  velocities=q)
    for variant in (0, 1):
        print(f"[gpu] D3Q{q} f64 variant {variant} {shape}", flush=True)
        for scheme in ("swap2", "swap1"):
            lat = Lattice(shape, 0.7, "f64", scheme, names, wall_u, f=ref.f.clone(), variant=variant, velocities=q)
            r = Lattice(shape, 0.7, "f64", "two_array", names, wall_u, f=ref.f.clone(), velocities=q)
            lat.step(5)
            r.step(5)
            torch.cuda.synchronize()
            assert torch.equal(lat.f.view(torch.int64), r.f.view(torch.int64)), (scheme, variant)
            lat.close()
            r.close()
    ref.close()


@pytest.mark.parametrize("q", [15, 27])
def test_sets_512_cubed_fp32_merged_sampled_cells(q):
    # The sets at the size they are measured at: 512^3 periodic Taylor-Green +
    # noise, FP32, two merged steps per pass, in the bench's launch
    # configuration (D3Q15: one round of 16 x 64 pair-and-ring tiles; D3Q27:
    # two rounds of 16 x 32 tiles, two columns per thread).  Sampled cells
    # against the set's oracle run on each cell's dependency cone (exact by
    # the locality of streaming, pinned on the CPU in test_cone_oracle.py).
    from tests.test_gpu_fullsize import gpu_cells, oracle_center
    cfg = wl.TGV_512
    shape, tau, n = cfg["shape"], cfg["tau"], 4
    print(f"[gpu] D3Q{q} 512^3 f32 swap2 sampled cells, {n} steps", flush=True)
    _, u0 = wl.tgv_512_fields(shape)
    lat = Lattice(shape, tau, "f32", "swap2", u0=torch.from_numpy(u0), velocities=q)
    s0 = lat.sums()
    lat.step(n)
    torch.cuda.synchronize()
    s1 = lat.sums()
    # tile seams (y: 16 rows; z: 64 or 32 columns), the D3Q27 band seam (rows
    # 255/256), corners and the x wrap
    cells = [(0, 255, 63), (1, 256, 64), (511, 15, 31), (256, 16, 32), (0, 0, 0), (511, 511, 511),
             (3, 511, 0)] + wl.sample_cells(shape, 10, 13)
    got = gpu_cells(lat, cells, q)
    worst = 0.0
    for c, g in zip(cells, got):
        ref = oracle_center(None, u0, shape, (PERIODIC,) * 6, (0.0, 0.0, 0.0), tau, c, n, q=q)
        err = float(np.abs(g - ref).max())
        worst = max(worst, err)
        assert err <= 2e-7, (c, err)  # FP32 rounding of the offsets over a few steps
    print(f"D3Q{q} 512^3 sampled cells: max abs error {worst:.2e}")
    assert abs(s1[0] - s0[0]) <= 1e-9 * s0[0]
    assert np.abs(s1[1:] - s0[1:]).max() <= 1e-9 * s0[0]
    lat.close()
    del lat
    torch.cuda.empty_cache()


@pytest.mark.parametrize("q", [15, 27])
def test_sets_1024_cubed_fp32_merged_rounds_sampled_cells(q):
    # 1024^3 single copy in rounds (D3Q15: 64 GB, four bands of 16 rows of
    # 16 x 64 tiles; D3Q27: 116 GB, eight bands of 8 rows of 16 x 32 tiles),
    # the random-phase Taylor-Green field built on the device; sampled cells at
    # the band seams, the x wrap and at random against the set's cone oracle
    from tests.test_gpu_fullsize import gpu_cells, oracle_center
    cfg = wl.TGV_1024
    shape, tau, n = cfg["shape"], cfg["tau"], 4
    ph = wl.random_phases(cfg["phase_seed"])
    print(f"[gpu] D3Q{q} 1024^3 f32 swap2 rounds, {n} steps", flush=True)
    u0 = wl.taylor_green_3d_device(shape, cfg["u0"], ph, "cuda")
    lat = Lattice(shape, tau, "f32", "swap2", u0=u0, velocities=q)
    del u0
    torch.cuda.empty_cache()
    s0 = lat.sums()
    lat.step(n)
    torch.cuda.synchronize()
    s1 = lat.sums()
    cells = [(0, 127, 0), (1, 128, 31), (1023, 255, 32), (512, 256, 63), (7, 511, 64), (100, 512, 1023),
             (9, 767, 500), (11, 768, 511), (1023, 1023, 1), (0, 0, 1022)] + wl.sample_cells(shape, 8, 14)
    got = gpu_cells(lat, cells, q)
    ufn = lambda ix, iy, iz: wl.taylor_green_3d_at(shape, cfg["u0"], ph, ix, iy, iz)  # noqa: E731
    for c, g in zip(cells, got):
        ref = oracle_center(None, ufn, shape, (PERIODIC,) * 6, (0.0, 0.0, 0.0), tau, c, n, q=q)
        assert np.abs(g - ref).max() <= 2e-7, c
    assert abs(s1[0] - s0[0]) <= 1e-9 * s0[0]
    assert np.abs(s1[1:] - s0[1:]).max() <= 1e-9 * s0[0]
    lat.close()
    del lat
    torch.cuda.empty_cache()


def test_d3q27_fp64_rounds_across_a_periodic_seam_equal_two_array_bitwise():
    # 257 rows: tiles 8 rows high would leave one row across the periodic seam,
    # so the plane runs 10 x 26 tiles (26 x 10 tiles, 2 rounds, a 7-row last
    # tile row)
    shape, faces = (4, 257, 256), (PERIODIC,) * 6
    rho0, u0 = _init(shape, 780)
    names = [NAMES[f] for f in faces]
    print(f"[gpu] D3Q27 f64 rounds across the seam {shape}", flush=True)
    ref = Lattice(shape, 0.7, "f64", "two_array", names, (0.0, 0.0, 0.0), None, torch.as_tensor(rho0),
                  torch.as_tensor(u0), velocities=27)
    for scheme in ("swap2", "swap1"):
        lat = Lattice(shape, 0.7, "f64", scheme, names, (0.0, 0.0, 0.0), f=ref.f.clone(), velocities=27)
        r = Lattice(shape, 0.7, "f64", "two_array", names, (0.0, 0.0, 0.0), f=ref.f.clone(), velocities=27)
        lat.step(5)
        r.step(5)
        torch.cuda.synchronize()
        assert torch.equal(lat.f.view(torch.int64), r.f.view(torch.int64)), scheme
        lat.close()
        r.close()
    ref.close()


@pytest.mark.parametrize("q", [15, 27])
def test_sets_16bit_rounds_across_a_periodic_seam_in_place_matches_out_of_place(q):
    # 16-bit sets on a 1025-row periodic plane in rounds: 16-row tiles would
    # leave a last row of one across the seam, so the plane takes 12 x 28 tiles
    # (a 5-row last tile row); in place equal to out of place to the bit
    shape = (4, 1025, 1024)
    rho0, u0 = _init(shape, 790 + q)
    print(f"[gpu] D3Q{q} bf16 rounds across the seam {shape}", flush=True)
    lat = Lattice(shape, 0.6, "bf16", "swap2", ["periodic"] * 6, (0.0, 0.0, 0.0), rho0=torch.as_tensor(rho0),
                  u0=torch.as_tensor(u0), velocities=q)
    a, b = torch.empty_like(lat.f), torch.empty_like(lat.f)
    lat.step_into(lat.f, a, 2)
    lat.step_into(a, b, 2)
    lat.step(4)
    torch.cuda.synchronize()
    assert torch.equal(lat.f.view(torch.int16), b.view(torch.int16))
    lat.close()
