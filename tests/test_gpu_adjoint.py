"""GPU discrete adjoint (through the C ABI) against the FP64 oracle's adjoint,
and the whole-run force gradient against central finite differences; 16-bit
storage against the FP32 adjoint on the decoded state; D3Q15 and D3Q27
against the adjoint of the oracle of the set."""
import numpy as np
import pytest
import torch

from oracle import PERIODIC, WALL, Oracle, OracleQ
from paper_2208_05429_amd import workloads as wl
from paper_2208_05429_amd import capi
from paper_2208_05429_amd.adjoint import force_gradient
from paper_2208_05429_amd.lattice import Lattice, real_dtype

pytestmark = pytest.mark.gpu

FACES = (PERIODIC, PERIODIC, WALL, WALL, WALL, WALL)
NAMES = ("periodic", "periodic", "wall", "wall", "wall", "wall")


def _init(shape, seed):
    rho0, u0 = wl.taylor_green_3d(shape, 0.03)
    return wl.random_density(shape, 0.01, seed), u0 + wl.uniform_noise(shape, 5e-3, seed + 1)


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 2e-6)])
def test_adjoint_seed_and_one_step_match_oracle(storage, tol):
    shape = (10, 13, 12)
    rho0, u0 = _init(shape, 5)
    F = wl.normal_field(shape, 1e-4, 6)
    o = Oracle(shape, 0.8, faces=FACES)
    f_t = o.run(o.init(rho0, u0), 3, F)
    lam_next = wl.normal_field(shape, 1.0, 7, comps=19)
    ut = wl.normal_field(shape, 1e-2, 8)
    seed_ref, gseed_ref = o.loss_seed(f_t, ut, F)
    lam_ref, g_ref = o.adjoint_step(f_t, lam_next, F)

    rdt = real_dtype(storage)
    lat = Lattice(shape, 0.8, storage, "swap2", NAMES, force=torch.as_tensor(F),
                  rho0=torch.as_tensor(rho0), u0=torch.as_tensor(u0))
    lat.step(3)
    _, u, _, _ = lat.macroscopic(want=("u",))
    gu = (2 * (u - torch.as_tensor(ut, device=u.device))).to(rdt).contiguous()
    lam = torch.empty((19,) + shape, dtype=rdt, device="cuda")
    gF = torch.zeros((3,) + shape, dtype=rdt, device="cuda")
    capi.lbm_macro_adjoint(lat.ctx, lat.f.data_ptr(), gu.data_ptr(), lam.data_ptr(), gF.data_ptr())
    torch.cuda.synchronize()
    e = np.abs(lam.double().cpu().numpy() - seed_ref).max() / np.abs(seed_ref).max()
    assert e <= 10 * tol, e
    assert np.abs(gF.double().cpu().numpy() - gseed_ref).max() <= 10 * tol * np.abs(gseed_ref).max()

    lin = torch.as_tensor(lam_next, dtype=rdt, device="cuda").contiguous()
    lout = torch.empty_like(lin)
    g = torch.zeros((3,) + shape, dtype=rdt, device="cuda")
    capi.lbm_step_adjoint(lat.ctx, lat.f.data_ptr(), lin.data_ptr(), lout.data_ptr(), g.data_ptr(), 1)
    torch.cuda.synchronize()
    e = np.abs(lout.double().cpu().numpy() - lam_ref).max() / np.abs(lam_ref).max()
    assert e <= 10 * tol, e
    eg = np.abs(g.double().cpu().numpy() - g_ref).max() / np.abs(g_ref).max()
    assert eg <= 10 * tol, eg
    lat.close()


def _channel_problem(shape, steps, storage):
    rho0, u0 = _init(shape, 11)
    o = Oracle(shape, 0.8, faces=FACES)
    f0 = o.init(rho0, u0)
    F = wl.normal_field(shape, 1e-6, 1)
    hidden = wl.normal_field(shape, 1e-6, 2)
    _, ut, _ = o.macro(o.run(f0, steps, hidden), hidden)
    lat0 = Lattice(shape, 0.8, storage, "swap2", NAMES, rho0=torch.as_tensor(rho0), u0=torch.as_tensor(u0))
    f0_dev = lat0.f.clone()
    lat0.close()
    return o, f0, F, ut, f0_dev


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_force_gradient_matches_oracle_adjoint(storage):
    shape, steps = (16, 12, 10), 12
    o, f0, F, ut, f0_dev = _channel_problem(shape, steps, storage)
    L_ref, g_ref = o.loss_and_grad(f0, F, ut, steps)
    spec = dict(shape=shape, tau=0.8, storage=storage, faces=NAMES, steps=steps, checkpoint=4)
    L, g = force_gradient(torch.as_tensor(F, device="cuda"), f0_dev, spec, torch.as_tensor(ut, device="cuda"))
    g = g.double().cpu().numpy()
    assert abs(L - L_ref) <= (1e-10 if storage == "f64" else 1e-3) * L_ref
    err = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    print(f"{storage}: gradient error vs oracle adjoint {err:.3e}")
    assert err <= (1e-10 if storage == "f64" else 1e-3)


def test_force_gradient_matches_central_differences_fp64():
    # FD in FP64 on the GPU path (eps 1e-4 on the force), like the adjoint workload, smaller
    shape, steps = (16, 12, 10), 12
    o, f0, F, ut, f0_dev = _channel_problem(shape, steps, "f64")
    spec = dict(shape=shape, tau=0.8, storage="f64", faces=NAMES, steps=steps, checkpoint=4)
    Ft = torch.as_tensor(F, device="cuda")
    utt = torch.as_tensor(ut, device="cuda")
    _, g = force_gradient(Ft, f0_dev, spec, utt)
    g = g.cpu().numpy()
    from paper_2208_05429_amd.adjoint import ForceAdjoint

    def fd(x, y, z, a, eps):
        vals = []
        for sgn in (1, -1):
            Fp = Ft.clone()
            Fp[a, x, y, z] += sgn * eps
            u = ForceAdjoint.apply(Fp, f0_dev, spec)
            vals.append(float(((u - utt) ** 2).sum()))
        return (vals[0] - vals[1]) / (2 * eps)

    gmax = np.abs(g).max()
    for (x, y, z) in wl.sample_cells(shape, 4, 3):
        for a in range(3):
            # the loss is not quadratic in F: central differences at the
            # workload's eps = 1e-4 carry an O(eps^2) term (up to 1e-4 of
            # max|grad| here); Richardson extrapolation over eps, eps/2 removes it
            d1, d2 = fd(x, y, z, a, 1e-4), fd(x, y, z, a, 5e-5)
            assert abs(d1 - g[a, x, y, z]) <= 2e-4 * gmax, (x, y, z, a)
            assert abs((4 * d2 - d1) / 3 - g[a, x, y, z]) <= 1e-6 * gmax, (x, y, z, a)


# Two merged reverse steps (one pass, f_{t+1} recomputed on chip) against two
# single reverse steps of the oracle.  Shapes span several tiles (FP32: the
# fewest tiles of 12x28, 10x32 and 16x16: 12x28 for the first four cases,
# 10x32 for the last; FP64: 8x16) with ragged last tiles and several x segments.
MERGED_CASES = [
    ((40, 21, 19), (PERIODIC, PERIODIC, WALL, WALL, WALL, WALL), (0.0, 0.0, 0.0), True),
    ((24, 18, 37), (PERIODIC,) * 6, (0.0, 0.0, 0.0), True),
    ((17, 20, 22), (WALL, WALL, WALL, 2, WALL, WALL), (0.04, 0.0, -0.01), True),
    ((19, 13, 26), (2, WALL, PERIODIC, PERIODIC, WALL, WALL), (0.0, 0.03, 0.02), False),
    ((18, 30, 61), (WALL, WALL, PERIODIC, PERIODIC, WALL, 2), (0.02, 0.03, 0.0), True),
]


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 2e-6)])
@pytest.mark.parametrize("case", range(len(MERGED_CASES)))
def test_merged_adjoint_matches_two_single_steps(storage, tol, case):
    shape, faces, wall_u, with_force = MERGED_CASES[case]
    names = [{PERIODIC: "periodic", WALL: "wall", 2: "moving"}[f] for f in faces]
    print(f"[gpu] merged adjoint {storage} {shape} {names} force={with_force}", flush=True)
    rho0, u0 = _init(shape, 31 + case)
    F = wl.normal_field(shape, 1e-4, 32 + case) if with_force else None
    o = Oracle(shape, 0.7, faces=faces, wall_u=wall_u)
    f_t = o.run(o.init(rho0, u0), 2, F)
    f_t1 = o.run(f_t, 1, F)
    lam2 = wl.normal_field(shape, 1.0, 33 + case, comps=19)
    lam1, g1 = o.adjoint_step(f_t1, lam2, F)
    lam0, g0 = o.adjoint_step(f_t, lam1, F, g1)

    rdt = real_dtype(storage)
    force = None if F is None else torch.as_tensor(F)
    lat = Lattice(shape, 0.7, storage, "swap2", names, wall_u, force=force, rho0=torch.as_tensor(rho0),
                  u0=torch.as_tensor(u0))
    lat.step(2)
    lin = torch.as_tensor(lam2, dtype=rdt, device="cuda").contiguous()
    lout = torch.empty_like(lin)
    gF = torch.zeros((3,) + shape, dtype=rdt, device="cuda")
    gptr = gF.data_ptr() if F is not None else None
    capi.lbm_step_adjoint(lat.ctx, lat.f.data_ptr(), lin.data_ptr(), lout.data_ptr(), gptr, 2)
    torch.cuda.synchronize()
    e = np.abs(lout.double().cpu().numpy() - lam0).max() / np.abs(lam0).max()
    assert e <= 10 * tol, e
    if F is not None:
        eg = np.abs(gF.double().cpu().numpy() - g0).max() / np.abs(g0).max()
        assert eg <= 10 * tol, eg
    # and against two single-step launches of the library itself
    f1 = lat.f.clone()
    lat.step(1)
    mid = torch.empty_like(lin)
    g2 = torch.zeros_like(gF)
    gptr2 = g2.data_ptr() if F is not None else None
    capi.lbm_step_adjoint(lat.ctx, lat.f.data_ptr(), lin.data_ptr(), mid.data_ptr(), gptr2, 1)
    lout1 = torch.empty_like(lin)
    capi.lbm_step_adjoint(lat.ctx, f1.data_ptr(), mid.data_ptr(), lout1.data_ptr(), gptr2, 1)
    torch.cuda.synchronize()
    e2 = (lout1.double() - lout.double()).abs().max().item() / lout1.double().abs().max().item()
    assert e2 <= 10 * tol, e2
    lat.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_force_gradient_merged_matches_oracle_adjoint(storage):
    shape, steps = (16, 12, 10), 12
    o, f0, F, ut, f0_dev = _channel_problem(shape, steps, storage)
    L_ref, g_ref = o.loss_and_grad(f0, F, ut, steps)
    for ck in (4, 5):  # even and odd checkpoint segments (odd ones end with one single reverse step)
        spec = dict(shape=shape, tau=0.8, storage=storage, faces=NAMES, steps=steps, checkpoint=ck, merged=True)
        L, g = force_gradient(torch.as_tensor(F, device="cuda"), f0_dev, spec, torch.as_tensor(ut, device="cuda"))
        g = g.double().cpu().numpy()
        err = np.abs(g - g_ref).max() / np.abs(g_ref).max()
        print(f"{storage} checkpoint {ck}: merged-adjoint gradient error vs oracle adjoint {err:.3e}")
        assert err <= (1e-10 if storage == "f64" else 1e-3)


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("merged,intervals", [(True, (2, 4, 6, 12)), (False, (1, 5, 12))])
def test_force_gradient_does_not_depend_on_the_checkpoint_interval(storage, merged, intervals):
    # The reverse passes group the steps the same way for all these intervals
    # (merged: even ones), and a state reached in place, out of place or
    # recomputed is the same to the bit (FP32 and FP64), so keeping every
    # (other) state, or only the first, gives the same gradient bitwise.
    shape, steps = (16, 12, 10), 12
    o, f0, F, ut, f0_dev = _channel_problem(shape, steps, storage)
    Fd, utd = torch.as_tensor(F, device="cuda"), torch.as_tensor(ut, device="cuda")
    out = {}
    for ck in intervals:
        spec = dict(shape=shape, tau=0.8, storage=storage, faces=NAMES, steps=steps, checkpoint=ck, merged=merged)
        out[ck] = force_gradient(Fd, f0_dev, spec, utd)
    L0, g0 = out[intervals[0]]
    assert torch.isfinite(g0).all() and g0.abs().max() > 0
    for ck in intervals[1:]:
        L, g = out[ck]
        assert L == L0, ck
        assert torch.equal(g, g0), (ck, (g - g0).abs().max().item())


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_force_gradient_does_not_depend_on_the_forward_scheme(storage):
    # the three schemes (and the merged one on the 16 x 16 tiles of kernel
    # variant 5) reach the same states to the bit, so the checkpointed forward
    # and the recompute give the same gradient whichever one runs them
    shape, steps = (16, 12, 10), 12
    o, f0, F, ut, f0_dev = _channel_problem(shape, steps, storage)
    Fd, utd = torch.as_tensor(F, device="cuda"), torch.as_tensor(ut, device="cuda")
    out = {}
    runs = [("swap2", 0), ("swap1", 0), ("two_array", 0)] + ([("swap2", 5)] if storage == "f32" else [])
    for scheme, variant in runs:
        spec = dict(shape=shape, tau=0.8, storage=storage, faces=NAMES, steps=steps, checkpoint=5, merged=True,
                    scheme=scheme, variant=variant)
        out[scheme if variant == 0 else f"{scheme} variant {variant}"] = force_gradient(Fd, f0_dev, spec, utd)
    L0, g0 = out["swap2"]
    for scheme in [k for k in out if k != "swap2"]:
        L, g = out[scheme]
        assert L == L0, scheme
        assert torch.equal(g, g0), (scheme, (g - g0).abs().max().item())


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("shape", [(10, 13, 12), (9, 30, 70), (8, 30, 61)])
def test_16bit_adjoint_equals_fp32_adjoint_on_the_decoded_state(storage, shape):
    # A 16-bit offset decodes exactly into FP32 and the adjoint computes in
    # FP32 for both storages, so on the same decoded state the seed, one
    # reverse step and two merged reverse steps (f_{t+1} recomputed on chip)
    # equal the FP32 ones bit for bit; the FP32 adjoint is held to the
    # oracle's above.  (10, 13, 12) takes 16 x 16 merged-adjoint tiles,
    # (9, 30, 70) 12 x 28 ones and (8, 30, 61) 10 x 32 ones (several, with
    # ragged edges).
    rho0, u0 = _init(shape, 21)
    F = torch.as_tensor(wl.normal_field(shape, 1e-4, 22))
    print(f"[gpu] 16-bit adjoint {storage} {shape}", flush=True)
    lat16 = Lattice(shape, 0.8, storage, "swap2", NAMES, force=F, rho0=torch.as_tensor(rho0),
                    u0=torch.as_tensor(u0))
    lat16.step(3)
    lat32 = Lattice(shape, 0.8, "f32", "swap2", NAMES, force=F, f=lat16.f.to(torch.float32).contiguous())
    torch.cuda.synchronize()
    gu = torch.as_tensor(wl.normal_field(shape, 1e-2, 23), dtype=torch.float32, device="cuda").contiguous()
    lam_next = torch.as_tensor(wl.normal_field(shape, 1.0, 24, comps=19), dtype=torch.float32,
                               device="cuda").contiguous()

    def adjoints(lat):
        lam = torch.empty((19,) + shape, dtype=torch.float32, device="cuda")
        gF = torch.zeros((3,) + shape, dtype=torch.float32, device="cuda")
        capi.lbm_macro_adjoint(lat.ctx, lat.f.data_ptr(), gu.data_ptr(), lam.data_ptr(), gF.data_ptr())
        out = [lam, gF]
        for k in (1, 2):
            lout = torch.empty_like(lam_next)
            g = torch.zeros((3,) + shape, dtype=torch.float32, device="cuda")
            capi.lbm_step_adjoint(lat.ctx, lat.f.data_ptr(), lam_next.data_ptr(), lout.data_ptr(), g.data_ptr(), k)
            out += [lout, g]
        torch.cuda.synchronize()
        return out

    names = ("seed lambda", "seed dL/dF", "1 step lambda", "1 step dL/dF", "2 steps lambda", "2 steps dL/dF")
    for name, x, y in zip(names, adjoints(lat16), adjoints(lat32)):
        assert torch.isfinite(x).all() and x.abs().max() > 0, name
        assert torch.equal(x.view(torch.int32), y.view(torch.int32)), (name, (x - y).abs().max().item())
    lat16.close()
    lat32.close()


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_16bit_force_gradient_does_not_depend_on_the_checkpoint_interval(storage):
    # Through autograd with 16-bit storage: with merged passes every even
    # interval reaches the same 16-bit states (in place, out of place or
    # recomputed: bitwise equal), so the gradient is the same to the bit.
    # (Single-step and merged passes round differently in 16 bits.)
    shape, steps = (16, 12, 10), 12
    o, f0, F, ut, f0_dev = _channel_problem(shape, steps, storage)
    Fd, utd = torch.as_tensor(F, device="cuda"), torch.as_tensor(ut, device="cuda")
    out = {}
    for ck in (2, 4, 6, 12):
        spec = dict(shape=shape, tau=0.8, storage=storage, faces=NAMES, steps=steps, checkpoint=ck, merged=True)
        out[ck] = force_gradient(Fd, f0_dev, spec, utd)
    L0, g0 = out[2]
    assert torch.isfinite(g0).all() and g0.abs().max() > 0
    for ck in (4, 6, 12):
        L, g = out[ck]
        assert L == L0, ck
        assert torch.equal(g, g0), (ck, (g - g0).abs().max().item())


# ---------------------------------------------------------------------------
# D3Q15 and D3Q27: the seed, one reverse step and two merged reverse steps,
# against the adjoint of the oracle of the set (pinned on the CPU by
# differences of its forward step)

@pytest.mark.parametrize("q", [15, 27])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 2e-6)])
def test_sets_adjoint_seed_and_one_step_match_oracle(q, storage, tol):
    shape = (10, 13, 12)
    rho0, u0 = _init(shape, 31)
    F = wl.normal_field(shape, 1e-4, 32)
    o = OracleQ(shape, 0.8, q, faces=FACES)
    f_t = o.run(o.init(rho0, u0), 3, F)
    lam_next = wl.normal_field(shape, 1.0, 33, comps=q)
    ut = wl.normal_field(shape, 1e-2, 34)
    seed_ref, gseed_ref = o.loss_seed(f_t, ut, F)
    lam_ref, g_ref = o.adjoint_step(f_t, lam_next, F)

    rdt = real_dtype(storage)
    print(f"[gpu] D3Q{q} adjoint {storage}", flush=True)
    lat = Lattice(shape, 0.8, storage, "swap2", NAMES, force=torch.as_tensor(F), rho0=torch.as_tensor(rho0),
                  u0=torch.as_tensor(u0), velocities=q)
    lat.step(3)
    _, u, _, _ = lat.macroscopic(want=("u",))
    gu = (2 * (u - torch.as_tensor(ut, device=u.device))).to(rdt).contiguous()
    lam = torch.empty((q,) + shape, dtype=rdt, device="cuda")
    gF = torch.zeros((3,) + shape, dtype=rdt, device="cuda")
    capi.lbm_macro_adjoint(lat.ctx, lat.f.data_ptr(), gu.data_ptr(), lam.data_ptr(), gF.data_ptr())
    torch.cuda.synchronize()
    e = np.abs(lam.double().cpu().numpy() - seed_ref).max() / np.abs(seed_ref).max()
    assert e <= 10 * tol, e
    assert np.abs(gF.double().cpu().numpy() - gseed_ref).max() <= 10 * tol * np.abs(gseed_ref).max()

    lin = torch.as_tensor(lam_next, dtype=rdt, device="cuda").contiguous()
    lout = torch.empty_like(lin)
    g = torch.zeros((3,) + shape, dtype=rdt, device="cuda")
    capi.lbm_step_adjoint(lat.ctx, lat.f.data_ptr(), lin.data_ptr(), lout.data_ptr(), g.data_ptr(), 1)
    torch.cuda.synchronize()
    e = np.abs(lout.double().cpu().numpy() - lam_ref).max() / np.abs(lam_ref).max()
    assert e <= 10 * tol, e
    eg = np.abs(g.double().cpu().numpy() - g_ref).max() / np.abs(g_ref).max()
    assert eg <= 10 * tol, eg
    lat.close()


@pytest.mark.parametrize("q", [15, 27])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_sets_force_gradient_matches_oracle_adjoint(q, storage):
    # through autograd with single reverse steps, checkpoint every 4 steps
    shape, steps = (16, 12, 10), 12
    rho0, u0 = _init(shape, 41)
    o = OracleQ(shape, 0.8, q, faces=FACES)
    f0 = o.init(rho0, u0)
    F = wl.normal_field(shape, 1e-6, 42)
    _, ut, _ = o.macro(o.run(f0, steps, wl.normal_field(shape, 1e-6, 43)))
    L_ref, g_ref = o.loss_and_grad(f0, F, ut, steps)
    lat0 = Lattice(shape, 0.8, storage, "swap2", NAMES, rho0=torch.as_tensor(rho0), u0=torch.as_tensor(u0),
                   velocities=q)
    f0_dev = lat0.f.clone()
    lat0.close()
    spec = dict(shape=shape, tau=0.8, storage=storage, faces=NAMES, steps=steps, checkpoint=4, merged=False)
    L, g = force_gradient(torch.as_tensor(F, device="cuda"), f0_dev, spec, torch.as_tensor(ut, device="cuda"))
    g = g.double().cpu().numpy()
    assert abs(L - L_ref) <= (1e-10 if storage == "f64" else 1e-3) * L_ref
    err = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    print(f"D3Q{q} {storage}: gradient error vs the set oracle's adjoint {err:.3e}")
    assert err <= (1e-10 if storage == "f64" else 1e-3)


@pytest.mark.parametrize("q", [15, 27])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 2e-6)])
@pytest.mark.parametrize("case", [0, 2, 4])
def test_sets_merged_adjoint_matches_the_oracle(q, storage, tol, case):
    # k = 2: f_{t+1} recomputed on chip, against two reverse steps of the set
    # oracle (case 0: 16 x 16 adjoint tiles; 2, 4: 12 x 28, walls, a lid, force)
    shape, faces, wall_u, with_force = MERGED_CASES[case]
    names = [{PERIODIC: "periodic", WALL: "wall", 2: "moving"}[f] for f in faces]
    print(f"[gpu] D3Q{q} merged adjoint {storage} {shape} {names} force={with_force}", flush=True)
    rho0, u0 = _init(shape, 61 + case)
    F = wl.normal_field(shape, 1e-4, 62 + case) if with_force else None
    o = OracleQ(shape, 0.7, q, faces=faces, wall_u=wall_u)
    f_t = o.run(o.init(rho0, u0), 2, F)
    f_t1 = o.run(f_t, 1, F)
    lam2 = wl.normal_field(shape, 1.0, 63 + case, comps=q)
    lam1, g1 = o.adjoint_step(f_t1, lam2, F)
    lam0, g0 = o.adjoint_step(f_t, lam1, F, g1)

    rdt = real_dtype(storage)
    lat = Lattice(shape, 0.7, storage, "swap2", names, wall_u, force=None if F is None else torch.as_tensor(F),
                  rho0=torch.as_tensor(rho0), u0=torch.as_tensor(u0), velocities=q)
    lat.step(2)
    lin = torch.as_tensor(lam2, dtype=rdt, device="cuda").contiguous()
    lout = torch.empty_like(lin)
    gF = torch.zeros((3,) + shape, dtype=rdt, device="cuda")
    capi.lbm_step_adjoint(lat.ctx, lat.f.data_ptr(), lin.data_ptr(), lout.data_ptr(),
                          gF.data_ptr() if F is not None else None, 2)
    torch.cuda.synchronize()
    e = np.abs(lout.double().cpu().numpy() - lam0).max() / np.abs(lam0).max()
    assert e <= 10 * tol, e
    if F is not None:
        eg = np.abs(gF.double().cpu().numpy() - g0).max() / np.abs(g0).max()
        assert eg <= 10 * tol, eg
    lat.close()


@pytest.mark.parametrize("q", [15, 27])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_sets_force_gradient_merged_matches_oracle_adjoint(q, storage):
    shape, steps = (16, 12, 10), 12
    rho0, u0 = _init(shape, 71)
    o = OracleQ(shape, 0.8, q, faces=FACES)
    f0 = o.init(rho0, u0)
    F = wl.normal_field(shape, 1e-6, 72)
    _, ut, _ = o.macro(o.run(f0, steps, wl.normal_field(shape, 1e-6, 73)))
    L_ref, g_ref = o.loss_and_grad(f0, F, ut, steps)
    lat0 = Lattice(shape, 0.8, storage, "swap2", NAMES, rho0=torch.as_tensor(rho0), u0=torch.as_tensor(u0),
                   velocities=q)
    f0_dev = lat0.f.clone()
    lat0.close()
    for ck in (4, 5):  # even and odd checkpoint segments (odd ones end with one single reverse step)
        spec = dict(shape=shape, tau=0.8, storage=storage, faces=NAMES, steps=steps, checkpoint=ck, merged=True)
        L, g = force_gradient(torch.as_tensor(F, device="cuda"), f0_dev, spec, torch.as_tensor(ut, device="cuda"))
        g = g.double().cpu().numpy()
        err = np.abs(g - g_ref).max() / np.abs(g_ref).max()
        print(f"D3Q{q} {storage} checkpoint {ck}: merged-adjoint gradient error {err:.3e}")
        assert err <= (1e-10 if storage == "f64" else 1e-3)


@pytest.mark.parametrize("q", [15, 27])
@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_sets_16bit_adjoint_equals_fp32_adjoint_on_the_decoded_state(q, storage):
    shape = (9, 30, 70)
    rho0, u0 = _init(shape, 51)
    F = torch.as_tensor(wl.normal_field(shape, 1e-4, 52))
    lat16 = Lattice(shape, 0.8, storage, "swap2", NAMES, force=F, rho0=torch.as_tensor(rho0),
                    u0=torch.as_tensor(u0), velocities=q)
    lat16.step(3)
    lat32 = Lattice(shape, 0.8, "f32", "swap2", NAMES, force=F, f=lat16.f.to(torch.float32).contiguous(),
                    velocities=q)
    torch.cuda.synchronize()
    gu = torch.as_tensor(wl.normal_field(shape, 1e-2, 53), dtype=torch.float32, device="cuda").contiguous()
    lam_next = torch.as_tensor(wl.normal_field(shape, 1.0, 54, comps=q), dtype=torch.float32,
                               device="cuda").contiguous()

    def adjoints(lat):
        lam = torch.empty((q,) + shape, dtype=torch.float32, device="cuda")
        gF = torch.zeros((3,) + shape, dtype=torch.float32, device="cuda")
        capi.lbm_macro_adjoint(lat.ctx, lat.f.data_ptr(), gu.data_ptr(), lam.data_ptr(), gF.data_ptr())
        lout = torch.empty_like(lam_next)
        g = torch.zeros((3,) + shape, dtype=torch.float32, device="cuda")
        capi.lbm_step_adjoint(lat.ctx, lat.f.data_ptr(), lam_next.data_ptr(), lout.data_ptr(), g.data_ptr(), 1)
        torch.cuda.synchronize()
        return [lam, gF, lout, g]

    for i, (x, y) in enumerate(zip(adjoints(lat16), adjoints(lat32))):
        assert torch.isfinite(x).all() and x.abs().max() > 0, i
        assert torch.equal(x.view(torch.int32), y.view(torch.int32)), (i, (x - y).abs().max().item())
    lat16.close()
    lat32.close()


def test_step_adjoint_rejects_overlapping_lambda():
    shape = (8, 16, 16)
    lat = Lattice(shape, 0.8, "f32", "swap2")
    n = 19 * 8 * 16 * 16
    buf = torch.zeros(2 * n, device="cuda")
    half = 64 * 19  # lambda_out starts inside lambda_in (256-byte aligned offset)
    with pytest.raises(capi.LbmError) as ei:
        capi.lbm_step_adjoint(lat.ctx, lat.f.data_ptr(), buf.data_ptr(), buf[half:].data_ptr(), None, 2)
    assert ei.value.status == capi.LBM_EINVAL
    lat.close()


def test_merged_adjoint_at_256_cubed_matches_two_single_steps():
    # the bench's bandwidth-bound adjoint workload: 256^3 channel with a body
    # force, FP32, in the launch configuration it is timed in (10 x 32 tiles,
    # six x segments, XCD-ordered work items); the merged kernel against two
    # launches of the single-step adjoint, an independent gather formulation
    # (measured: bit-identical; the bound allows for a different rounding order)
    shape = (256, 256, 256)
    names = ("periodic", "periodic", "wall", "wall", "wall", "wall")
    F = torch.as_tensor(wl.normal_field(shape, 1e-4, 70), dtype=torch.float32)
    print("[gpu] merged adjoint 256^3 f32 channel with force", flush=True)
    lat = Lattice(shape, 0.8, "f32", "swap2", names, force=F)
    lat.step(4)
    f_t = lat.f.clone()
    lat.step(1)
    f_t1 = lat.f.clone()
    g = torch.Generator(device="cuda").manual_seed(71)
    lam2 = torch.randn((19,) + shape, device="cuda", generator=g)
    lout = torch.empty_like(lam2)
    gF = torch.zeros((3,) + shape, device="cuda")
    capi.lbm_step_adjoint(lat.ctx, f_t.data_ptr(), lam2.data_ptr(), lout.data_ptr(), gF.data_ptr(), 2)
    mid = torch.empty_like(lam2)
    ref = torch.empty_like(lam2)
    gR = torch.zeros_like(gF)
    capi.lbm_step_adjoint(lat.ctx, f_t1.data_ptr(), lam2.data_ptr(), mid.data_ptr(), gR.data_ptr(), 1)
    capi.lbm_step_adjoint(lat.ctx, f_t.data_ptr(), mid.data_ptr(), ref.data_ptr(), gR.data_ptr(), 1)
    torch.cuda.synchronize()
    e = ((lout - ref).abs().max() / ref.abs().max()).item()
    eg = ((gF - gR).abs().max() / gR.abs().max()).item()
    print(f"merged vs single steps at 256^3: lambda {e:.3e}, force gradient {eg:.3e}")
    assert e <= 2e-5 and eg <= 2e-5, (e, eg)
    lat.close()


def _oracle_checkpointed_gradient(o, f0, F, ut, steps, k):
    """(L, dL/dF) of the oracle's discrete adjoint at a size where keeping
    every state would not fit: states every k steps, each interval's states
    recomputed by plain steps before its reverse steps.  Only oracle calls, in
    the order of the plain definition (forward, seed, reverse steps)."""
    ckpts = [np.array(f0, copy=True)]
    for _ in range(steps // k):
        ckpts.append(o.run(ckpts[-1], k, F))
    L = o.loss(ckpts[-1], ut, F)
    lam, gF = o.loss_seed(ckpts[-1], ut, F)
    for seg in range(steps // k - 1, -1, -1):
        states = [ckpts[seg]]
        for _ in range(k - 1):
            states.append(o.run(states[-1], 1, F))
        for t in range(k - 1, -1, -1):
            lam, gF = o.adjoint_step(states[t], lam, F, gF)
    return L, gF


def test_adjoint_workload_at_its_stated_size():
    # 128 x 64 x 64 channel (periodic x, bounce-back walls in y and z), tau 0.8,
    # rest state, force N(0, 1e-12) per component (seed 1), target u* = u(T)
    # under a hidden force (seed 2), T = 200, a checkpoint every 20 steps, the
    # merged reverse pass; finite differences at 16 cells (seed 3) x 3 components
    import os

    import oracle
    cfg = wl.CHANNEL_ADJ
    shape, steps, k, tau = cfg["shape"], cfg["steps"], cfg["checkpoint"], cfg["tau"]
    oracle.set_threads(max(1, min(16, os.cpu_count() or 1)))
    o = Oracle(shape, tau, faces=FACES)
    f0 = o.init()
    F = wl.normal_field(shape, cfg["force_std"], cfg["force_seed"])
    hidden = wl.normal_field(shape, cfg["force_std"], cfg["target_seed"])
    _, ut, _ = o.macro(o.run(f0, steps, hidden), hidden)
    print("[gpu] oracle checkpointed adjoint 128x64x64 T=200", flush=True)
    L_ref, g_ref = _oracle_checkpointed_gradient(o, f0, F, ut, steps, k)
    oracle.set_threads(1)
    gmax = np.abs(g_ref).max()
    utt = torch.as_tensor(ut, device="cuda")
    grads = {}
    for storage in ("f64", "f32"):
        print(f"[gpu] merged adjoint {storage} 128x64x64 T=200 checkpoint 20", flush=True)
        lat0 = Lattice(shape, tau, storage, "swap2", NAMES)  # rest state
        f0_dev = lat0.f.clone()
        lat0.close()
        spec = dict(shape=shape, tau=tau, storage=storage, faces=NAMES, steps=steps, checkpoint=k, merged=True)
        L, g = force_gradient(torch.as_tensor(F, device="cuda"), f0_dev, spec, utt.to(real_dtype(storage)))
        grads[storage] = g.double().cpu().numpy()
        err = np.abs(grads[storage] - g_ref).max() / gmax
        print(f"{storage}: L {L:.9e} vs oracle {L_ref:.9e}; gradient error vs oracle adjoint {err:.3e}")
        assert abs(L - L_ref) <= (1e-10 if storage == "f64" else 1e-3) * L_ref
        assert err <= (1e-10 if storage == "f64" else 1e-3)

    # central differences of the FP64 GPU forward (eps 1e-4 on F, Richardson
    # with eps/2 to remove the O(eps^2) term of a loss that is not quadratic)
    f0_64 = Lattice(shape, tau, "f64", "two_array", NAMES).f.clone()
    Fd = torch.as_tensor(F, device="cuda")

    def loss(Fp):
        lat = Lattice(shape, tau, "f64", "two_array", NAMES, force=Fp, f=f0_64.clone())
        lat.step(steps)
        _, u, _, _ = lat.macroscopic(sums=True, want=("u",))
        val = float(((u - utt) ** 2).sum())
        lat.close()
        return val

    def fd(x, y, z, a, eps):
        vals = []
        for sgn in (1, -1):
            Fp = Fd.clone()
            Fp[a, x, y, z] += sgn * eps
            vals.append(loss(Fp))
        return (vals[0] - vals[1]) / (2 * eps)

    worst = [0.0, 0.0, 0.0]
    for (x, y, z) in wl.sample_cells(shape, cfg["fd_cells"], cfg["cell_seed"]):
        for a in range(3):
            d1, d2 = fd(x, y, z, a, cfg["fd_eps"]), fd(x, y, z, a, cfg["fd_eps"] / 2)
            rich = (4 * d2 - d1) / 3
            worst[0] = max(worst[0], abs(rich - grads["f64"][a, x, y, z]) / gmax)
            worst[1] = max(worst[1], abs(rich - grads["f32"][a, x, y, z]) / gmax)
            worst[2] = max(worst[2], abs(d1 - grads["f64"][a, x, y, z]) / gmax)
    print(f"FD (Richardson) vs FP64 adjoint {worst[0]:.3e}, vs FP32 adjoint {worst[1]:.3e}; "
          f"plain eps=1e-4 FD vs FP64 adjoint {worst[2]:.3e} (of max|grad|)")
    assert worst[0] <= 1e-6
    assert worst[1] <= 1e-3
