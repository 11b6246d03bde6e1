"""Error of the reduced-precision storage forms on the full bench workload.

512^3 periodic Taylor-Green + noise, tau 0.6, 500 steps.  Reference: the FP64
two-array kernel, itself held to 1e-12 of the CPU oracle by the parity tests
(a 512^3 FP64 oracle run of 500 steps is out of reach of the host).  Reported
on the cells [0, 64)^3: err(X) = max|X - X_ref| / max|X_ref| for rho - 1 and
for u as one vector field.  FP16/BF16 storage has no exact reference (every
store rounds): these bounds are the measured orders with a safety factor, not
a parity claim.  The 16-bit forms are pinned instead by the error bound of a
single rounding (the last test).
"""
import numpy as np
import pytest
import torch

from paper_2208_05429_amd import workloads as wl
from paper_2208_05429_amd.lattice import Lattice

pytestmark = pytest.mark.gpu

BOUNDS = {"f32": 1e-5, "f16": 2e-2, "bf16": 1e-1}


def _crop_fields(lat):
    rho, u, _, _ = lat.macroscopic(want=("rho", "u"))
    return (rho[:64, :64, :64] - 1).double().cpu().numpy(), u[:, :64, :64, :64].double().cpu().numpy()


def test_reduced_precision_error_vs_fp64_on_crop():
    cfg = wl.TGV_512
    shape, tau, steps = cfg["shape"], cfg["tau"], cfg["steps"]
    _, u0 = wl.tgv_512_fields(shape)
    u0 = torch.from_numpy(u0).cuda()
    print(f"[gpu] 512^3 FP64 two-array reference, {steps} steps", flush=True)
    ref = Lattice(shape, tau, "f64", "two_array", u0=u0)
    ref.step(steps)
    r_ref, u_ref = _crop_fields(ref)
    ref.close()
    del ref
    torch.cuda.empty_cache()
    errs = {}
    for st in ("f32", "f16", "bf16"):
        print(f"[gpu] 512^3 {st} merged, {steps} steps", flush=True)
        lat = Lattice(shape, tau, st, "swap2", u0=u0)
        lat.step(steps)
        r, u = _crop_fields(lat)
        s = lat.sums()
        lat.close()
        del lat
        torch.cuda.empty_cache()
        er = np.abs(r - r_ref).max() / np.abs(r_ref).max()
        eu = np.abs(u - u_ref).max() / np.abs(u_ref).max()
        errs[st] = (er, eu)
        print(f"{st}: err(rho-1) = {er:.3e}  err(u) = {eu:.3e}  mass drift = {s[0] / np.prod(shape) - 1:.3e}")
        assert np.isfinite(s).all()
        assert eu <= BOUNDS[st], (st, er, eu)
        if st == "f32":
            assert er <= 1e-3, er
    assert errs["f32"][1] < errs["f16"][1] < errs["bf16"][1]


# ---------------------------------------------------------------------------
# Rounding bound of one 16-bit store.  From a state whose stored offsets are
# exact 16-bit values, one pass (one step, or two merged steps whose
# intermediate stays in FP32) computes in FP32 and rounds each offset g once
# to nearest even, so every stored value lies within half a 16-bit ulp of the
# exact FP64 result (the oracle run from the same decoded state), plus the
# FP32 arithmetic error of the collision.  A pin of the 16-bit forms against
# the oracle by the error bound of their one rounding.

def _half_ulp(x, storage):
    a = np.abs(x)
    if storage == "f16":
        e = np.floor(np.log2(np.maximum(a, 2.0 ** -14)))  # subnormals: fixed spacing 2^-24
        return 0.5 * 2.0 ** (e - 10)
    e = np.floor(np.log2(np.maximum(a, 2.0 ** -126)))
    return 0.5 * 2.0 ** (e - 7)


@pytest.mark.parametrize("force", [False, True])
@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("scheme,steps", [("swap1", 1), ("swap2", 2), ("two_array", 1)])
def test_one_16bit_store_is_within_half_an_ulp_of_the_oracle(storage, scheme, steps, force):
    from oracle import MOVING_WALL, WALL, Oracle
    from paper_2208_05429_amd.lattice import lattice_weights
    shape = (12, 20, 70)
    faces = (WALL, WALL, WALL, MOVING_WALL, WALL, WALL)
    names = ("wall", "wall", "wall", "moving", "wall", "wall")
    wall_u = (0.05, 0.0, 0.01)
    rho0, u0 = wl.taylor_green_3d(shape, 0.03)
    u0 = u0 + wl.uniform_noise(shape, 5e-3, 480)
    rho0 = wl.random_density(shape, 0.01, 481)
    # a body force (Guo forcing) is read in FP32: the oracle gets the same FP32 values
    F = wl.normal_field(shape, 1e-3, 482).astype(np.float32).astype(np.float64) if force else None
    print(f"[gpu] one {storage} store, {scheme}, {steps} step(s), force {force}", flush=True)
    lat = Lattice(shape, 0.7, storage, scheme, names, wall_u, force=None if F is None else torch.as_tensor(F),
                  rho0=torch.as_tensor(rho0), u0=torch.as_tensor(u0))
    f0 = lat.distributions()  # the decoded 16-bit state: exact in FP64
    lat.step(steps)
    torch.cuda.synchronize()
    w = lattice_weights()[:, None, None, None]
    g_gpu = lat.distributions() - w
    o = Oracle(shape, 0.7, faces=faces, wall_u=wall_u)
    g_ref = o.run(np.ascontiguousarray(f0), steps, F) - w
    err = np.abs(g_gpu - g_ref)
    # (the binade of the larger of the two: rounding up across a power of two)
    bound = _half_ulp(np.maximum(np.abs(g_ref), np.abs(g_gpu)), storage) * (1 + 1e-3) + 2e-7
    worst = float((err / bound).max())
    print(f"{storage} {scheme} force {force}: max |g - g_ref| = {err.max():.3e}, max err/bound = {worst:.3f}")
    assert worst <= 1.0, worst
    lat.close()
