"""lbm_step_static, the entry point that allocates nothing (its scratch is a
static device array), against lbm_step on a context with a caller-provided
work buffer: the same kernels run on the same state, so the results must be
identical to the bit.  Two calls in a row share the static scratch, the
second on a smaller lattice, so stale contents of the first would show."""
import pytest
import torch

from paper_2208_05429_amd import capi
from paper_2208_05429_amd import workloads as wl
from paper_2208_05429_amd.lattice import Lattice, real_dtype

pytestmark = pytest.mark.gpu


def _compare(shape, tau, storage, scheme, faces, wall_u, steps, force=None, u_amp=0.03, seed=5):
    print(f"[gpu] lbm_step_static vs lbm_step: {storage} {scheme} {shape} {steps} steps faces={faces}", flush=True)
    if shape[0] * shape[1] * shape[2] > 1 << 24:
        # large lattices: the Taylor-Green field built on the device
        u0 = wl.taylor_green_3d_device(shape, u_amp, (0.0, 0.0, 0.0), "cuda")
    else:
        _, u0 = wl.taylor_green_3d(shape, u_amp)
        u0 = torch.as_tensor(u0 + wl.uniform_noise(shape, 1e-3, seed))
    F = None if force is None else torch.as_tensor(force, dtype=real_dtype(storage))
    lat = Lattice(shape, tau, storage, scheme, faces, wall_u, F, None, u0)
    del u0
    f_static = lat.f.clone()
    lat.step(steps)
    timed_out = capi.lbm_step_static(lat.cfg, f_static.data_ptr(), None if lat.force is None else lat.force.data_ptr(),
                                     steps, torch.cuda.current_stream().cuda_stream, report_timeout=True)
    torch.cuda.synchronize()
    assert not timed_out
    view = torch.int64 if storage == "f64" else (torch.int32 if storage == "f32" else torch.int16)
    same = torch.equal(lat.f.view(view), f_static.view(view))
    changed = not torch.equal(f_static.view(view), lat.f.view(view).new_zeros(()).expand_as(f_static))
    lat.close()
    assert same, (shape, storage, scheme)
    assert changed


def test_static_scratch_matches_work_buffer_two_calls_second_smaller():
    # the 512^3 FP32 Taylor-Green workload (merged passes and, for the odd
    # count, one single-step pass), then a smaller ragged lid-driven cavity
    _compare((512, 512, 512), 0.6, "f32", "swap2", ["periodic"] * 6, (0, 0, 0), 3, u_amp=0.02)
    torch.cuda.empty_cache()
    _compare((40, 48, 56), 0.52, "f32", "swap2", ["wall", "wall", "wall", "moving", "wall", "wall"], (0.05, 0, 0), 7)


def test_static_scratch_other_storages_and_force():
    shape = (48, 36, 40)
    F = wl.normal_field(shape, 1e-5, 11)
    _compare(shape, 0.8, "f64", "swap2", ["periodic", "periodic", "wall", "wall", "wall", "wall"], (0, 0, 0), 5,
             force=F)
    _compare((24, 20, 30), 0.7, "bf16", "swap2", ["periodic"] * 6, (0, 0, 0), 4)
    _compare((20, 30, 26), 0.7, "f32", "two_array", ["wall", "wall", "moving", "wall", "periodic", "periodic"],
             (0, 0, 0.04), 3)


def test_static_scratch_rejects_what_does_not_fit():
    # 1024^3 FP32 merged needs about 1.3 GiB of scratch: rejected before any
    # device work (the distribution buffer is never touched)
    cfg = capi.make_config((1024, 1024, 1024), 0.6, capi.LBM_F32, capi.LBM_SWAP2)
    dummy = torch.empty(256, dtype=torch.uint8, device="cuda")
    with pytest.raises(capi.LbmError) as e:
        capi.lbm_step_static(cfg, dummy.data_ptr(), None, 2, torch.cuda.current_stream().cuda_stream)
    assert e.value.status == capi.LBM_EUNSUPPORTED and "scratch" in str(e.value)
    with pytest.raises(capi.LbmError) as e:
        capi.lbm_step_static(capi.make_config((8, 8, 8), 0.5), dummy.data_ptr(), None, 2,
                             torch.cuda.current_stream().cuda_stream)
    assert e.value.status == capi.LBM_EINVAL
