"""The measurement probes of the C ABI: the streaming copy copies, and the
access-pattern replica of a marching pass leaves the lattice unchanged (it
stores back what it loaded).  Neither computes anything of the method; they
bound what the marching kernel can reach (bench.py reports both)."""
import pytest
import torch

from paper_2208_05429_amd import capi
from paper_2208_05429_amd.lattice import Lattice

pytestmark = pytest.mark.gpu


def test_copy_probe_copies():
    n = (1 << 22) + 4 * 1000  # bytes, not a multiple of the grid's stride
    src = torch.randint(0, 1 << 30, (n // 4,), dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    for blocks in (1, 256, 4096):
        dst.zero_()
        print(f"[gpu] copy probe {n} bytes, {blocks} workgroups", flush=True)
        capi.lbm_probe_copy(src.data_ptr(), dst.data_ptr(), n, blocks, torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        assert torch.equal(src, dst)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("M", [1, 2])
def test_pattern_probe_leaves_the_lattice_unchanged(storage, M):
    shape = (37, 40, 130)  # ragged tiles in y and z, several x segments
    print(f"[gpu] pattern probe {storage} M={M} {shape}", flush=True)
    lat = Lattice(shape, 0.7, storage, "swap2")
    lat.f.copy_(torch.randn(lat.f.shape, device="cuda").to(lat.f.dtype))
    before = lat.f.clone()
    capi.lbm_probe_pattern(lat.cfg, lat.f.data_ptr(), M, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    view = torch.int32 if storage == "f32" else torch.int16
    assert torch.equal(before.view(view), lat.f.view(view))
    lat.close()


def test_pattern_probe_rejects_what_it_does_not_replicate():
    dummy = torch.empty(256, dtype=torch.uint8, device="cuda")
    for cfg in (capi.make_config((8, 8, 9), 0.7, capi.LBM_F32),  # odd nz: plain layout
                capi.make_config((8, 8, 8), 0.7, capi.LBM_F64)):
        with pytest.raises(capi.LbmError) as e:
            capi.lbm_probe_pattern(cfg, dummy.data_ptr(), 2, torch.cuda.current_stream().cuda_stream)
        assert e.value.status == capi.LBM_EUNSUPPORTED
