"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/lbm.h declares, and rejects bad arguments with the
documented status codes before touching the device."""
import ctypes

import pytest

from paper_2208_05429_amd import capi


def test_library_exports_every_declared_function():
    L = capi.lib()
    names = capi.header_functions()
    assert set(names) >= {"lbm_buffer_sizes", "lbm_init", "lbm_attach", "lbm_step", "lbm_macroscopic",
                          "lbm_macro_adjoint", "lbm_step_adjoint", "lbm_set_stream", "lbm_last_error", "lbm_destroy"}
    for n in names:
        assert hasattr(L, n), n


def _cfg(**kw):
    base = dict(shape=(32, 32, 32), tau=0.8, storage=capi.LBM_F32, scheme=capi.LBM_SWAP2)
    base.update(kw)
    return capi.make_config(**base)


def _status(cfg):
    f = ctypes.c_size_t(0)
    w = ctypes.c_size_t(0)
    return capi.lib().lbm_buffer_sizes(ctypes.byref(cfg), ctypes.byref(f), ctypes.byref(w)), f.value, w.value


@pytest.mark.parametrize("kw,code", [
    (dict(tau=0.5), capi.LBM_EINVAL),
    (dict(tau=float("nan")), capi.LBM_EINVAL),
    (dict(shape=(0, 4, 4)), capi.LBM_EINVAL),
    (dict(shape=(1, 65536, 32768)), capi.LBM_EINVAL),  # ny*nz must stay below 2^31
    (dict(storage=7), capi.LBM_EINVAL),
    (dict(scheme=5), capi.LBM_EINVAL),
    (dict(faces=(capi.LBM_WALL, capi.LBM_PERIODIC, 0, 0, 0, 0)), capi.LBM_EINVAL),
    (dict(faces=(capi.LBM_MOVING_WALL, capi.LBM_MOVING_WALL, 0, 0, 0, 0)), capi.LBM_EINVAL),
    (dict(faces=(3, 3, 0, 0, 0, 0)), capi.LBM_EINVAL),
    (dict(variant=99), capi.LBM_EUNSUPPORTED),
    # rounds across a periodic y seam: a last tile row thinner than the halo for
    # every tile height built (16, 32 and 12 rows: 1057 = 66 x 16 + 1 = 33 x 32 + 1
    # = 88 x 12 + 1)
    (dict(shape=(64, 1057, 1024)), capi.LBM_EUNSUPPORTED),
    # the same with odd nz (plain layout only)
    (dict(shape=(64, 1057, 1023)), capi.LBM_EUNSUPPORTED),
    # FP64 across a periodic y seam: a last tile row thinner than the halo for both
    # tile heights built (121 = 12 x 10 + 1 = 10 x 12 + 1)
    (dict(shape=(64, 121, 1024), storage=capi.LBM_F64), capi.LBM_EUNSUPPORTED),
])
def test_invalid_configs_are_rejected(kw, code):
    assert _status(_cfg(**kw))[0] == code


def test_buffer_sizes():
    for storage, s in ((capi.LBM_F64, 8), (capi.LBM_F32, 4), (capi.LBM_F16_OFS, 2), (capi.LBM_BF16_OFS, 2)):
        st, fb, wb = _status(_cfg(storage=storage))
        assert st == capi.LBM_OK and fb == 19 * 32 ** 3 * s and wb > 0
        for scheme in (capi.LBM_TWO_ARRAY, capi.LBM_SWAP1, capi.LBM_SWAP2):  # a body force with every storage
            assert _status(_cfg(storage=storage, scheme=scheme, use_force=True))[0] == capi.LBM_OK
    st, fb, wb = _status(_cfg(scheme=capi.LBM_TWO_ARRAY))
    assert st == capi.LBM_OK and wb >= fb  # the plain scheme's second lattice lives in the work buffer
    st, fb, wb2 = _status(_cfg(scheme=capi.LBM_SWAP2))
    assert wb2 < fb  # single copy: the work buffer is a small fraction of the lattice
    assert _status(_cfg(shape=(512, 512, 512)))[0] == capi.LBM_OK


def test_planes_of_4_gib_per_direction_are_rejected():
    # in-plane byte offsets are 32-bit: a direction's y-z plane must stay below 4 GiB
    assert _status(_cfg(shape=(1, 65536, 16384)))[0] == capi.LBM_EUNSUPPORTED           # FP32, 2^32 bytes
    assert _status(_cfg(shape=(1, 32768, 16384), storage=capi.LBM_F64))[0] == capi.LBM_EUNSUPPORTED
    assert _status(_cfg(shape=(1, 65536, 16384), storage=capi.LBM_BF16_OFS))[0] == capi.LBM_OK  # 2 GiB
    assert _status(_cfg(shape=(1, 32768, 16384)))[0] == capi.LBM_OK                     # FP32, 2 GiB


def test_variant_values_per_storage():
    # variant 5 (16 x 16 plain tiles) is built for the 32- and 16-bit
    # storages; FP64 has variants 0-2 only
    for storage in (capi.LBM_F32, capi.LBM_F16_OFS, capi.LBM_BF16_OFS):
        assert _status(_cfg(shape=(128, 64, 64), storage=storage, variant=5))[0] == capi.LBM_OK, storage
    for v in (0, 1, 2):
        assert _status(_cfg(shape=(128, 64, 64), storage=capi.LBM_F64, variant=v))[0] == capi.LBM_OK, v
    assert _status(_cfg(shape=(128, 64, 64), storage=capi.LBM_F64, variant=5))[0] == capi.LBM_EUNSUPPORTED
    assert _status(_cfg(shape=(128, 64, 64), variant=6))[0] == capi.LBM_OK  # 12 x 28 plain tiles
    assert _status(_cfg(shape=(128, 64, 64), variant=7))[0] == capi.LBM_EUNSUPPORTED


def test_d3q27_fp64_rounds_across_a_periodic_seam():
    # D3Q27 in FP64 tiles 8 rows high (8 x 32, 8 x 24); across a periodic y
    # seam in rounds a last row of one would be thinner than the halo, so the
    # planner takes the 10-row tile (10 x 26): 257 rows run, 281 (= 35 x 8 + 1
    # = 28 x 10 + 1) do not
    q27 = dict(storage=capi.LBM_F64, velocities=27)
    assert _status(_cfg(shape=(32, 257, 256), **q27))[0] == capi.LBM_OK
    assert _status(_cfg(shape=(32, 281, 256), **q27))[0] == capi.LBM_EUNSUPPORTED
    assert _status(_cfg(shape=(32, 257, 256), variant=2, **q27))[0] == capi.LBM_OK
    assert _status(_cfg(shape=(32, 257, 256), variant=3, **q27))[0] == capi.LBM_EUNSUPPORTED


def test_rounds_plan_for_large_planes():
    # 1024^2 planes need 1024 tiles of 16x64: four rounds of 256 tile rows' bands;
    # the work buffer holds 2 M boundary rows of every band for all x
    nx = 64
    st, fb, wb = _status(_cfg(shape=(nx, 1024, 1024)))
    assert st == capi.LBM_OK
    shells = 4 * 2 * 2 * 1024 * nx * 19 * 4
    assert shells <= wb < shells + 19 * 4 * 1024 * 1024 * 4 + (1 << 24)
    # with walls in y any row count works (the last band may end in a partial tile)
    walls = (0, 0, capi.LBM_WALL, capi.LBM_WALL, 0, 0)
    assert _status(_cfg(shape=(nx, 1000, 1024), faces=walls))[0] == capi.LBM_OK
    # across a periodic y seam a ragged last tile row takes the plain layout of the same tile,
    # and one thinner than the halo another tile height (1009 = 31 x 32 + 17)
    assert _status(_cfg(shape=(nx, 1000, 1024)))[0] == capi.LBM_OK
    assert _status(_cfg(shape=(nx, 1009, 1024)))[0] == capi.LBM_OK
    # 1025 rows: 16- and 32-row tiles leave one row, the 12-row plain tile five
    assert _status(_cfg(shape=(nx, 1025, 1024)))[0] == capi.LBM_OK
    assert _status(_cfg(shape=(nx, 1025, 1023)))[0] == capi.LBM_OK
    # FP64 (plain layout, 10 x 32 tiles): 103 x 32 tiles, bands of 8 tile rows
    # (256 // 32), 13 rounds, each band's 2 M boundary rows saved, and the side
    # planes of one x segment; variant 1 (12 x 28 tiles): 86 x 37 tiles, bands
    # of 6 tile rows, 15 rounds, the last of 2 rows (74 tiles) in 3 x segments
    # of its own, whose side planes follow (and a 4 KB progress counter per
    # tile and segment of the most numerous segmentation)
    # (variant 2: the 10 x 32 tile with loads two planes ahead, the same plan)
    for variant, rounds, segs, tiles in ((0, 13, 1, 103 * 32), (1, 15, 1 + 3, 86 * 37), (2, 13, 1, 103 * 32)):
        st, fb, wb = _status(_cfg(shape=(nx, 1024, 1024), storage=capi.LBM_F64, variant=variant))
        assert st == capi.LBM_OK
        shells = rounds * 2 * 2 * 1024 * nx * 19 * 8
        side = segs * 2 * 19 * 1024 * 1024 * 8
        flags = (tiles * (segs - 1 if segs > 1 else 1) + 1) * 4096
        assert shells + side + flags <= wb < shells + side + flags + (1 << 24), (variant, wb)
    # FP64 512^3 (10 x 32 tiles): 52 x 16 tiles in bands of 16, 16, 16 and 4 tile
    # rows; the short last band marches in 4 x segments of its own (64 tiles x 4
    # = 256 workgroups), whose side planes (M planes of 19 per segment) follow
    # the other bands' one segment
    st, fb, wb = _status(_cfg(shape=(512, 512, 512), storage=capi.LBM_F64))
    assert st == capi.LBM_OK
    shells = 4 * 2 * 2 * 512 * 512 * 19 * 8
    side_one = 2 * 19 * 512 * 512 * 8
    assert shells + 5 * side_one <= wb < shells + 5 * side_one + (1 << 24), wb
    # a ragged last tile row across the periodic seam at least as thick as the halo
    assert _status(_cfg(shape=(nx, 1000, 1024), storage=capi.LBM_F64))[0] == capi.LBM_OK
    # 1009 rows: 10-row tiles leave a last row of 9; 12-row ones (variant 1) a row of
    # 1, so that variant falls back to the 10-row tiles there
    for variant in (0, 1):
        assert _status(_cfg(shape=(nx, 1009, 1024), storage=capi.LBM_F64, variant=variant))[0] == capi.LBM_OK
    # odd nz: the plain layout (16 x 64 tiles) runs the same four rounds, in every storage
    for storage, s in ((capi.LBM_F32, 4), (capi.LBM_BF16_OFS, 2), (capi.LBM_F16_OFS, 2)):
        st, fb, wb = _status(_cfg(shape=(nx, 1024, 1023), storage=storage))
        assert st == capi.LBM_OK
        shells = 4 * 2 * 2 * 1023 * nx * 19 * s
        assert shells <= wb < shells + 19 * s * 1024 * 1023 * 4 + (1 << 24)


def test_null_and_state_errors():
    L = capi.lib()
    cfg = _cfg()
    out = ctypes.c_void_p(1)
    st = L.lbm_init(ctypes.byref(cfg), None, None, None, None, None, None, ctypes.byref(out))
    assert st == capi.LBM_EINVAL and not out.value
    assert "required" in capi.lbm_last_error(None)
    st = L.lbm_init(ctypes.byref(cfg), ctypes.c_void_p(256 * 3 + 8), ctypes.c_void_p(512), None, None, None, None,
                    ctypes.byref(out))
    assert st == capi.LBM_EINVAL and "aligned" in capi.lbm_last_error(None)
    cfg_f = _cfg(use_force=True)
    st = L.lbm_init(ctypes.byref(cfg_f), ctypes.c_void_p(256), ctypes.c_void_p(512), None, None, None, None,
                    ctypes.byref(out))
    assert st == capi.LBM_EINVAL
    assert L.lbm_step(None, 1) == capi.LBM_ESTATE
    assert L.lbm_step_into(None, None, None, 2) == capi.LBM_ESTATE
    assert L.lbm_macroscopic(None, None, None, None, None) == capi.LBM_ESTATE
    assert L.lbm_step_adjoint(None, None, None, None, None, 1) == capi.LBM_ESTATE
    assert L.lbm_set_stream(None, None) == capi.LBM_ESTATE
    assert L.lbm_test_force_wait_timeout(None, 1) == capi.LBM_ESTATE
    L.lbm_destroy(None)


def test_three_merged_steps_are_built_for_fp32_only():
    assert _status(_cfg(scheme=capi.LBM_SWAP3))[0] == capi.LBM_OK
    assert _status(_cfg(scheme=capi.LBM_SWAP3, variant=1))[0] == capi.LBM_OK
    for st in (capi.LBM_F64, capi.LBM_F16_OFS, capi.LBM_BF16_OFS):
        assert _status(_cfg(scheme=capi.LBM_SWAP3, storage=st))[0] == capi.LBM_EUNSUPPORTED
    assert _status(_cfg(scheme=capi.LBM_SWAP3, variant=2))[0] == capi.LBM_OK
    assert _status(_cfg(scheme=capi.LBM_SWAP3, variant=3))[0] == capi.LBM_EUNSUPPORTED
    assert _status(_cfg(scheme=4))[0] == capi.LBM_EINVAL


def test_velocity_sets_sizes_and_limits():
    for q in (15, 19, 27):
        for storage, s in ((capi.LBM_F64, 8), (capi.LBM_F32, 4), (capi.LBM_F16_OFS, 2), (capi.LBM_BF16_OFS, 2)):
            st, fb, wb = _status(_cfg(storage=storage, velocities=q))
            assert st == capi.LBM_OK and fb == q * 32 ** 3 * s
    assert _status(_cfg(velocities=0))[1] == 19 * 32 ** 3 * 4  # 0 is D3Q19
    for q, last in ((15, 2), (27, 1)):
        # 16-bit storage: the default tiles, D3Q15's plain 16 x 64 as variant 1,
        # and 12 x 28 plain tiles (a second tile height across a periodic seam)
        assert _status(_cfg(storage=capi.LBM_F16_OFS, velocities=q, variant=last))[0] == capi.LBM_OK
        assert _status(_cfg(storage=capi.LBM_F16_OFS, velocities=q, variant=last + 1))[0] == capi.LBM_EUNSUPPORTED
        # across a periodic y seam in rounds 16-row tiles would leave one row of
        # 1025; the 12-row tiles leave five
        assert _status(_cfg(shape=(8, 1025, 1024), storage=capi.LBM_BF16_OFS, velocities=q))[0] == capi.LBM_OK
        assert _status(_cfg(scheme=capi.LBM_SWAP3, velocities=q))[0] == capi.LBM_EUNSUPPORTED
        assert _status(_cfg(velocities=q, variant=4))[0] == capi.LBM_EUNSUPPORTED
    # a plane of more tiles than co-resident workgroups runs in rounds: the
    # work buffer then holds the band boundary rows of all Q directions
    wb = {q: _status(_cfg(shape=(8, 1024, 1024), velocities=q)) for q in (15, 19, 27)}
    assert all(v[0] == capi.LBM_OK for v in wb.values())
    assert wb[15][2] < wb[19][2] < wb[27][2]
    assert _status(_cfg(velocities=20))[0] == capi.LBM_EINVAL
