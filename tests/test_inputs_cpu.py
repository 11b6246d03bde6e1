"""The seeded input generators agree with each other (host, indexed, device
forms of the Taylor-Green field), so the large-lattice tests can build the
GPU's field on the device and the oracle's on a small index box."""
import numpy as np

from paper_2208_05429_amd import workloads as wl


def test_taylor_green_generators_agree():
    shape = (8, 6, 10)
    ph = wl.random_phases(4)
    _, u = wl.taylor_green_3d(shape, 0.02, ph)
    ua = wl.taylor_green_3d_at(shape, 0.02, ph, range(8), range(6), range(10))
    ud = wl.taylor_green_3d_device(shape, 0.02, ph, "cpu").numpy()
    assert np.array_equal(u, ua)
    assert np.abs(u - ud).max() <= 1e-17
    # an index box with wrap-around picks the same values
    ix, iy, iz = [7, 0, 1], [5, 0], [9, 0, 1, 2]
    assert np.array_equal(wl.taylor_green_3d_at(shape, 0.02, ph, ix, iy, iz), u[:, ix][:, :, iy][:, :, :, iz])
