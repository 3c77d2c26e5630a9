"""CPU checks of the seeded input generators."""
import numpy as np

from paper_1904_11147_amd import workloads as W


def test_device_point_values_equal_host_point_values():
    """The torch builder of four-state Riemann point values gives the host
    builder's numbers exactly (ragged sizes, several node sets and row windows)."""
    for n, order, seed, ny, j0, nr in ((37, 3, 5, 29, 3, 11), (64, 1, 7, 64, 0, 64), (20, 2, 9, 33, 30, 3)):
        wl = W.riemann2d(n=n, order=order, seed=seed).with_(ny=ny)
        r = np.polynomial.legendre.leggauss(order + 4)[0]
        a = wl.point_values(r, j0, nr)
        b = wl.point_values_device(r, j0, nr, "cpu").numpy()
        assert a.shape == b.shape == (4, order + 4, order + 4, nr, n)
        assert np.array_equal(a, b)
    assert W.density_wave(n=8).point_values_device([0.0], 0, 1, "cpu") is None


def test_batch_composition_is_seeded():
    a = W.riemann2d_batch(count=16)
    b = W.riemann2d_batch(count=16)
    assert [(w.nx, w.order, w.seed) for w in a] == [(w.nx, w.order, w.seed) for w in b]
    assert all(64 <= w.nx <= 512 and w.nx == w.ny and w.order in (1, 2, 3) for w in a)
    assert len({w.order for w in W.riemann2d_batch(count=64)}) == 3
