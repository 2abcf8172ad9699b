"""The seeded input generators (no lattice Boltzmann arithmetic in them)."""
import math

import numpy as np

from paper_2304_06437_amd import inputs


def test_splitmix64_published_first_outputs():
    # SplitMix64 seeded with 0 (Steele, Lea & Flood; Vigna's reference code):
    # the first outputs mix 1, 2, 3 times the golden-ratio increment
    x = np.array([0, 0x9E3779B97F4A7C15, (2 * 0x9E3779B97F4A7C15) & ((1 << 64) - 1)],
                 dtype=np.uint64)
    got = [int(v) for v in inputs.splitmix64(x)]
    assert got[0] == 0xE220A8397B1DCDAF
    assert got[1] == 0x6E789E6AA1B965F4
    assert got[2] == 0x06C45D188009454F


def test_counter_uniform_is_deterministic_and_uniform():
    a = inputs.counter_uniform(12345, np.arange(200000, dtype=np.uint64))
    b = inputs.counter_uniform(12345, np.arange(200000, dtype=np.uint64))
    assert np.array_equal(a, b)
    assert a.min() >= 0.0 and a.max() < 1.0
    assert abs(a.mean() - 0.5) < 0.005 and abs(a.var() - 1 / 12) < 0.002
    c = inputs.counter_uniform(54321, np.arange(200000, dtype=np.uint64))
    assert abs(np.corrcoef(a, c)[0, 1]) < 0.01


def test_taylor_green_fields_are_divergence_free():
    for n in (16, 24):
        rho, u = inputs.taylor_green_3d(n, n, n, 0.02)
        nx, ny, nz = n, n, n
        U = u.reshape(3, nz, ny, nx)
        k = [np.fft.fftfreq(m) * 2 * np.pi for m in (nz, ny, nx)]
        div = (1j * k[2][None, None, :] * np.fft.fftn(U[0]) +
               1j * k[1][None, :, None] * np.fft.fftn(U[1]) +
               1j * k[0][:, None, None] * np.fft.fftn(U[2]))
        assert np.abs(div).max() < 1e-10 * U.size
        x, y, z = 3, 5, 7
        kx, ky, kz = 2 * math.pi / nx, 2 * math.pi / ny, 2 * math.pi / nz
        n0 = x + nx * (y + ny * z)
        assert math.isclose(u[0, n0], 0.02 * math.sin(kx * x) * math.cos(ky * y) * math.cos(kz * z),
                            rel_tol=1e-12, abs_tol=1e-15)
    rho2, u2 = inputs.taylor_green_2d(32, 48, 0.01)
    U2 = u2.reshape(2, 48, 32)
    kx2 = np.fft.fftfreq(32)[None, :] * 2 * np.pi
    ky2 = np.fft.fftfreq(48)[:, None] * 2 * np.pi
    div2 = 1j * kx2 * np.fft.fft2(U2[0]) + 1j * ky2 * np.fft.fft2(U2[1])
    assert np.abs(div2).max() < 1e-10 * U2.size


def test_droplets_do_not_overlap_and_have_their_volume():
    n, R = 96, 8.0
    centres = inputs.droplet_centres(n, 12, R, gap=2.0, seed=7)
    for i in range(len(centres)):
        for j in range(i):
            d = np.abs(centres[i] - centres[j])
            d = np.minimum(d, n - d)
            assert np.sqrt((d * d).sum()) >= 2 * R + 2.0
    _, _, phi = inputs.droplets(n, centres, R)
    vol = (phi > 0).sum()
    assert abs(vol / (12 * 4 / 3 * math.pi * R ** 3) - 1.0) < 0.03


def test_ellipsoid_droplet_volume():
    n, R, d = 96, 20.0, 1.15
    _, u, phi = inputs.ellipsoid_droplet(n, (R * d, R * d, R / d ** 2))
    assert np.all(u == 0.0)
    assert abs((phi > 0).sum() / (4 / 3 * math.pi * R ** 3) - 1.0) < 0.01
