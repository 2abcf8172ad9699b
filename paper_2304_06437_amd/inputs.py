"""Seeded synthetic initial fields (host, FP64).

This module holds no lattice Boltzmann arithmetic: it only produces the
macroscopic fields (density, velocity, phase field) that a simulation starts
from.  The same arrays are handed to the GPU library and to the CPU oracle.

Layout: node index n = x + nx*(y + ny*z); rho[N]; u[D, N] (SoA); phi[N].
Node coordinates are the integer indices (x = i).

Flows (shaped like the paper's validation and performance runs):
  * taylor_green_2d / taylor_green_3d: decaying vortex arrays,
  * shear_wave: a single Fourier mode of transverse velocity, optionally
    advected by a uniform stream,
  * channel_noise: fluid at rest with seeded density noise (the body-forced
    channel start),
  * droplets: non-overlapping spheres of one species in the other.
"""
from __future__ import annotations

import math

import numpy as np

_M64 = (1 << 64) - 1


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea & Flood 2014) on uint64 arrays."""
    z = (x + np.uint64(0x9E3779B97F4A7C15)) & np.uint64(_M64)
    z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & np.uint64(_M64)
    z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & np.uint64(_M64)
    return z ^ (z >> np.uint64(31))


def counter_uniform(seed: int, index: np.ndarray) -> np.ndarray:
    """Uniform [0, 1) doubles from a counter-based hash of (seed, index)."""
    with np.errstate(over="ignore"):
        key = splitmix64(np.uint64(seed) * np.uint64(0xD1B54A32D192ED03) + index.astype(np.uint64))
        h = splitmix64(key)
    return (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def _grid(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x.reshape(-1), y.reshape(-1), z.reshape(-1)


def _axis(n):
    return np.arange(n, dtype=np.float64)


def taylor_green_2d(nx: int, ny: int, u0: float, rho0: float = 1.0):
    """2D Taylor-Green vortex with its pressure field (rho = rho0 + 3 p).

    u_x = -u0 cos(kx x) sin(ky y), u_y = u0 (kx/ky) sin(kx x) cos(ky y),
    p = -(rho0 u0^2 / 4) (cos 2kx x + (kx/ky)^2 cos 2ky y).
    Built from 1D factors broadcast over the grid.
    """
    kx, ky = 2 * math.pi / nx, 2 * math.pi / ny
    x, y = _axis(nx)[None, :], _axis(ny)[:, None]
    r = kx / ky
    ux = -u0 * np.cos(kx * x) * np.sin(ky * y)
    uy = u0 * r * np.sin(kx * x) * np.cos(ky * y)
    p = -(rho0 * u0 * u0 / 4.0) * (np.cos(2 * kx * x) + r * r * np.cos(2 * ky * y))
    return (rho0 + 3.0 * p).reshape(-1), np.stack([ux.reshape(-1), uy.reshape(-1)])


def taylor_green_3d(nx: int, ny: int, nz: int, u0: float, rho0: float = 1.0):
    """3D Taylor-Green vortex (periodic cube).

    u = u0 sin kx cos ky cos kz, v = -u0 cos kx sin ky cos kz, w = 0,
    rho = rho0 + (3 u0^2 / 16)(cos 2kx + cos 2ky)(cos 2kz + 2).
    Divergence-free for nx = ny (kx = ky); on other boxes it is a smooth
    periodic test field.  Built from 1D factors broadcast over the grid.
    """
    kx, ky, kz = 2 * math.pi / nx, 2 * math.pi / ny, 2 * math.pi / nz
    x = _axis(nx)[None, None, :]
    y = _axis(ny)[None, :, None]
    z = _axis(nz)[:, None, None]
    N = nx * ny * nz
    u = np.empty((3, N))
    u[0] = (u0 * np.sin(kx * x) * np.cos(ky * y) * np.cos(kz * z)).reshape(-1)
    u[1] = (-u0 * np.cos(kx * x) * np.sin(ky * y) * np.cos(kz * z)).reshape(-1)
    u[2] = 0.0
    rho = (rho0 + (3.0 * u0 * u0 / 16.0) * (np.cos(2 * kx * x) + np.cos(2 * ky * y)) * (
        np.cos(2 * kz * z) + 2.0)).reshape(-1)
    return rho, u


def shear_wave(nx: int, ny: int, nz: int, D: int, u0: float, axis_u: int = 0,
               axis_k: int = 1, advect=(0.0, 0.0, 0.0), rho0: float = 1.0):
    """u_{axis_u} = u0 sin(k x_{axis_k}) plus a uniform stream ``advect``."""
    n = (nx, ny, nz)[axis_k]
    k = 2 * math.pi / n
    coords = _grid(nx, ny, nz)
    u = np.zeros((D, nx * ny * nz))
    for al in range(D):
        u[al] += advect[al]
    u[axis_u] += u0 * np.sin(k * coords[axis_k])
    return np.full(nx * ny * nz, rho0), u


def channel_noise(nx: int, ny: int, nz: int, D: int = 3, amplitude: float = 1e-4,
                  seed: int = 12345, rho0: float = 1.0):
    """Fluid at rest, rho = rho0 + amplitude * U[-1, 1) per node (counter hash)."""
    N = nx * ny * nz
    U = counter_uniform(seed, np.arange(N, dtype=np.uint64))
    return rho0 + amplitude * (2.0 * U - 1.0), np.zeros((D, N))


def droplet_centres(n: int, count: int, radius: float, gap: float = 2.0, seed: int = 7,
                    max_tries: int = 100000):
    """Seeded rejection sampling of sphere centres in a periodic cube of side n,
    pairwise minimum-image distance >= 2 radius + gap."""
    rng = np.random.default_rng(seed)
    centres = []
    tries = 0
    while len(centres) < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place droplets")
        c = rng.uniform(0, n, size=3)
        ok = True
        for d in centres:
            dd = np.abs(c - d)
            dd = np.minimum(dd, n - dd)
            if np.sqrt((dd * dd).sum()) < 2 * radius + gap:
                ok = False
                break
        if ok:
            centres.append(c)
    return np.array(centres)


def droplets(n: int, centres, radius: float, rho0: float = 1.0):
    """phi = +1 inside any sphere (periodic minimum image), -1 outside; rest."""
    phi = -np.ones((n, n, n))
    r = int(math.ceil(radius)) + 1
    off = np.arange(-r, r + 1)
    for c in centres:
        base = np.floor(np.asarray(c)).astype(np.int64)
        ix, iy, iz = base[0] + off, base[1] + off, base[2] + off
        dz, dy, dx = np.meshgrid(iz - c[2], iy - c[1], ix - c[0], indexing="ij")
        inside = dx * dx + dy * dy + dz * dz <= radius * radius
        zz, yy, xx = np.meshgrid(iz % n, iy % n, ix % n, indexing="ij")
        phi[zz[inside], yy[inside], xx[inside]] = 1.0
    return np.full(n ** 3, rho0), np.zeros((3, n ** 3)), phi.reshape(-1)


def random_state(N: int, D: int, seed: int, drho: float = 1e-2, du: float = 0.05,
                 rho0: float = 1.0):
    """Uniform random density and velocity fields (for small consistency tests)."""
    rng = np.random.default_rng(seed)
    return rho0 + drho * rng.uniform(-1, 1, N), du * rng.uniform(-1, 1, (D, N))


def ellipsoid_droplet(n: int, radii, centre=None, rho0: float = 1.0):
    """phi = +1 inside the ellipsoid (x/a)^2 + (y/b)^2 + (z/c)^2 <= 1 around
    `centre` (default: the middle of the periodic cube of side n), -1
    outside; fluid at rest.  An oblate droplet of equivalent radius R and
    deformation d has radii (R(1+d), R(1+d), R/(1+d)^2)."""
    c = np.full(3, (n - 1) / 2.0) if centre is None else np.asarray(centre, dtype=np.float64)
    a, b, cz = radii
    z = np.arange(n, dtype=np.float64)[:, None, None]
    y = np.arange(n, dtype=np.float64)[None, :, None]
    x = np.arange(n, dtype=np.float64)[None, None, :]
    inside = ((x - c[0]) / a) ** 2 + ((y - c[1]) / b) ** 2 + ((z - c[2]) / cz) ** 2 <= 1.0
    N = n ** 3
    return np.full(N, rho0), np.zeros((3, N)), np.where(inside, 1.0, -1.0).reshape(-1)
