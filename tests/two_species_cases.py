"""Two-species parity cases shared by the GPU tests, the float32-floor CPU
test and the script that writes tests/golden/two_species_fp32_floor.json.

Inputs only (seeded phase fields and flows); no arithmetic of the method.
"""
import numpy as np

from paper_2304_06437_amd import inputs


def sharp_state(lattice, shape, seed):
    """Three seeded spherical (circular) droplets, phi = +-1, at rest up to a
    1e-3 density and velocity noise."""
    nx, ny, nz = shape
    N = nx * ny * nz
    D = 2 if lattice == 9 else 3
    rng = np.random.default_rng(seed)
    x = np.arange(N) % nx
    y = (np.arange(N) // nx) % ny
    z = np.arange(N) // (nx * ny)
    phi = -np.ones(N)
    for _ in range(3):
        c = rng.uniform(0, 1, 3) * np.array(shape)
        R = 0.22 * min(s for s in shape if s > 1)
        d2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + ((z - c[2]) ** 2 if D == 3 else 0)
        phi[d2 <= R * R] = 1.0
    rho = 1.0 + 1e-3 * rng.uniform(-1, 1, N)
    u = 1e-3 * rng.uniform(-1, 1, (D, N))
    return rho, u, phi


def flow_state(lattice, shape):
    """The droplets of sharp_state(seed 5) in a Taylor-Green flow (u0 0.02)."""
    nx, ny, nz = shape
    _, _, phi = sharp_state(lattice, shape, 5)
    if lattice == 9:
        rho, u = inputs.taylor_green_2d(nx, ny, 0.02)
    else:
        rho, u = inputs.taylor_green_3d(nx, ny, nz, 0.02)
    return rho, u, phi


# name: (lattice, shape, tau, steps, bc, sigma, beta); fields sharp_state(seed 3)
CASES = {
    "d3q19_periodic_ragged": (19, (37, 24, 20), 1.0, 300, (0, 0, 0), 0.03, 0.7),
    "d3q19_walls_z": (19, (64, 16, 18), 0.8, 300, (0, 0, 1), 0.02, 0.6),
    "d3q19_walls_xyz": (19, (20, 14, 12), 0.9, 200, (1, 1, 1), 0.03, 0.7),
    "d3q19_two_segments": (19, (300, 6, 5), 1.0, 150, (0, 0, 0), 0.03, 0.7),
    "d2q9_periodic": (9, (96, 80, 1), 1.0, 500, (0, 0, 0), 0.03, 0.7),
    "d2q9_walls_xy": (9, (67, 45, 1), 0.7, 300, (1, 1, 0), 0.02, 0.5),
}

# name: (lattice, shape, tau, steps, sigma, beta): periodic, flow_state fields
FLOW_CASES = {
    "d3q19_tg_droplets": (19, (48, 32, 32), 0.55, 1000, 0.03, 0.7),
    "d2q9_tg_droplets": (9, (128, 96, 1), 0.8, 1000, 0.03, 0.7),
}

# species-mass conservation case: D3Q19, sharp_state(seed 9), tau 1.0,
# sigma 0.03, beta 0.7, periodic, 300 steps
CONSERVATION = (19, (48, 20, 16), 1.0, 300, 0.03, 0.7)
