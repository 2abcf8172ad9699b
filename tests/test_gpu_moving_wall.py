"""GPU parity of moving-wall bounce-back (lid-driven cavity, Section 5).

The HIP path through the C ABI against the FP64 oracle: the cavity of the
paper's validation (D2Q9, lid moving along x, walls on all four sides), 3D
boxes with several moving faces including x walls, edges and corners, and the
third-order D3Q27 path.  Bar: FP32 velocity max-relative error <= 1e-5 after
up to 1000 steps, FP64 <= 1e-11; plus the closed forms the oracle is pinned
to (Couette profile, mass conservation) checked on the GPU directly.
"""
import numpy as np
import pytest

import oracle
from paper_2304_06437_amd import inputs, lb
from paper_2304_06437_amd.sim import Simulation, make_params, max_rel, run

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
FP64_TOL = 1e-11


def _walls(**faces):
    wu = np.zeros((3, 2, 3))
    for k, v in faces.items():
        wu["xyz".index(k[0]), int(k[1])] = v
    return wu


CASES = {
    # name: (lattice, shape, tau, steps, bc, walls, order, force)
    "cavity_d2q9_re100": (9, (128, 128, 1), 0.6, 1000, (1, 1, 0),
                          dict(y1=(0.1, 0, 0)), 2, (0, 0, 0)),
    "cavity_d2q9_ragged": (9, (200, 72, 1), 0.55, 600, (1, 1, 0),
                           dict(y1=(0.08, 0, 0), x0=(0, -0.03, 0)), 2, (0, 0, 0)),
    "box_d3q19_xz_walls": (19, (130, 20, 18), 0.6, 500, (1, 0, 1),
                           dict(z1=(0.06, 0.02, 0), z0=(-0.02, 0, 0), x1=(0, 0.03, -0.02)),
                           2, (1e-6, 0, 0)),
    "box_d3q19_all_walls": (19, (64, 18, 16), 0.7, 400, (1, 1, 1),
                            dict(y1=(0.05, 0, 0.02), z0=(0.03, -0.02, 0), x0=(0, 0.02, 0.01)),
                            2, (0, 0, 0)),
    "box_d3q27_order3": (27, (70, 14, 12), 0.65, 300, (0, 1, 1),
                         dict(y0=(0.04, 0, 0.01), z1=(-0.03, 0.02, 0)), 3, (0, 0, 0)),
    # rows of 64 nodes inside one layout block (row-base addressing), moving
    # walls on every axis
    "box_d3q27_order3_rows64": (27, (64, 10, 8), 0.65, 300, (1, 1, 1),
                                dict(x0=(0, 0.02, 0.01), y1=(0.04, 0, 0.01), z0=(-0.03, 0.02, 0)),
                                3, (0, 0, 0)),
}


def _oracle(case):
    lattice, shape, tau, steps, bc, walls, order, force = CASES[case]
    p = oracle.Params(lattice=lattice, nx=shape[0], ny=shape[1], nz=shape[2], tau=tau, bb=bc,
                      order=order, force=force, wall_u=_walls(**walls))
    D = p.D
    return oracle.simulate(p, np.ones(p.N), np.zeros((D, p.N)), steps)


def _gpu(case, storage):
    lattice, shape, tau, steps, bc, walls, order, force = CASES[case]
    p = make_params(lattice=lattice, shape=shape, tau=tau, bc=bc, order=order, force=force,
                    storage=storage, wall_velocity=_walls(**walls))
    N = shape[0] * shape[1] * shape[2]
    D = 2 if lattice == 9 else 3
    return run(p, np.ones(N), np.zeros((D, N)), steps)


@pytest.mark.parametrize("case", list(CASES))
def test_moving_walls_fp32_against_oracle(case):
    ref = _oracle(case)
    got = _gpu(case, "f32")
    err = max_rel(got["u"], ref["u"])
    print(f"{case}: f32 max-rel u {err:.2e}")
    assert err <= FP32_TOL


@pytest.mark.parametrize("case", ["cavity_d2q9_ragged", "box_d3q19_all_walls", "box_d3q27_order3"])
def test_moving_walls_fp64_against_oracle(case):
    ref = _oracle(case)
    got = _gpu(case, "f64")
    err = max_rel(got["u"], ref["u"])
    print(f"{case}: f64 max-rel u {err:.2e}")
    assert err <= FP64_TOL
    assert np.abs(got["rho"] - ref["rho"]).max() <= 1e-12


@pytest.mark.parametrize("storage", ["f16s", "bf16s"])
def test_cavity_16bit_storage_reported(storage):
    case = "cavity_d2q9_re100"
    ref = _oracle(case)
    got = _gpu(case, storage)
    err = max_rel(got["u"], ref["u"])
    print(f"{case}: {storage} max-rel u {err:.2e} (reported, no bar)")
    assert err <= 0.1


def test_couette_profile_on_gpu_fp64():
    H, U, tau = 16, 0.05, 1.0
    p = make_params(lattice=9, shape=(64, H, 1), tau=tau, bc=(0, 1, 0), storage="f64",
                    wall_velocity=_walls(y1=(U, 0, 0)))
    nu = (tau - 0.5) / 3.0
    steps = int(40.0 / (nu * (np.pi / H) ** 2))
    out = run(p, np.ones(64 * H), np.zeros((2, 64 * H)), steps)
    ux = out["u"][0].reshape(H, 64)
    exact = U * (np.arange(H) + 0.5) / H
    assert np.abs(ux - exact[:, None]).max() <= 1e-12


def test_cavity_mass_conservation_fp32():
    n = 96
    p = make_params(lattice=9, shape=(n, n, 1), tau=0.6, bc=(1, 1, 0), storage="f32",
                    wall_velocity=_walls(y1=(0.1, 0, 0)))
    rho, u = inputs.random_state(n * n, 2, seed=4, drho=1e-3, du=0.01)
    with Simulation(p) as sim:
        sim.init(rho, u)
        m0 = sim.moments(rho=False, u=False, pineq=False, conserved=True)["conserved"][0]
        sim.step(2000)
        m1 = sim.moments(rho=False, u=False, pineq=False, conserved=True)["conserved"][0]
    drift = abs(m1 - m0) / (n * n)
    print(f"cavity f32 per-node mass drift over 2000 steps: {drift:.2e}")
    assert drift <= 1e-6


def test_moving_walls_batched_equals_single():
    case = "box_d3q19_xz_walls"
    lattice, shape, tau, steps, bc, walls, order, force = CASES[case]
    p = make_params(lattice=lattice, shape=shape, tau=tau, bc=bc, order=order, force=force,
                    storage="f32", wall_velocity=_walls(**walls))
    N = shape[0] * shape[1] * shape[2]
    single = run(p, np.ones(N), np.zeros((3, N)), 100)
    import torch

    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        sim = Simulation(p)
        sim.init(np.ones(N), np.zeros((3, N)))
        b = lb.lb_batch_create(side.cuda_stream)
        lb.lb_batch_step(b, [sim.handle], [100])
        got = sim.moments()
        lb.lb_batch_destroy(b)
        sim.close()
    assert np.array_equal(got["u"], single["u"])
