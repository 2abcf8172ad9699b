"""Launches with more wavefronts than one grid dimension holds.

A D2Q9 domain of one column (nx = 1) and ny = 4096 * 16385 rows has
67,112,960 row segments: the stream-collide sweep needs 2^24 + 1024 blocks of
four wavefronts, past the 2^32 work-items of one grid dimension, so its
blocks go over a 2D grid.  The initial fields repeat every 4096 rows, and
the periodic domain stays a tiling of the 4096-row domain: every node of the
long column must equal, bit for bit, its node of the short column stepped
alone (one grid row), which is itself checked against the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_2304_06437_amd.sim import Simulation, make_params, max_rel

pytestmark = pytest.mark.gpu

PERIOD = 4096
TILES = 16385
STEPS = 12


def _fields(seed=5):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 1e-3 * rng.uniform(-1, 1, PERIOD)
    u = 0.02 * rng.uniform(-1, 1, (2, PERIOD))
    return rho, u


def _run(ny, rho, u):
    p = make_params(lattice=9, shape=(1, ny, 1), tau=0.7)
    with Simulation(p) as sim:
        sim.init(rho, u)
        sim.step(STEPS)
        return sim.moments(pineq=False, conserved=False)


def test_stream_collide_grid_past_one_dimension():
    rho, u = _fields()
    small = _run(PERIOD, rho, u)
    ref = oracle.simulate(oracle.Params(lattice=9, nx=1, ny=PERIOD, nz=1, tau=0.7), rho, u,
                          STEPS)
    err = max_rel(small["u"], ref["u"])
    print(f"1 x {PERIOD} column vs oracle: max-rel u {err:.2e}")
    assert err <= 1e-5
    ny = PERIOD * TILES
    assert (ny + 3) // 4 > (1 << 24) - 1  # the sweep's blocks exceed one grid dimension
    big = _run(ny, np.tile(rho, TILES), np.tile(u, (1, TILES)))
    for t in (0, 1, TILES // 2, TILES - 1):
        sl = slice(t * PERIOD, (t + 1) * PERIOD)
        assert np.array_equal(big["rho"][sl], small["rho"]), t
        assert np.array_equal(big["u"][:, sl], small["u"]), t
    # every tile: compare all at once without a second copy of the column
    assert np.array_equal(big["u"][0].reshape(TILES, PERIOD), np.broadcast_to(
        small["u"][0], (TILES, PERIOD)))
    assert np.array_equal(big["u"][1].reshape(TILES, PERIOD), np.broadcast_to(
        small["u"][1], (TILES, PERIOD)))
