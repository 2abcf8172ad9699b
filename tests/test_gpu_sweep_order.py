"""The stream-collide sweep does not depend on the order its wavefronts run
in (the thread-safety claim of Section 3): every wavefront reads only
moments, which the sweep never writes, and writes populations no other
wavefront writes.  Reversing the wavefront-to-row-segment map, or striding
it so that neighbouring wavefronts take distant rows, must give the same
bits as the natural order, for every lattice, boundary and storage mode."""
import numpy as np
import pytest

from paper_2304_06437_amd import inputs, lb
from paper_2304_06437_amd.sim import Simulation, make_params

pytestmark = pytest.mark.gpu

CASES = {
    "d3q19_walls_force": dict(lattice=19, shape=(97, 20, 18), bc=(0, 0, 1), force=(1e-5, 0, 0)),
    "d3q27_o3_xwalls_f16": dict(lattice=27, shape=(70, 14, 12), bc=(1, 0, 0), order=3,
                                storage="f16s"),
    "d2q9_cavity": dict(lattice=9, shape=(257, 130, 1), bc=(1, 1, 0),
                        wall_velocity=[[[0] * 3] * 2, [[0] * 3, [0.05, 0, 0]], [[0] * 3] * 2]),
    "d3q19_bf16_ragged": dict(lattice=19, shape=(131, 9, 7), storage="bf16s"),
    "d3q19_f64": dict(lattice=19, shape=(40, 17, 9), storage="f64", bc=(1, 1, 1)),
    "two_species": dict(lattice=19, shape=(72, 20, 16), species=2, sigma=0.03, beta=0.7,
                        tau=1.0),
    "two_species_nci": dict(lattice=9, shape=(96, 48, 1), species=2, sigma=0.03, beta=0.7,
                            tau=1.0, nci_strength=0.1, nci_eps=0.3, nci_reach=2),
}


def _run(case, order, steps=60):
    kw = dict(CASES[case])
    p = make_params(**kw)
    with Simulation(p) as sim:
        N, D = sim.N, sim.D
        rho, u = inputs.random_state(N, D, seed=7, drho=1e-3, du=0.03)
        phi = None
        if p.species == 2:
            phi = np.where(np.random.default_rng(3).uniform(size=N) > 0.6, 1.0, -1.0)
        sim.init(rho, u, phi)
        lb.lb_set_sweep_order(sim.handle, order)
        sim.step(steps)
        return sim.moments(phi=p.species == 2)


@pytest.mark.parametrize("case", sorted(CASES))
def test_result_is_independent_of_wavefront_order(case):
    ref = _run(case, 0)
    for order in (1, 2):
        got = _run(case, order)
        for k in ("rho", "u", "pineq") + (("phi",) if "phi" in ref else ()):
            assert np.array_equal(got[k], ref[k]), (case, order, k)


def test_order_values_checked():
    p = make_params(lattice=19, shape=(16, 8, 8))
    with Simulation(p) as sim:
        for bad in (-1, 3):
            with pytest.raises(lb.LbError):
                lb.lb_set_sweep_order(sim.handle, bad)
