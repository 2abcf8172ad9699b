"""Data dependencies of the two sweeps (the thread-safety of Section 3).

The stream-collide sweep rebuilds every population from moments only, so it
never reads the population arrays it overwrites: poisoning them with NaN
between the sweeps must not change the result.  The moments sweep never
reads the moment arrays it writes.
"""
import numpy as np
import pytest

from paper_2304_06437_amd import inputs, lb
from paper_2304_06437_amd.sim import Simulation, make_params

pytestmark = pytest.mark.gpu

CASES = [
    dict(lattice=19, shape=(96, 20, 12), bc=(0, 0, 1), force=(1e-5, 0, 0), species=1),
    dict(lattice=27, shape=(40, 12, 10), bc=(1, 0, 0), force=(0, 0, 0), species=1, order=3),
    dict(lattice=9, shape=(130, 40, 1), bc=(0, 1, 0), force=(0, 1e-5, 0), species=1),
    dict(lattice=19, shape=(48, 16, 16), bc=(0, 0, 0), force=(0, 0, 0), species=2,
         sigma=0.03, beta=0.7),
]


def _setup(case, storage="f32"):
    kw = dict(case)
    species = kw.pop("species")
    p = make_params(storage=storage, species=species, **kw)
    sim = Simulation(p)
    N = sim.N
    rho, u = inputs.random_state(N, sim.D, seed=4, drho=1e-3, du=0.02)
    phi = None
    if species == 2:
        rng = np.random.default_rng(2)
        phi = np.where(rng.uniform(size=N) > 0.7, 1.0, -1.0)
    sim.init(rho, u, phi)
    return sim


def _views(sim):
    """The population region and the moment region (M arrays of npad nodes:
    drho, j, Pi^neq, and phi for two species) of the device buffer."""
    import torch

    pop_off, mom_off, _, npad, _ = lb.lb_layout(sim.handle)
    buf = sim.buffer
    esz = 4 if sim.params.storage == lb.LB_STORE_F32 else 8
    D = sim.D
    M = 1 + D + D * (D + 1) // 2 + (1 if sim.params.species == 2 else 0)
    pops = buf[pop_off:mom_off]
    moms = buf[mom_off:mom_off + M * npad * esz]
    dt = torch.float32 if esz == 4 else torch.float64
    return pops.view(dt), moms.view(dt)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_stream_collide_never_reads_populations(case):
    ref = _setup(CASES[case])
    ref.step(5)
    a = ref.moments(phi=CASES[case]["species"] == 2)
    ref.close()

    sim = _setup(CASES[case])
    sim.step(4)
    lb.lb_sweep(sim.handle, 0)
    sim.synchronize()
    pops, _ = _views(sim)
    pops.fill_(float("nan"))
    lb.lb_sweep(sim.handle, 1)
    b = sim.moments(phi=CASES[case]["species"] == 2)
    assert lb.lb_step_count(sim.handle) == 5
    sim.close()
    for k in ("rho", "u", "pineq"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("case", range(len(CASES)))
def test_moments_sweep_never_reads_moments(case):
    ref = _setup(CASES[case])
    ref.step(3)
    a = ref.moments()
    ref.close()

    sim = _setup(CASES[case])
    sim.step(2)
    sim.synchronize()
    _, moms = _views(sim)
    moms.fill_(float("nan"))
    sim.step(1)
    b = sim.moments()
    sim.close()
    for k in ("rho", "u", "pineq"):
        assert np.array_equal(a[k], b[k]), k


def test_distinct_handles_from_concurrent_host_threads():
    """The library keeps no shared mutable state: simulations driven from
    several host threads at once (each on its own stream) give bit for bit
    the results of the same runs one after another."""
    import threading

    import torch

    def one(i, case, out):
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            sim = _setup(CASES[case], storage=("f32", "f16s", "f32", "f32")[i])
            sim.step(60)
            out[i] = sim.moments(phi=CASES[case]["species"] == 2)
            sim.close()

    order = list(range(len(CASES)))
    seq = {}
    for i in order:
        one(i, i, seq)
    par = {}
    threads = [threading.Thread(target=one, args=(i, i, par)) for i in order]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert all(not t.is_alive() for t in threads)
    for i in order:
        for k in ("rho", "u", "pineq"):
            assert np.array_equal(seq[i][k], par[i][k]), (i, k)
