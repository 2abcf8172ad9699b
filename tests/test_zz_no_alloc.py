"""lb_step_batch_noalloc (descriptor tables in the library's fixed device
array) against lb_step_batch (tables allocated per call): bit for bit, on two
calls in a row, the second with fewer and smaller simulations."""
import numpy as np
import pytest

from paper_2304_06437_amd import inputs, lb
from paper_2304_06437_amd.serving import JobSpec
from paper_2304_06437_amd.sim import Simulation, make_params

pytestmark = pytest.mark.gpu

FIRST = [
    JobSpec(0, 19, (40, 24, 20), 300, storage="f32", flow="tg"),
    JobSpec(1, 9, (96, 64, 1), 500, storage="f32", flow="channel"),
    JobSpec(2, 19, (64, 16, 12), 120, storage="f16s", flow="channel"),
    JobSpec(3, 19, (33, 17, 9), 300, storage="f32", flow="channel"),
    JobSpec(4, 27, (24, 12, 10), 77, storage="f32", flow="tg"),
    JobSpec(5, 9, (128, 32, 1), 300, storage="bf16s", flow="tg"),
    JobSpec(6, 19, (128, 8, 8), 1, storage="f32", flow="tg"),
    JobSpec(7, 19, (20, 18, 16), 0, storage="f32", flow="tg"),
]
SECOND = [
    JobSpec(10, 9, (40, 24, 1), 90, storage="f32", flow="tg"),
    JobSpec(11, 19, (16, 12, 10), 45, storage="f16s", flow="channel"),
]
TWO_SPECIES_STEPS = 60


def _stream():
    import torch

    global _S
    try:
        return _S
    except NameError:
        _S = torch.cuda.Stream()
        return _S


def _sims(specs):
    out = []
    for s in specs:
        p = make_params(lattice=s.lattice, shape=s.shape, tau=s.tau, force=s.force(), bc=s.bc(),
                        storage=s.storage)
        sim = Simulation(p)
        rho, u = s.fields()
        sim.init(rho, u)
        out.append(sim)
    return out


def _two_species_sim():
    n = 24
    rho, u, phi = inputs.droplets(n, [(8.0, 9.0, 10.0), (16.5, 15.0, 13.0)], 5.0)
    p = make_params(lattice=19, shape=(n, n, n), tau=1.0, species=2, sigma=0.03, beta=0.7)
    sim = Simulation(p)
    sim.init(rho, u, phi)
    return sim


def _run(specs, noalloc, with_two_species):
    import torch

    with torch.cuda.stream(_stream()):
        sims = _sims(specs)
        steps = [s.steps for s in specs]
        if with_two_species:
            sims.append(_two_species_sim())
            steps.append(TWO_SPECIES_STEPS)
        handles = [s.handle for s in sims]
        if noalloc:
            lb.lb_step_batch_noalloc(handles, steps)
        else:
            lb.lb_step_batch(handles, steps)
        out = [sim.moments(phi=sim.params.species == 2) for sim in sims]
        counts = [lb.lb_step_count(h) for h in handles]
        for sim in sims:
            sim.close()
    assert counts == steps
    return out


def _same(a, b, tag):
    for k in a:
        if k == "status":
            continue
        assert np.array_equal(a[k], b[k]), (tag, k)


def test_noalloc_matches_step_batch_on_two_calls():
    ref1 = _run(FIRST, noalloc=False, with_two_species=True)
    ref2 = _run(SECOND, noalloc=False, with_two_species=False)
    got1 = _run(FIRST, noalloc=True, with_two_species=True)
    got2 = _run(SECOND, noalloc=True, with_two_species=False)
    for i, (a, b) in enumerate(zip(got1, ref1)):
        _same(a, b, ("first", i))
    for i, (a, b) in enumerate(zip(got2, ref2)):
        _same(a, b, ("second", i))


def test_noalloc_rejects_bad_arguments():
    import torch

    with torch.cuda.stream(_stream()):
        sims = _sims(SECOND[:1])
        h = sims[0].handle
        with pytest.raises(lb.LbError) as e:
            lb.lb_step_batch_noalloc([h, h], [1, 1])  # duplicate
        assert e.value.status == lb.LB_EINVAL
        with pytest.raises(lb.LbError) as e:
            lb.lb_step_batch_noalloc([h], [-1])
        assert e.value.status == lb.LB_EINVAL
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            other = _sims(SECOND[1:2])
        with pytest.raises(lb.LbError) as e:
            lb.lb_step_batch_noalloc([h, other[0].handle], [1, 1])  # two streams
        assert e.value.status == lb.LB_EINVAL
        assert lb.lb_step_count(h) == 0
        lb.lb_step_batch_noalloc([h], [0])
        for s in sims + other:
            s.close()
