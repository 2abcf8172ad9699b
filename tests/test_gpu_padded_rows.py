"""Rows whose length is not a multiple of the stream-collide sweep's vector.

Rows are stored px >= nx nodes apart (nx rounded up to the sweep's vector
chunk), so that every vector access stays aligned whatever nx is; the vector
holding a row's last node then also covers padding.  These cases pick nx so
that the row end falls inside a vector (the position tl < E - 1 in it), for
every lattice, storage type, wall kind and species count, and compare the
HIP path with the FP64 oracle at the same bars as the unpadded cases:
FP32 velocity max-relative error <= 1e-5, FP64 <= 1e-11 (two species from
random velocities: 1e-4, the colour-gradient step's own FP32 rounding
floor, and 1e-11).  Padding must never reach a lattice node: poisoning the
padding populations with NaN leaves every result bit for bit unchanged.
"""
import numpy as np
import pytest

import oracle
from paper_2304_06437_amd import inputs, lb
from paper_2304_06437_amd.sim import Simulation, make_params, max_rel

pytestmark = pytest.mark.gpu


def _walls(**faces):
    wu = np.zeros((3, 2, 3))
    for k, v in faces.items():
        wu["xyz".index(k[0]), int(k[1])] = v
    return wu


# name: (lattice, shape, storage, steps, kwargs, expected row pitch)
CASES = {
    # D3Q19 FP32, two nodes per lane, one padding node per row
    "d3q19_f32_periodic_97": (19, (97, 6, 5), "f32", 300, dict(force=(1e-5, 0, 0)), 98),
    # four nodes per lane in two chunks: the row ends in chunk 1
    "d3q19_f32_xwalls_131": (19, (131, 5, 4), "f32", 300,
                             dict(bc=(1, 0, 1), force=(0, 1e-5, 0)), 132),
    "d3q19_f32_moving_xwalls_195": (19, (195, 4, 4), "f32", 300,
                                    dict(bc=(1, 1, 0), wall_velocity=_walls(x1=(0, 0.03, -0.02),
                                                                            y0=(0.02, 0, 0.01))),
                                    196),
    "d3q19_f64_xwalls_97": (19, (97, 6, 5), "f64", 300, dict(bc=(1, 0, 0)), 98),
    # D3Q27 third order, four-node chunks, three padding nodes
    "d3q27_f32_order3_xwalls_197": (27, (197, 4, 3), "f32", 200,
                                    dict(bc=(1, 0, 1), order=3, force=(1e-5, 0, 0)), 200),
    "d3q27_f64_order3_67": (27, (67, 5, 4), "f64", 200, dict(order=3), 68),
    # D2Q9 with a moving lid and x walls; FP64 two-node chunks
    "d2q9_f32_cavity_131": (9, (131, 40, 1), "f32", 400,
                            dict(bc=(1, 1, 0), wall_velocity=_walls(y1=(0.08, 0, 0))), 132),
    "d2q9_f64_cavity_65": (9, (65, 33, 1), "f64", 400,
                           dict(bc=(1, 1, 0), wall_velocity=_walls(y1=(0.08, 0, 0))), 66),
}

# 16-bit storage: eight- and four-node chunks (reported against FP64)
CASES_16 = {
    "d3q19_f16s_161": (19, (161, 4, 3), "f16s", 200, dict(bc=(1, 0, 0)), 164),
    "d2q9_bf16s_300": (9, (300, 20, 1), "bf16s", 200, dict(), 304),
    "d3q27_f16s_order3_199": (27, (199, 3, 3), "f16s", 100, dict(order=3, bc=(1, 0, 0)), 200),
}

# two species (colour gradient): chunks of two (FP32 and FP64) and four nodes
CASES_2 = {
    "two_species_f32_99": ((99, 12, 10), "f32", 150, dict(), 100),
    "two_species_f32_xwalls_197": ((197, 6, 5), "f32", 150, dict(bc=(1, 0, 0)), 200),
    "two_species_f64_xwalls_131": ((131, 6, 5), "f64", 150, dict(bc=(1, 1, 0)), 132),
}


def _fields(lattice, shape, seed):
    N = shape[0] * shape[1] * shape[2]
    D = 2 if lattice == 9 else 3
    return inputs.random_state(N, D, seed=seed, drho=1e-3, du=0.02)


def _oracle_params(lattice, shape, kw, species=1, **extra):
    return oracle.Params(lattice=lattice, nx=shape[0], ny=shape[1], nz=shape[2],
                         tau=kw.get("tau", 0.6), bb=kw.get("bc", (0, 0, 0)),
                         order=kw.get("order", 2), force=kw.get("force", (0.0, 0.0, 0.0)),
                         wall_u=kw.get("wall_velocity", np.zeros((3, 2, 3))), species=species,
                         **extra)


def _run(p, rho, u, steps, phi=None, poison=False):
    with Simulation(p) as sim:
        sim.init(rho, u, phi)
        if poison:
            _poison_padding(sim)
        sim.step(steps)
        return sim.moments(phi=phi is not None)


def _pitch(p):
    with Simulation(p) as sim:
        return lb.lb_layout(sim.handle)[4]


def _poison_padding(sim):
    """NaN into every population of every padding node (x >= nx of a row)."""
    import torch

    pop_off, mom_off, B, npad, px = lb.lb_layout(sim.handle)
    p = sim.params
    nx, rows = p.nx, p.ny * p.nz
    assert px > nx
    NA = p.lattice * p.species  # the lattice constant is Q
    dt = {lb.LB_STORE_F32: torch.float32, lb.LB_STORE_F64: torch.float64,
          lb.LB_STORE_F16S: torch.float16, lb.LB_STORE_BF16S: torch.bfloat16}[p.storage]
    esz = torch.tensor([], dtype=dt).element_size()
    pops = sim.buffer[pop_off:pop_off + NA * npad * esz].view(dt)
    n = (np.arange(rows)[:, None] * px + np.arange(nx, px)[None, :]).reshape(-1)
    idx = ((n // B)[None, :] * (NA * B) + np.arange(NA)[:, None] * B + (n % B)[None, :]).reshape(-1)
    pops[torch.from_numpy(idx).to(pops.device)] = float("nan")
    sim.synchronize()


@pytest.mark.parametrize("name", sorted(CASES))
def test_padded_rows_against_oracle(name):
    lattice, shape, storage, steps, kw, px = CASES[name]
    p = make_params(lattice=lattice, shape=shape, storage=storage, **kw)
    assert _pitch(p) == px
    rho, u = _fields(lattice, shape, seed=11)
    got = _run(p, rho, u, steps)
    ref = oracle.simulate(_oracle_params(lattice, shape, kw), rho, u, steps)
    err = max_rel(got["u"], ref["u"])
    print(f"{name}: pitch {px}, max-rel u {err:.2e}")
    assert err <= (1e-5 if storage == "f32" else 1e-11)
    if storage == "f64":
        assert np.abs(got["rho"] - ref["rho"]).max() <= 1e-12


@pytest.mark.parametrize("name", sorted(CASES_16))
def test_padded_rows_16bit_reported(name):
    lattice, shape, storage, steps, kw, px = CASES_16[name]
    p = make_params(lattice=lattice, shape=shape, storage=storage, **kw)
    assert _pitch(p) == px
    rho, u = _fields(lattice, shape, seed=12)
    got = _run(p, rho, u, steps)
    ref = oracle.simulate(_oracle_params(lattice, shape, kw), rho, u, steps)
    err = max_rel(got["u"], ref["u"])
    print(f"{name}: pitch {px}, max-rel u {err:.2e} (reported, no bar)")
    assert err <= 0.1


def _droplet(shape, seed):
    nx, ny, nz = shape
    N = nx * ny * nz
    rho, u = inputs.random_state(N, 3, seed=seed, drho=1e-3, du=0.01)
    x = np.arange(N) % nx
    y = (np.arange(N) // nx) % ny
    z = np.arange(N) // (nx * ny)
    r = np.sqrt((x - nx / 2 + 0.3) ** 2 + (y - ny / 2 - 0.21) ** 2 + (z - nz / 2 + 0.17) ** 2)
    phi = np.tanh((min(ny, nz) * 0.35 - r) / 1.5)
    # a smooth red slab across the row end (periodic distance).  Its centre is
    # off the lattice: at a node of exact symmetry the phase gradient vanishes
    # with rho_R rho_B > 0, and the interface normal there is rounding noise
    # (FP64 takes the |G| = 0 branch, FP32 a random direction)
    d = np.abs(x - (nx - 1.37))
    d = np.minimum(d, nx - d)
    phi = np.maximum(phi, np.tanh((3.0 - d) / 1.5))
    return rho, u, np.clip(phi, -1.0, 1.0)


@pytest.mark.parametrize("name", sorted(CASES_2))
def test_padded_rows_two_species_against_oracle(name):
    shape, storage, steps, kw, px = CASES_2[name]
    kw = dict(kw, tau=1.0)
    p = make_params(lattice=19, shape=shape, storage=storage, species=2, sigma=0.03, beta=0.7,
                    **kw)
    assert _pitch(p) == px
    rho, u, phi = _droplet(shape, seed=13)
    got = _run(p, rho, u, steps, phi=phi)
    ref = oracle.simulate(_oracle_params(19, shape, kw, species=2, sigma=0.03, beta=0.7),
                          rho, u, steps, phi=phi)
    err = max_rel(got["u"], ref["u"])
    dphi = np.abs(got["phi"] - ref["phi"]).max()
    print(f"{name}: pitch {px}, max-rel u {err:.2e}, |d phi| {dphi:.2e}")
    assert err <= (1e-4 if storage == "f32" else 1e-11)
    assert dphi <= (1e-4 if storage == "f32" else 1e-12)


POISON = ["d3q19_f32_xwalls_131", "d3q19_f32_moving_xwalls_195", "d3q27_f32_order3_xwalls_197",
          "d2q9_f64_cavity_65"]


@pytest.mark.parametrize("name", POISON + ["d3q19_f16s_161", "two_species_f32_xwalls_197"])
def test_padding_never_reaches_lattice_nodes(name):
    if name in CASES:
        lattice, shape, storage, steps, kw, _ = CASES[name]
        p = make_params(lattice=lattice, shape=shape, storage=storage, **kw)
        phi = None
        rho, u = _fields(lattice, shape, seed=14)
    elif name in CASES_16:
        lattice, shape, storage, steps, kw, _ = CASES_16[name]
        p = make_params(lattice=lattice, shape=shape, storage=storage, **kw)
        phi = None
        rho, u = _fields(lattice, shape, seed=14)
    else:
        shape, storage, steps, kw, _ = CASES_2[name]
        p = make_params(lattice=19, shape=shape, storage=storage, species=2, sigma=0.03,
                        beta=0.7, tau=1.0, **kw)
        rho, u, phi = _droplet(shape, seed=14)
    clean = _run(p, rho, u, 50, phi=phi)
    dirty = _run(p, rho, u, 50, phi=phi, poison=True)
    for k in clean:
        assert np.array_equal(clean[k], dirty[k]), k
    assert np.all(np.isfinite(dirty["conserved"]))


@pytest.mark.parametrize("name", ["d3q19_f32_periodic_97", "d3q19_f32_moving_xwalls_195",
                                  "d3q19_f16s_161", "two_species_f32_99"])
def test_padding_populations_stay_zero(name):
    """The sweep stores whole vectors at a padded row end, with zeros for the
    padding: after stepping, every padding population is exactly zero."""
    import torch

    if name in CASES:
        lattice, shape, storage, _, kw, _ = CASES[name]
        p = make_params(lattice=lattice, shape=shape, storage=storage, **kw)
        rho, u = _fields(lattice, shape, seed=15)
        phi = None
    elif name in CASES_16:
        lattice, shape, storage, _, kw, _ = CASES_16[name]
        p = make_params(lattice=lattice, shape=shape, storage=storage, **kw)
        rho, u = _fields(lattice, shape, seed=15)
        phi = None
    else:
        shape, storage, _, kw, _ = CASES_2[name]
        p = make_params(lattice=19, shape=shape, storage=storage, species=2, sigma=0.03,
                        beta=0.7, tau=1.0, **kw)
        rho, u, phi = _droplet(shape, seed=15)
    with Simulation(p) as sim:
        sim.init(rho, u, phi)
        sim.step(25)
        sim.synchronize()
        pop_off, _, B, npad, px = lb.lb_layout(sim.handle)
        NA = p.lattice * p.species
        esz = 4 if storage == "f32" else 2
        raw = sim.buffer[pop_off:pop_off + NA * npad * esz].cpu().numpy()
    vals = raw.view(np.float32 if storage == "f32" else np.uint16)
    nx, rows = shape[0], shape[1] * shape[2]
    n = (np.arange(rows)[:, None] * px + np.arange(nx, px)[None, :]).reshape(-1)
    idx = (n // B)[None, :] * (NA * B) + np.arange(NA)[:, None] * B + (n % B)[None, :]
    assert np.all(vals[idx] == 0)


@pytest.mark.parametrize("shape", [(64, 6, 5), (128, 3, 4), (256, 2, 2), (67, 6, 5), (130, 3, 4)])
@pytest.mark.parametrize("storage", ["f16s", "f32"])
def test_batched_and_single_variants_agree_bitwise(shape, storage):
    """Batched launches always use the padded-row variant of the sweep; a
    single D3Q27 16-bit simulation with aligned rows uses the variant
    without it.  Both must give the same bits, padded rows or not."""
    import torch

    p = make_params(lattice=27, shape=shape, storage=storage, order=3, bc=(1, 0, 0),
                    force=(1e-5, 0, 0))
    rho, u = _fields(27, shape, seed=16)
    with Simulation(p) as sim:
        sim.init(rho, u)
        sim.step(40)
        single = sim.moments()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        sim = Simulation(p)
        sim.init(rho, u)
        b = lb.lb_batch_create(side.cuda_stream)
        lb.lb_batch_step(b, [sim.handle], [40])
        batched = sim.moments()
        lb.lb_batch_destroy(b)
        sim.close()
    for k in ("rho", "u", "pineq"):
        assert np.array_equal(single[k], batched[k]), k
