"""Pins of the oracle's near-contact interactions (Section 2.2).

Readings (the paper gives the mechanism, not the constants):
  - a node x is bulk (continuous phase) when phi(x) < -1 + eps;
  - sitting on a bulk node, phi is sampled at x + d c_a and x - d c_a for
    every pair of opposite lattice directions (d = nci_reach); when neither
    point is bulk, both are flagged (points beyond a wall are not sampled);
  - a flagged node y with a defined phase gradient G gets the body force
    A rho_R(y) G/|G| (along the normal, into the dispersed red phase), which
    enters the collision like the constant force.

Pins: a hand-built phase field whose flags and forces follow from the rule
alone; an isolated convex droplet, which can never have interfaces on both
sides of a bulk node; exact momentum balance over one step; NCI off is the
plain colour-gradient step bit for bit; the numpy twin (gather form of the
flag rule) agrees with the C oracle (scatter form); two droplets pushed
together coalesce without NCI and stay apart with it.
"""
import numpy as np
import pytest

import oracle
from oracle import twoarray


def _params(nx, ny, nz=1, lattice=9, **kw):
    base = dict(lattice=lattice, nx=nx, ny=ny, nz=nz, tau=1.0, species=2, sigma=0.03,
                beta=0.7, nci_strength=0.1, nci_eps=0.1, nci_reach=1)
    base.update(kw)
    return oracle.Params(**base)


def _state(p, phi, u=None):
    N = p.N
    if u is None:
        u = np.zeros((p.D, N))
    return oracle.init(p, np.ones(N), u, phi)


def test_worked_example_flags_and_forces():
    """Row y = 2 of a periodic 12 x 5 grid holds a thin red slab at x = 2
    (phi 1) with interface values 0.5 at x = 3 and x = 5 around a bulk node
    x = 4, and a second slab at x = 6; everything else is bulk (-1).

    d = 1: only the bulk node (4, 2) sees non-bulk points on both sides (the
    pair along x), so exactly (3, 2) and (5, 2) are flagged.  Rows 1 and 3
    are equal, so G is along x: at (3, 2) phi falls from 1 to -1 (force
    along -x), at (5, 2) it rises (+x), each of magnitude A rho_R =
    A (1 + 0.5)/2.  d = 2: the bulk node (4, 2) samples (2, 2) and (6, 2)
    instead, and those are the only flags."""
    nx, ny = 12, 5
    phi = -np.ones((ny, nx))
    phi[2, [2, 6]] = 1.0
    phi[2, [3, 5]] = 0.5
    A = 0.1
    p = _params(nx, ny, nci_strength=A, nci_eps=0.1, nci_reach=1)
    flags, F = oracle.nci(p, _state(p, phi.reshape(-1)))
    flags = flags.reshape(ny, nx)
    assert sorted(zip(*np.nonzero(flags))) == [(2, 3), (2, 5)]
    Fx, Fy = F[0].reshape(ny, nx), F[1].reshape(ny, nx)
    assert Fx[2, 3] == pytest.approx(-0.75 * A, rel=1e-12)
    assert Fx[2, 5] == pytest.approx(0.75 * A, rel=1e-12)
    assert np.abs(Fy).max() < 1e-15
    assert np.count_nonzero(Fx) == 2
    p2 = _params(nx, ny, nci_strength=A, nci_eps=0.1, nci_reach=2)
    flags2, _ = oracle.nci(p2, _state(p2, phi.reshape(-1)))
    assert sorted(zip(*np.nonzero(flags2.reshape(ny, nx)))) == [(2, 2), (2, 6)]


def _disc(nx, ny, cx, cy, R):
    x = np.arange(nx)[None, :]
    y = np.arange(ny)[:, None]
    return (x - cx) ** 2 + (y - cy) ** 2 <= R * R


@pytest.mark.parametrize("reach", [1, 2, 3])
def test_isolated_droplet_never_flags(reach):
    """A line through a point outside a convex droplet meets the droplet on
    one side of the point only, so no bulk node has non-bulk points on both
    sides: no flags while the droplet relaxes."""
    nx = ny = 48
    phi = np.where(_disc(nx, ny, 23.5, 23.5, 10), 1.0, -1.0).reshape(-1)
    p = _params(nx, ny, nci_strength=0.1, nci_eps=0.3, nci_reach=reach)
    f = _state(p, phi)
    for _ in range(4):
        flags, F = oracle.nci(p, f)
        assert not flags.any()
        assert not F.any()
        oracle.run(p, f, 50)


def test_isolated_sphere_never_flags():
    n = 24
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    phi = np.where((x - 11.5) ** 2 + (y - 11.5) ** 2 + (z - 11.5) ** 2 <= 36, 1.0, -1.0)
    p = _params(n, n, n, lattice=19, nci_strength=0.1, nci_eps=0.3, nci_reach=2)
    f = _state(p, phi.reshape(-1))
    for _ in range(3):
        flags, _ = oracle.nci(p, f)
        assert not flags.any()
        oracle.run(p, f, 20)


def _two_drops(nx, ny, R1, R2, gap, U):
    cy = ny / 2 - 0.5
    c1 = nx / 2 - R1 - gap / 2 - 0.5
    c2 = nx / 2 + R2 + gap / 2 - 0.5
    in1, in2 = _disc(nx, ny, c1, cy, R1), _disc(nx, ny, c2, cy, R2)
    phi = np.where(in1 | in2, 1.0, -1.0).reshape(-1)
    u = np.zeros((2, nx * ny))
    u[0] = np.where(in1.reshape(-1), U, np.where(in2.reshape(-1), -U, 0.0))
    return phi, u


def _total_momentum(p, f):
    m = oracle.moments(p, f)
    F = np.asarray(p.force[: p.D]).reshape(p.D, 1)
    return (p.rho0 * m["u"] - 0.5 * F).sum(axis=1)   # j = rho0 u - F/2


def test_momentum_gain_equals_summed_nci_force():
    """Surface tension and recolouring conserve momentum, so one step changes
    the total momentum by N F plus the summed near-contact force.  Unequal
    droplets make that sum non-zero."""
    nx, ny = 64, 40
    phi, u = _two_drops(nx, ny, 11, 7, 1.5, 0.0)
    p = _params(nx, ny, nci_strength=0.1, nci_eps=0.3, nci_reach=2, force=(2e-6, -1e-6, 0.0))
    f = _state(p, phi, u)
    flags, Fn = oracle.nci(p, f)
    assert flags.sum() > 4
    total = Fn.sum(axis=1)
    assert np.abs(total[0]) > 1e-4  # the configuration is not symmetric
    j0 = _total_momentum(p, f)
    oracle.run(p, f, 1)
    j1 = _total_momentum(p, f)
    gain = j1 - j0
    expect = total + p.N * np.asarray(p.force[:2])
    assert np.abs(gain - expect).max() < 1e-12 * max(1.0, np.abs(expect).max()), (gain, expect)


def test_nci_off_is_the_plain_step_bit_for_bit():
    nx, ny = 48, 32
    phi, u = _two_drops(nx, ny, 9, 9, 3, 0.01)
    plain = oracle.Params(lattice=9, nx=nx, ny=ny, nz=1, tau=1.0, species=2, sigma=0.03,
                          beta=0.7)
    off = _params(nx, ny, nci_strength=0.0, nci_eps=0.3, nci_reach=2)
    a = oracle.simulate(plain, np.ones(nx * ny), u, 30, phi=phi)
    b = oracle.simulate(off, np.ones(nx * ny), u, 30, phi=phi)
    for k in ("rho", "u", "pineq", "phi"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("reach", [1, 2])
def test_numpy_gather_form_matches_c_scatter_form(reach):
    nx, ny = 40, 28
    phi, u = _two_drops(nx, ny, 8, 6, 3, 0.01)
    p = _params(nx, ny, nci_strength=0.08, nci_eps=0.2, nci_reach=reach, force=(1e-5, 0.0, 0.0))
    a = oracle.simulate(p, np.ones(nx * ny), u, 30, phi=phi)
    b = twoarray.simulate(p, np.ones(nx * ny), u, 30, phi=phi)
    assert np.abs(a["u"] - b["u"]).max() < 1e-13
    assert np.abs(a["rho"] - b["rho"]).max() < 1e-13
    assert np.abs(a["phi"] - b["phi"]).max() < 1e-11


def test_nci_keeps_approaching_droplets_apart():
    """Two equal droplets moving toward each other across a 4-node gap:
    without NCI the film drains and they merge (phi at the mid-plane -> +1);
    with NCI (A 0.1, eps 0.3, d 2) the film stays (mid-plane phi < 0)."""
    nx, ny = 96, 48
    phi, u = _two_drops(nx, ny, 12, 12, 4, 0.01)
    mids = {}
    for A in (0.0, 0.1):
        p = _params(nx, ny, nci_strength=A, nci_eps=0.3, nci_reach=2)
        f = _state(p, phi, u)
        oracle.run(p, f, 600)
        ph = oracle.moments(p, f)["phi"].reshape(ny, nx)
        mids[A] = ph[:, nx // 2 - 1: nx // 2 + 1].max()
    print(mids)
    assert mids[0.0] > 0.9
    assert mids[0.1] < 0.0
