"""Pin of the oracle's recolouring amplitude (Section 2.1, recolouring step).

With no surface tension and the fluid at rest, the mixture stays at rest and
each colour only streams and is recoloured.  Expanding one step to second
order in the interface gradient, the red fraction obeys

    (cs2 / 2) d2(rho_R)/dx2  =  beta n K d/dx (rho_R rho_B / rho),
    K = sum_a t_a c_ax^2 / |c_a|,

whose steady solution across a flat interface is phi = tanh((x - x0) / w)
with the closed-form width

    w = cs2 / (beta K).

K is 2/9 + 4/(36 sqrt 2) for D2Q9 and 2/18 + 8/(36 sqrt 2) for D3Q19.  The
continuum form holds while w spans several nodes (beta <= 0.2 here: within
0.2 % in a run to steady state).  A factor in beta, a dropped t_a or 1/|c_a|
in the recolouring term, or a missing 1/rho (the test runs at rho = 1.5,
where rho_R rho_B and rho_R rho_B / rho differ) moves w by 10 % or more.
"""
import numpy as np
import pytest
from scipy.optimize import curve_fit

import oracle

CS2 = 1.0 / 3.0
K = {9: 2 / 9 + 4 / 36 / np.sqrt(2), 19: 2 / 18 + 8 / 36 / np.sqrt(2)}


def _steady_width(lattice, beta, rho=1.5, n=96, steps=6000):
    D = 2 if lattice == 9 else 3
    p = oracle.Params(lattice=lattice, nx=n, ny=1, nz=1, tau=1.0, species=2, sigma=0.0,
                      beta=beta)
    x = np.arange(n)
    phi = np.where((x >= n // 4) & (x < 3 * n // 4), 1.0, -1.0)
    f = oracle.init(p, np.full(n, rho), np.zeros((D, n)), phi)
    oracle.run(p, f, steps)
    m = oracle.moments(p, f)
    assert np.abs(m["u"]).max() < 1e-13  # sigma = 0: the mixture stays at rest
    prof = m["phi"]
    sel = (x > n / 8) & (x < 3 * n / 8)   # the interface at x = n/4 - 1/2
    (x0, w), _ = curve_fit(lambda xx, x0, w: np.tanh((xx - x0) / w), x[sel].astype(float),
                           prof[sel], p0=(n / 4 - 0.5, 3.0))
    return x0, w


@pytest.mark.parametrize("lattice", [9, 19])
@pytest.mark.parametrize("beta", [0.1, 0.2])
def test_flat_interface_width_is_cs2_over_beta_K(lattice, beta):
    x0, w = _steady_width(lattice, beta)
    expect = CS2 / (beta * K[lattice])
    assert abs(x0 - (96 / 4 - 0.5)) < 1e-3   # the interface does not move
    assert abs(w / expect - 1.0) < 0.005, (w, expect)
