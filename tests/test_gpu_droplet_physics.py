"""Two-species droplet physics on the GPU: oscillation period and Laplace law.

An oblate droplet relaxing to a sphere oscillates in its second mode.  For a
drop in a fluid of the same density and viscosity the inviscid (Lamb)
frequency is omega*^2 = m(m-1)(m+1)(m+2) sigma / (R^3 [(m+1) + m]), i.e.
24 sigma / (5 R^3) for m = 2, and Miller & Scriven's viscous correction gives
  omega = omega* - chi sqrt(omega*)/2 + chi^2/4,
  chi = (2m+1)^2 sqrt(mu1 mu2 rho1 rho2) /
        (2 R [m rho2 + (m+1) rho1] [sqrt(mu1 rho1) + sqrt(mu2 rho2)])
      = 1.25 sqrt(nu)/R  (m = 2, equal fluids).
The two-species GPU path (D3Q19, FP32) runs the paper's own setup (360^3,
R_e 40, sigma 0.03, tau 0.55 and 0.75) with the period taken from two
subsequent peaks as in the paper, and reduced sizes where the interface
height on the vertical mid-line is fitted with a damped sinusoid: within
8 % of the Miller-Scriven value at R = 32 (diffuse-interface and
finite-resolution effects: measured 1.058 at deformation 0.08), and the gap
must shrink with resolution (R = 24 -> 40).
"""
import math

import numpy as np
import pytest
from scipy.optimize import curve_fit

from paper_2304_06437_amd import inputs, lb
from paper_2304_06437_amd.sim import Simulation, make_params

pytestmark = pytest.mark.gpu

SIGMA, BETA, TAU = 0.03, 0.7, 0.55


def miller_scriven_period(R, tau, sigma=SIGMA):
    nu = (tau - 0.5) / 3.0
    w0 = math.sqrt(24.0 * sigma / (5.0 * R ** 3))
    chi = 1.25 * math.sqrt(nu) / R
    return 2.0 * math.pi / (w0 - 0.5 * chi * math.sqrt(w0) + 0.25 * chi * chi)


def interface_history(n, R, delta, steps, every=20):
    d = 1.0 + delta
    rho, u, phi = inputs.ellipsoid_droplet(n, (R * d, R * d, R / d ** 2))
    p = make_params(lattice=19, shape=(n, n, n), tau=TAU, storage="f32", species=2,
                    sigma=SIGMA, beta=BETA)
    c, ic = (n - 1) / 2.0, n // 2
    ts, zs = [], []
    with Simulation(p) as sim:
        sim.init(rho, u, phi)
        for k in range(steps // every + 1):
            if k:
                sim.step(every)
            ph = sim.moments(rho=False, u=False, pineq=False, phi=True, conserved=False)["phi"]
            ph = ph.reshape(n, n, n)
            line = 0.5 * (ph[:, ic, ic] + ph[:, ic - 1, ic - 1])  # the axis through the centre
            up = line[ic:]
            j = int(np.nonzero(up < 0)[0][0])
            ts.append(k * every)
            zs.append(ic + j - 1 + up[j - 1] / (up[j - 1] - up[j]) - c)
    return np.array(ts, dtype=np.float64), np.array(zs)


def fitted_period(ts, zs, T0, skip=300):
    keep = ts >= skip
    t, z = ts[keep], zs[keep]

    def f(t, zi, A, g, w, ps):
        return zi + A * np.exp(-g * t) * np.cos(w * t + ps)

    best = None
    for ps0 in np.linspace(0.0, 2.0 * np.pi, 8, endpoint=False):
        try:
            p, _ = curve_fit(f, t, z, p0=[z[-len(z) // 3:].mean(), np.ptp(z) / 2, 1e-4,
                                         2 * np.pi / T0, ps0], maxfev=20000)
        except RuntimeError:
            continue
        r = float(np.sqrt(np.mean((f(t, *p) - z) ** 2)))
        if best is None or r < best[1]:
            best = (p, r)
    assert best is not None
    return 2.0 * np.pi / abs(best[0][3]), best[1]


@pytest.mark.timeout(300)
def test_second_mode_period_matches_miller_scriven():
    R = 32.0
    T_ms = miller_scriven_period(R, TAU)
    ts, zs = interface_history(160, R, 0.08, 9000)
    T, rms = fitted_period(ts, zs, T_ms)
    ratio = T / T_ms
    print(f"R 32: T_LB {T:.1f}, Miller-Scriven {T_ms:.1f}, ratio {ratio:.4f} (fit rms {rms:.3f})")
    assert rms < 0.3
    assert 0.95 <= ratio <= 1.08


@pytest.mark.timeout(300)
def test_period_converges_with_resolution():
    ratios = []
    for n, R, steps in ((128, 24.0, 6000), (200, 40.0, 11000)):
        T_ms = miller_scriven_period(R, TAU)
        ts, zs = interface_history(n, R, 0.15, steps)
        T, _ = fitted_period(ts, zs, T_ms)
        ratios.append(T / T_ms)
    print(f"T_LB / T_MS: R 24 {ratios[0]:.4f}, R 40 {ratios[1]:.4f}")
    assert abs(ratios[1] - 1.0) < abs(ratios[0] - 1.0)


def midline_history(n, R, delta, tau, steps, every=25):
    """Upper interface height on the box's vertical mid-line, read every
    `every` steps straight from the phase-field moment array (one moments
    sweep refreshes it; lb_layout gives where it lives), so that a 360^3
    run does not copy the whole field to the host each time."""
    import torch

    d = 1.0 + delta
    rho, u, phi = inputs.ellipsoid_droplet(n, (R * d, R * d, R / d ** 2))
    p = make_params(lattice=19, shape=(n, n, n), tau=tau, storage="f32", species=2,
                    sigma=SIGMA, beta=BETA)
    ic, c = n // 2, (n - 1) / 2.0
    ts, zs = [], []
    with Simulation(p) as sim:
        sim.init(rho, u, phi)
        del rho, u, phi
        _, mom_off, B, npad, px = lb.lb_layout(sim.handle)
        M1 = 11  # drho, j (3), Pi^neq (6), phi
        mom = sim.buffer[mom_off:mom_off + M1 * npad * 4].view(torch.float32)
        z = np.arange(n)
        idx = []
        for xx, yy in ((ic, ic), (ic - 1, ic - 1)):
            nn = xx + px * (yy + n * z)
            idx.append(torch.as_tensor((nn // B) * M1 * B + 10 * B + nn % B, device="cuda"))
        for k in range(steps // every + 1):
            if k:
                sim.step(every)
            lb.lb_sweep(sim.handle, 0)
            sim.synchronize()
            line = (0.5 * (mom[idx[0]].double() + mom[idx[1]].double())).cpu().numpy()
            up = line[ic:]
            j = int(np.nonzero(up < 0)[0][0])
            ts.append(k * every)
            zs.append(ic + j - 1 + up[j - 1] / (up[j - 1] - up[j]) - c)
    return np.array(ts, dtype=np.float64), np.array(zs)


def peak_spacing(ts, zs, skip=200):
    """Time between the first two maxima (above the signal's mean) of the
    sampled signal after `skip`, each refined by a parabola through three
    samples: the paper measures the period from two subsequent peaks."""
    keep = ts >= skip
    t, z = ts[keep], zs[keep]
    mid = z.mean()  # wiggles of the sampled signal near a trough are not peaks
    peaks = []
    for i in range(1, len(z) - 1):
        if z[i] > mid and z[i] > z[i - 1] and z[i] >= z[i + 1]:
            a = z[i - 1] - 2 * z[i] + z[i + 1]
            peaks.append(t[i] + (0.5 * (z[i - 1] - z[i + 1]) / a) * (t[1] - t[0]))
    assert len(peaks) >= 2, peaks
    return peaks[1] - peaks[0]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("tau,bar", [(0.55, 0.07), (0.75, 0.10)])
def test_oscillation_at_the_papers_setup(tau, bar):
    """Section 5.2's setup: a 360^3 box, equivalent radius 40, sigma 0.03,
    equal densities and viscosities (deformation 0.1, beta 0.7: readings).
    The period from two subsequent peaks of the mid-line interface against
    Miller-Scriven (measured: tau 0.55 4635 vs 4406, +5.2 %; tau 0.65 4944 vs
    4563, +8.4 %; tau 0.75 5060 vs 4669, +8.4 %; the paper prints T_LB ~ 5400
    at its "nu" 0.75).  The theory's viscous term is a first-order
    correction (11.6 % of the frequency at tau 0.75, 5.2 % at 0.55), so the
    bar is tighter where the correction is small."""
    R = 40.0
    T_ms = miller_scriven_period(R, tau)
    ts, zs = midline_history(360, R, 0.1, tau, 7800)
    T = peak_spacing(ts, zs)
    print(f"360^3 R 40 tau {tau}: T_LB {T:.1f} (peak to peak), Miller-Scriven {T_ms:.1f}, "
          f"ratio {T / T_ms:.4f}")
    assert abs(T / T_ms - 1.0) <= bar


def laplace_ratio(n, R, steps=16000, tau=1.0):
    """Static droplet of radius R in a periodic box of side n, run to rest:
    (p_in - p_out) R_eff / (2 sigma) with p = cs^2 rho averaged over the
    sphere r < R/2 (inside) and over r > 1.5 R (outside), R_eff from the
    droplet volume (phi > 0)."""
    c = (n - 1) / 2.0
    rho, u, phi = inputs.ellipsoid_droplet(n, (R, R, R))
    p = make_params(lattice=19, shape=(n, n, n), tau=tau, storage="f32", species=2,
                    sigma=SIGMA, beta=BETA)
    with Simulation(p) as sim:
        sim.init(rho, u, phi)
        sim.step(steps)
        out = sim.moments(rho=True, u=True, pineq=False, phi=True, conserved=False)
    z = np.arange(n)[:, None, None]
    y = np.arange(n)[None, :, None]
    x = np.arange(n)[None, None, :]
    r = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)
    r3 = out["rho"].reshape(n, n, n)
    dp = (r3[r < 0.5 * R].mean() - r3[r > 1.5 * R].mean()) / 3.0
    R_eff = (3.0 * (out["phi"] > 0).sum() / (4.0 * math.pi)) ** (1.0 / 3.0)
    return dp * R_eff / (2.0 * SIGMA), R_eff, np.abs(out["u"]).max()


@pytest.mark.timeout(300)
def test_laplace_law_converges_with_radius():
    """Delta p = 2 sigma / R in 3D, at rest after 16000 steps: the ratio
    approaches 1 as the droplet grows relative to the interface width
    (measured 1.037, 1.025, 1.0125, 1.006, 1.003 for R = 8, 12, 16, 24, 32;
    the oracle pins 1.07 at R = 6 and 1.04 at R = 8)."""
    res = {R: laplace_ratio(4 * R, float(R)) for R in (12, 24)}
    for R, (ratio, R_eff, umax) in res.items():
        print(f"R {R}: R_eff {R_eff:.2f}, Laplace ratio {ratio:.4f}, spurious |u| {umax:.1e}")
    assert 1.0 <= res[12][0] <= 1.05
    assert 1.0 <= res[24][0] <= 1.02
    assert res[24][0] < res[12][0]
    assert all(r[2] < 1e-3 for r in res.values())
