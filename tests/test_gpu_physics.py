"""Physics pins of the GPU path at sizes the oracle would take long on: the
Plateau-Rayleigh instability of a liquid cylinder against Weber's viscous
long-wave dispersion relation (the linear theory of the paper's break-up
problem), at radii 16 and 24, and the stability of a short wave.

sigma comes from the Laplace law on quasi-2D cylinders run through the
library; the growth rate is fitted to the Fourier amplitude of the radius
r(z) (from the liquid area of each cross-section) over the window where it
grows from 3% to 20% of R.  Bars: 5% at R = 16 and 3% at R = 24 (measured
+1.5% and -0.7% on MI355X; the linear theory neglects the interface width,
whose relative size shrinks as R grows, and the oracle's own run at R = 8 is
8% off); at kR = 1.2 the perturbation must decay.
"""
import math

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

G, TAU = -5.5, 1.0


@pytest.fixture(scope="module")
def lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_11792_amd import lbm as mod

    return mod


@pytest.fixture(scope="module")
def fluid(lbm):
    from paper_1904_11792_amd import analysis

    rho_l, rho_v = lbm.lbm_coexistence(G, TAU)
    sigma, _ = analysis.laplace_sigma(lbm, G, TAU, rho_l, rho_v)
    return rho_l, rho_v, sigma


def _radius_amplitude(rho, rho_l, rho_v, R):
    area = ((rho - rho_v) / (rho_l - rho_v)).clip(0, None).sum(axis=(1, 2))
    r = np.sqrt(area / math.pi)
    L = r.size
    return 2.0 / L * abs((r * np.exp(-2j * math.pi * np.arange(L) / L)).sum()) / R


def _rayleigh(lbm, fluid, R, kR, amp, max_steps, every):
    rho_l, rho_v, _ = fluid
    N = workloads.round_half_up(4 * R)
    L = workloads.round_half_up(2 * math.pi * R / kR)
    lat = lbm.Lattice(N, N, L, TAU, G, storage="f64")
    lat.init_ligament(R0=float(R), amp_rel=amp, wavelength=float(L), rho_l=rho_l, rho_v=rho_v)
    mid = 0.5 * (rho_l + rho_v)
    ts, amps, broke = [], [], None
    while lat.step_count <= max_steps:
        ts.append(lat.step_count)
        amps.append(_radius_amplitude(lat.fields()["rho"].cpu().numpy(), rho_l, rho_v, R))
        if lat.diagnostics()["neck_rho"] < mid:
            broke = lat.step_count
            break
        lat.step(every)
    lat.close()
    return 2 * math.pi * R / L, np.array(ts), np.array(amps), broke


def _weber(x, R, sigma, rho_l, nu):
    b = 3.0 * nu * x * x / (2.0 * R * R)
    return math.sqrt(sigma * x * x * (1.0 - x * x) / (2.0 * rho_l * R ** 3) + b * b) - b


@pytest.mark.parametrize("R,tol", [(16, 0.05), (24, 0.03)])
def test_growth_rate_matches_weber(lbm, fluid, R, tol):
    rho_l, _, sigma = fluid
    x, ts, amps, broke = _rayleigh(lbm, fluid, R, 0.7, 0.02, 30000, every=R * 4)
    assert broke is not None
    sel = (amps > 0.03) & (amps < 0.2)
    assert sel.sum() >= 6
    rate = np.polyfit(ts[sel], np.log(amps[sel]), 1)[0]
    expect = _weber(x, R, sigma, rho_l, (TAU - 0.5) / 3.0)
    print(f"R={R}: kR={x:.3f} growth {rate:.4e}/step, Weber {expect:.4e} ({rate / expect - 1:+.1%}), "
          f"break-up at {broke}")
    assert rate == pytest.approx(expect, rel=tol)


def test_short_wave_decays(lbm, fluid):
    x, ts, amps, broke = _rayleigh(lbm, fluid, 16, 1.2, 0.1, 4000, every=100)
    assert x > 1.0 and broke is None
    assert amps[-1] < 0.1 * amps[0]


def test_laplace_law_sphere_and_cylinder_agree(lbm, fluid):
    """Laplace law in 3-D: static droplets of radius 9 ... 15 in a periodic 64^3
    box satisfy dp = 2 sigma / R, and that sigma equals the one the quasi-2D
    cylinders give (dp = sigma / R) within 5% (measured 1.1%).  The intercept
    of the linear fit, which absorbs the higher-order curvature terms of a
    diffuse interface, stays below 5% of the smallest droplet's dp (measured
    3%)."""
    import torch

    rho_l, rho_v, sigma_cyl = fluid
    N = 64
    z, y, x = np.indices((N, N, N), dtype=np.float64)
    r = np.sqrt((x - N / 2) ** 2 + (y - N / 2) ** 2 + (z - N / 2) ** 2)
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)

    def pressure(v):
        psi = -math.expm1(-v)
        return v / 3.0 + G * psi * psi / 6.0

    inv_r, dps = [], []
    for R in (9.0, 11.0, 13.0, 15.0):
        rho = 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * np.tanh(2.0 * (r - R) / 4.0)
        lat = lbm.Lattice(N, N, N, TAU, G, storage="f64")
        lat.set_populations(torch.tensor(w[:, None, None, None] * rho[None], device="cuda"))
        lat.step(6000)
        out = lat.fields()["rho"].cpu().numpy()
        assert lat.diagnostics()["nonfinite"] == 0
        lat.close()
        rin, rout = out[N // 2, N // 2, N // 2], out[0, 0, 0]
        vol = ((out - rout) / (rin - rout)).sum()
        inv_r.append(1.0 / (3.0 * vol / (4.0 * math.pi)) ** (1.0 / 3.0))
        dps.append(pressure(rin) - pressure(rout))
    slope, icpt = np.polyfit(inv_r, dps, 1)
    print(f"sphere: 2 sigma = {slope:.5f}, sigma {slope / 2:.5f}, intercept {icpt:.2e}; "
          f"cylinders: sigma {sigma_cyl:.5f}")
    assert abs(icpt) < 0.05 * min(dps)
    assert slope / 2.0 == pytest.approx(sigma_cyl, rel=0.05)
