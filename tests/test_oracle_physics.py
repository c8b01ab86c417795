"""Physics pins of the oracle: coexistence, Table 1, Laplace law, Rayleigh-Plateau.

These run the oracle's step for thousands of iterations and compare what it
produces with results fixed outside it:

* the Shan-Chen mechanical-stability (equal-area) construction for the EOS of
  Eq. (7) with the psi of Section 2, solved here with scipy;
* the paper's Table 1 (Section 4), with tau fixed by Oh = 0.1 read as
  Oh = nu sqrt(rho_l / (sigma R0)) (the printed Eq. (8) lacks the square root);
* the Laplace law dp = sigma / R for quasi-2D cylinders;
* Weber's viscous long-wave dispersion relation for the Plateau-Rayleigh
  instability of a liquid cylinder (stable for kR > 1, unstable below).
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate, optimize

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def table1():
    rows = []
    for line in open(os.path.join(GOLDEN, "table1.txt")):
        if line.strip() and not line.startswith("#"):
            R0, rl, rv, sg = line.split()
            rows.append((int(R0), float(rl), float(rv), float(sg)))
    return rows


def tau_from_oh(R0, rho_l, sigma, oh=0.1):
    """Oh = nu sqrt(rho_l/(sigma R0)), nu = (tau - 1/2)/3 (lattice units)."""
    return 0.5 + 3.0 * oh * math.sqrt(sigma * R0 / rho_l)


def test_workloads_table1_matches_golden():
    """The sweep's parameters in workloads.py are the golden Table 1, with tau
    from Oh = 0.1 as read here."""
    assert [tuple(r) for r in workloads.TABLE1] == table1()
    for R0, rl, _, sg in table1():
        assert workloads.table1_tau(R0) == pytest.approx(tau_from_oh(R0, rl, sg), rel=1e-15)
        s = workloads.paper_table1(R0)
        assert (s.G, s.amp_rel, s.R0) == (-5.3, 0.1, float(R0))
        assert s.nx == s.ny == workloads.round_half_up(4 * R0)
        assert 0.69 < 2 * math.pi * R0 / s.nz < 0.71  # kR = 0.7 up to rounding of L


def sc94_construction(G):
    """Equal-area rule with weight psi'/psi^2 for P = rho/3 + G psi^2/6, psi = 1 - e^-rho."""
    psi = lambda r: 1.0 - math.exp(-r)
    dpsi = lambda r: math.exp(-r)
    P = lambda r: r / 3.0 + G * psi(r) ** 2 / 6.0

    def eqs(v):
        rv, rl = v
        area = integrate.quad(lambda r: (P(rv) - P(r)) * dpsi(r) / psi(r) ** 2, rv, rl,
                              epsabs=1e-14, epsrel=1e-13)[0]
        return [P(rl) - P(rv), area]

    rv, rl = optimize.fsolve(eqs, [0.1, 2.3], xtol=1e-14)
    return rl, rv


def test_sc94_construction_reference_values(oracle_mod):
    """The construction itself at G = -5.5 against values computed beforehand
    with a separate numpy solver (2.30752 / 0.10481), and the oracle's
    bracketing implementation against this test's fsolve one."""
    rl, rv = sc94_construction(-5.5)
    assert rl == pytest.approx(2.30752, abs=2e-5)
    assert rv == pytest.approx(0.10481, abs=2e-5)
    for G in (-4.5, -5.3, -6.0):
        a = sc94_construction(G)
        b = oracle_mod.equal_area(G)
        assert a[0] == pytest.approx(b[0], rel=1e-10) and a[1] == pytest.approx(b[1], rel=1e-9)


@pytest.mark.parametrize("G", [-5.5, -6.0])
def test_flat_interface_matches_equal_area_at_tau_one(oracle_mod, G):
    """Started away from the construction (2.1 / 0.1), the flat interface
    relaxes to within 0.1% / 1% of it."""
    rl_c, rv_c = sc94_construction(G)
    co = oracle_mod.coexistence(G, 1.0, rho_hi=2.1, rho_lo=0.1)
    assert co.residual < 1e-8
    assert co.rho_l == pytest.approx(rl_c, rel=1e-3)
    assert co.rho_v == pytest.approx(rv_c, rel=1e-2)


def test_coexistence_depends_on_tau(oracle_mod):
    """Velocity-shift forcing: coexistence moves with tau (why Table 1 varies with R0)."""
    a = oracle_mod.coexistence(-5.5, 0.8)
    b = oracle_mod.coexistence(-5.5, 1.0)
    assert a.rho_v < b.rho_v - 0.01 and a.rho_l < b.rho_l


@pytest.mark.slow
def test_table1_coexistence_densities(oracle_mod):
    for R0, rl, rv, sg in table1():
        tau = tau_from_oh(R0, rl, sg)
        co = oracle_mod.coexistence(-5.3, tau)
        assert co.residual < 1e-6, (R0, co)
        assert co.rho_l == pytest.approx(rl, rel=1e-3), (R0, co)
        assert co.rho_v == pytest.approx(rv, rel=1.5e-2), (R0, co)


def laplace_sigma(oracle_mod, G, tau, rho_l, rho_v, radii=(10, 14, 18, 22), N=80, steps=8000):
    """Surface tension from quasi-2D cylinders: fit dp = sigma / R_eq + b."""
    inv_r, dps = [], []
    for R in radii:
        f = oracle_mod.init_ligament(N, N, 1, R0=float(R), amp_rel=0.0, wavelength=1.0,
                                     rho_l=rho_l, rho_v=rho_v)
        f = oracle_mod.run(f, steps, tau, G)
        rho = f.sum(axis=0)[0]
        rin, rout = rho[N // 2, N // 2], rho[0, 0]
        area = ((rho - rout) / (rin - rout)).sum()
        inv_r.append(1.0 / math.sqrt(area / math.pi))
        dps.append(oracle_mod.pressure(rin, G) - oracle_mod.pressure(rout, G))
    slope, icpt = np.polyfit(inv_r, dps, 1)
    return slope, icpt


@pytest.mark.slow
@pytest.mark.parametrize("R0", [42, 84])
def test_table1_surface_tension_by_laplace(oracle_mod, R0):
    row = {r[0]: r for r in table1()}[R0]
    _, rl, rv, sg = row
    tau = tau_from_oh(R0, rl, sg)
    co = oracle_mod.coexistence(-5.3, tau)
    sigma, icpt = laplace_sigma(oracle_mod, -5.3, tau, co.rho_l, co.rho_v)
    assert sigma == pytest.approx(sg, rel=0.05)
    assert abs(icpt) < 2e-4


@pytest.fixture(scope="module")
def sigma_55(oracle_mod):
    co = oracle_mod.coexistence(-5.5, 1.0)
    sigma, _ = laplace_sigma(oracle_mod, -5.5, 1.0, co.rho_l, co.rho_v)
    return co, sigma


def _radius_amplitude(f, rho_l, rho_v, R):
    rho = f.sum(axis=0)
    area = ((rho - rho_v) / (rho_l - rho_v)).clip(0, None).sum(axis=(1, 2))
    r = np.sqrt(area / math.pi)
    L = r.size
    z = np.arange(L)
    return 2.0 / L * abs((r * np.exp(-2j * math.pi * z / L)).sum()) / R


def _rayleigh_run(oracle_mod, co, R, kR, amp, max_steps, every=50):
    N = workloads.round_half_up(4 * R)
    L = workloads.round_half_up(2 * math.pi * R / kR)
    f = oracle_mod.init_ligament(N, N, L, R0=float(R), amp_rel=amp, wavelength=float(L),
                                 rho_l=co.rho_l, rho_v=co.rho_v)
    mid = 0.5 * (co.rho_l + co.rho_v)
    ts, amps, broke = [], [], None
    t = 0
    while t <= max_steps:
        ts.append(t)
        amps.append(_radius_amplitude(f, co.rho_l, co.rho_v, R))
        if oracle_mod.diag(f)["neck_rho"] < mid:
            broke = t
            break
        f = oracle_mod.run(f, every, 1.0, -5.5)
        t += every
    return 2 * math.pi * R / L, np.array(ts), np.array(amps), broke


def weber_rate(x, R, sigma, rho_l, nu):
    """Weber (1931) viscous long-wave growth rate of a liquid cylinder."""
    b = 3.0 * nu * x * x / (2.0 * R * R)
    return math.sqrt(sigma * x * x * (1.0 - x * x) / (2.0 * rho_l * R ** 3) + b * b) - b


@pytest.mark.slow
def test_laplace_sigma_at_g55(sigma_55):
    co, sigma = sigma_55
    assert 0.085 < sigma < 0.10


@pytest.mark.slow
def test_rayleigh_plateau_unstable_growth_matches_weber(oracle_mod, sigma_55):
    co, sigma = sigma_55
    R = 8
    x, ts, amps, broke = _rayleigh_run(oracle_mod, co, R, 0.7, 0.02, 3000)
    assert broke is not None
    sel = (amps > 0.03) & (amps < 0.2)
    assert sel.sum() >= 6
    rate = np.polyfit(ts[sel], np.log(amps[sel]), 1)[0]
    expect = weber_rate(x, R, sigma, co.rho_l, (1.0 - 0.5) / 3.0)
    assert rate == pytest.approx(expect, rel=0.15)


@pytest.mark.slow
def test_rayleigh_plateau_short_wave_is_stable(oracle_mod, sigma_55):
    co, _ = sigma_55
    x, ts, amps, broke = _rayleigh_run(oracle_mod, co, 8, 1.2, 0.1, 1500)
    assert x > 1.0
    assert broke is None
    assert amps[-1] < 0.1 * amps[0]
