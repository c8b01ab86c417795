"""Pins of the oracle's lattice, equilibrium, pseudo-potential and EOS.

Each test checks the oracle against a fact fixed by the paper or by the
mathematics of the D3Q19 model (Section 2 of the paper), not against a
re-typing of the oracle's own formula.
"""
import itertools
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_velocity_set_is_d3q19(oracle_mod):
    cx, cy, cz, w = oracle_mod.lattice()
    c = np.stack([cx, cy, cz], axis=1)
    assert len({tuple(v) for v in c}) == 19
    n2 = (c * c).sum(axis=1)
    # one rest vector, the six faces and the twelve edges of the unit cube
    assert sorted(n2.tolist()) == [0] + [1] * 6 + [2] * 12
    assert np.all(np.abs(c) <= 1)


def test_direction_order_is_the_canonical_export_order(oracle_mod):
    cx, cy, cz, _ = oracle_mod.lattice()
    c = [tuple(v) for v in np.stack([cx, cy, cz], axis=1)]
    expected = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
                (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1),
                (1, 0, -1), (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
    assert c == expected
    for k in range(1, 10):
        assert c[2 * k] == tuple(-v for v in c[2 * k - 1])


def test_weight_isotropy_gives_cs2_one_third(oracle_mod):
    """Lattice tensors of D3Q19 up to fourth order (textbook isotropy)."""
    cx, cy, cz, w = oracle_mod.lattice()
    c = np.stack([cx, cy, cz], axis=1).astype(float)
    assert math.isclose(w.sum(), 1.0, abs_tol=1e-15)
    d = np.eye(3)
    for i in range(3):
        assert abs((w * c[:, i]).sum()) < 1e-16
        for j in range(3):
            assert abs((w * c[:, i] * c[:, j]).sum() - d[i, j] / 3.0) < 1e-15
            for k in range(3):
                assert abs((w * c[:, i] * c[:, j] * c[:, k]).sum()) < 1e-16
                for l in range(3):
                    t4 = (w * c[:, i] * c[:, j] * c[:, k] * c[:, l]).sum()
                    iso = (d[i, j] * d[k, l] + d[i, k] * d[j, l] + d[i, l] * d[j, k]) / 9.0
                    assert abs(t4 - iso) < 1e-15


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments(oracle_mod, seed):
    """sum feq = rho, sum c feq = rho u, sum c c feq = rho/3 I + rho u u."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.05, 2.7)
    u = rng.uniform(-0.15, 0.15, 3)
    cx, cy, cz, _ = oracle_mod.lattice()
    c = np.stack([cx, cy, cz], axis=1).astype(float)
    fe = oracle_mod.feq(rho, u)
    assert abs(fe.sum() - rho) < 1e-14 * rho
    assert np.allclose(c.T @ fe, rho * u, atol=1e-15, rtol=0)
    second = np.einsum("a,ai,aj->ij", fe, c, c)
    assert np.allclose(second, rho / 3.0 * np.eye(3) + rho * np.outer(u, u), atol=1e-14, rtol=0)


def test_equilibrium_at_rest_is_weighted_density(oracle_mod):
    _, _, _, w = oracle_mod.lattice()
    fe = oracle_mod.feq(1.7, (0.0, 0.0, 0.0))
    assert np.array_equal(fe, w * 1.7)


def test_pseudopotential_limits(oracle_mod):
    """psi(0) = 0, psi'(0) = 1, psi -> rho0 as rho -> infinity, monotone."""
    assert oracle_mod.psi(0.0) == 0.0
    h = 1e-6
    assert abs(oracle_mod.psi(h) / h - 1.0) < 1e-5
    assert abs(oracle_mod.psi(60.0) - 1.0) < 1e-15
    assert abs(oracle_mod.psi(60.0, rho0=2.0) - 2.0) < 1e-12
    xs = np.linspace(0, 5, 101)
    ps = [oracle_mod.psi(x) for x in xs]
    assert all(b > a for a, b in zip(ps, ps[1:]))


def test_eos_critical_point(oracle_mod):
    """Eq. (7) with psi = 1 - exp(-rho): P' = P'' = 0 at G = -4, rho = ln 2.

    Closed form: P'(rho) = (1 + G psi (1 - psi))/3 vanishes with P'' at
    psi = 1/2 when G = -4.  Checked by finite differences of the oracle's P.
    """
    rc, h = math.log(2.0), 1e-4
    P = lambda r, G: oracle_mod.pressure(r, G)
    d1 = (P(rc + h, -4.0) - P(rc - h, -4.0)) / (2 * h)
    d2 = (P(rc + h, -4.0) - 2 * P(rc, -4.0) + P(rc - h, -4.0)) / h ** 2
    assert abs(d1) < 1e-8 and abs(d2) < 1e-6
    # supercritical attraction gives a van der Waals loop, subcritical none
    xs = np.linspace(0.01, 4, 400)
    dp = np.diff([P(x, -5.5) for x in xs])
    assert (dp < 0).any()
    dp = np.diff([P(x, -3.5) for x in xs])
    assert (dp > 0).all()
    # ideal-gas limit
    assert P(1.3, 0.0) == pytest.approx(1.3 / 3.0, rel=1e-15)


def test_splitmix64_reference_vector(oracle_mod):
    vals = [int(line) for line in open(os.path.join(GOLDEN, "splitmix64.txt"))
            if line.strip() and not line.startswith("#")]
    seed, expected = vals[0], vals[1:]
    gamma = 0x9E3779B97F4A7C15
    got = [oracle_mod.splitmix64((seed + k * gamma) % 2 ** 64) for k in range(len(expected))]
    assert got == expected


def test_uniform_in_unit_interval(oracle_mod):
    us = np.array([oracle_mod.uniform(7, i) for i in range(4000)])
    assert us.min() >= 0.0 and us.max() < 1.0
    assert abs(us.mean() - 0.5) < 0.02
    assert oracle_mod.uniform(0, 0) == (oracle_mod.splitmix64(0) >> 11) / 2.0 ** 53
