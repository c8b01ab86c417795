"""Invariants, closed forms and symmetries that pin the oracle's step.

Section 2 of the paper: Eq. (3) update, Eq. (4) moments, Eq. (5) force,
Eq. (6) velocity shift.  Every check here would fail for a plausible mistake
in the oracle: a dropped term of the equilibrium (moments, tau = 1 identity),
a wrong sign or index of a velocity (symmetries, closed-form force, zero net
force), a wrong relaxation (shear-wave decay), a wrong stream direction
(translation test against the brute-force twin with pull streaming).
"""
import math

import numpy as np
import pytest

import workloads
from oracle import ref_twin


def _rest_populations(oracle_mod, rho):
    _, _, _, w = oracle_mod.lattice()
    return w[:, None, None, None] * rho[None]


def test_uniform_state_is_a_fixed_point(oracle_mod):
    f = _rest_populations(oracle_mod, np.full((5, 4, 6), 0.731))
    g = oracle_mod.run(f, 7, 0.8, -5.5)
    # every node stays identical (no spatial structure can appear) ...
    assert np.all(g.reshape(19, -1).max(axis=1) == g.reshape(19, -1).min(axis=1))
    # ... the force and the momentum are exactly zero, and the populations
    # move only by the rounding of sum_a w_a rho
    fl = oracle_mod.fields(g, -5.5)
    assert np.all(fl["F"] == 0.0) and np.all(fl["j"] == 0.0)
    assert np.allclose(f, g, rtol=1e-14, atol=0)


def test_mass_conserved_on_ligament(oracle_mod):
    s = workloads.SMALL_FP64
    f = oracle_mod.init_ligament(s.nx, s.ny, s.nz, R0=s.R0, amp_rel=s.amp_rel,
                                 wavelength=s.wavelength, rho_l=2.3068, rho_v=0.1041)
    m0 = oracle_mod.diag(f)["mass"]
    g = oracle_mod.run(f, 300, s.tau, s.G)
    d = oracle_mod.diag(g)
    assert abs(d["mass"] - m0) / m0 < 1e-13
    assert np.all(np.abs(d["mom"]) < 1e-11)
    assert d["nonfinite"] == 0


def test_momentum_conserved_on_generic_state(oracle_mod):
    f = workloads.random_populations((6, 5, 7), seed=3, base=1.2, spread=0.3)
    p0 = oracle_mod.diag(f)["mom"]
    assert np.abs(p0).max() > 1e-3
    g = oracle_mod.run(f, 50, 0.9, -5.5)
    assert np.allclose(oracle_mod.diag(g)["mom"], p0, atol=1e-13, rtol=0)


def test_net_force_vanishes_on_periodic_domain(oracle_mod):
    rho = workloads.smooth_density((9, 11, 13), seed=5, mean=1.0, amp=0.9)
    f = _rest_populations(oracle_mod, rho)
    F = oracle_mod.fields(f, -5.5)["F"]
    scale = np.abs(F).sum()
    assert scale > 1e-2
    assert np.all(np.abs(F.sum(axis=(1, 2, 3))) < 1e-15 * scale)


@pytest.mark.parametrize("nx,eps", [(16, 0.05), (10, 0.2)])
def test_force_closed_form_on_sinusoidal_psi(oracle_mod, nx, eps):
    """psi = 0.5 + eps cos(kx): F_x = (G eps / 3) psi(x) sin(k) sin(kx), F_y = F_z = 0.

    Directions with c_x = +1 carry total weight 1/6 (one face at 1/18 and
    four edges at 1/36), so the Eq. (5) sum is (psi(x+1) - psi(x-1))/6.
    """
    G = -5.5
    k = 2 * math.pi / nx
    x = np.arange(nx)
    psi = 0.5 + eps * np.cos(k * x)
    rho_x = -np.log(1.0 - psi)
    rho = np.broadcast_to(rho_x, (3, 4, nx)).copy()
    F = oracle_mod.fields(_rest_populations(oracle_mod, rho), G)["F"]
    expect = G * eps / 3.0 * psi * math.sin(k) * np.sin(k * x)
    assert np.allclose(F[0], np.broadcast_to(expect, (3, 4, nx)), atol=1e-15, rtol=1e-13)
    assert np.all(np.abs(F[1]) < 1e-16) and np.all(np.abs(F[2]) < 1e-16)


def test_tau_one_gives_equilibrium_of_shifted_velocity(oracle_mod):
    """At tau = 1, f* = f^eq(rho, u + F/rho), streamed to x + c."""
    cx, cy, cz, _ = oracle_mod.lattice()
    f = workloads.random_populations((4, 5, 6), seed=11, base=1.0, spread=0.4)
    G = -5.5
    fl = oracle_mod.fields(f, G)
    g = oracle_mod.step(f, 1.0, G)
    for z, y, x in [(0, 0, 0), (3, 4, 5), (1, 2, 3), (2, 0, 5)]:
        r = fl["rho"][z, y, x]
        up = (fl["j"][:, z, y, x] + fl["F"][:, z, y, x]) / r
        fe = oracle_mod.feq(r, up)
        for a in range(19):
            dz, dy, dx = (z + cz[a]) % 4, (y + cy[a]) % 5, (x + cx[a]) % 6
            assert g[a, dz, dy, dx] == pytest.approx(fe[a], rel=1e-14, abs=1e-16)


def test_shear_wave_decay_without_interaction(oracle_mod):
    """G = 0 reduces to plain BGK: a shear wave decays as exp(-nu k^2 t), nu = (tau - 1/2)/3."""
    nx, tau, U, steps = 64, 0.8, 1e-3, 800
    k = 2 * math.pi / nx
    x = np.arange(nx)
    f = np.empty((19, 1, 1, nx))
    for i in range(nx):
        f[:, 0, 0, i] = oracle_mod.feq(1.0, (0.0, U * math.sin(k * i), 0.0))
    g = oracle_mod.run(f, steps, tau, 0.0)
    uy = oracle_mod.fields(g, 0.0)["u"][1, 0, 0]
    amp = 2.0 / nx * (uy * np.sin(k * x)).sum()
    rate = -math.log(amp / U) / steps
    nu = (tau - 0.5) / 3.0
    assert rate == pytest.approx(nu * k * k, rel=0.01)


def test_translation_equivariance_is_exact(oracle_mod):
    s = workloads.SMALL_FP64
    f = oracle_mod.init_ligament(16, 16, 24, R0=4.0, amp_rel=0.1, wavelength=24.0,
                                 rho_l=2.3068, rho_v=0.1041, noise_amp=1e-3, seed=9)
    shift = (5, 3, 7)  # (z, y, x)
    a = oracle_mod.run(np.roll(f, shift, axis=(1, 2, 3)), 12, 0.8, s.G)
    b = np.roll(oracle_mod.run(f, 12, 0.8, s.G), shift, axis=(1, 2, 3))
    assert np.array_equal(a, b)


def _mirror_map(oracle_mod, transform):
    cx, cy, cz, _ = oracle_mod.lattice()
    c = [tuple(v) for v in np.stack([cx, cy, cz], axis=1)]
    return [c.index(transform(v)) for v in c]


def test_reflection_and_axis_exchange_symmetry(oracle_mod):
    """Mirror x -> -x and exchange x <-> y commute with the step."""
    f = oracle_mod.init_ligament(12, 12, 10, axis=2, R0=3.0, amp_rel=0.2, wavelength=10.0,
                                 c1=5.0, c2=6.0, rho_l=2.3, rho_v=0.1, noise_amp=5e-3, seed=4)
    G, tau, n = -5.5, 0.9, 15
    ref = oracle_mod.run(f, n, tau, G)
    # mirror in x: node x -> (-x) mod nx, velocity (cx,cy,cz) -> (-cx,cy,cz)
    m = _mirror_map(oracle_mod, lambda v: (-v[0], v[1], v[2]))
    mir = lambda a: np.roll(a[m][..., ::-1], 1, axis=3)
    got = oracle_mod.run(mir(f), n, tau, G)
    assert np.allclose(got, mir(ref), rtol=1e-13, atol=1e-15)
    # exchange x and y: node (x,y) -> (y,x), velocity (cx,cy,cz) -> (cy,cx,cz)
    e = _mirror_map(oracle_mod, lambda v: (v[1], v[0], v[2]))
    ex = lambda a: np.ascontiguousarray(np.swapaxes(a[e], 2, 3))
    got = oracle_mod.run(ex(f), n, tau, G)
    assert np.allclose(got, ex(ref), rtol=1e-13, atol=1e-15)


def test_brute_force_twin_agrees(oracle_mod):
    """Independent pull-streaming pure-Python twin on a 3 x 4 x 5 grid."""
    cx, cy, cz, _ = oracle_mod.lattice()
    cvecs = np.stack([cx, cy, cz], axis=1)
    f = workloads.random_populations((5, 4, 3), seed=21, base=1.4, spread=0.5)
    G, tau = -5.5, 0.85
    state = ref_twin.from_array(f, cvecs)
    for _ in range(3):
        state = ref_twin.step(state, tau, G)
    twin = ref_twin.to_array(state, cvecs, (5, 4, 3))
    ora = oracle_mod.run(f, 3, tau, G)
    assert np.allclose(ora, twin, rtol=1e-13, atol=0)


def test_twin_velocity_set_matches_weights(oracle_mod):
    cx, cy, cz, w = oracle_mod.lattice()
    tw = dict(ref_twin.velocities())
    for a in range(19):
        assert tw[(int(cx[a]), int(cy[a]), int(cz[a]))] == w[a]


def test_ligament_initial_state(oracle_mod):
    """Section 3 set-up: rest equilibrium, tanh profile, exact mass, noise bounds."""
    _, _, _, w = oracle_mod.lattice()
    f = oracle_mod.init_ligament(20, 16, 24, R0=5.0, amp_rel=0.1, wavelength=24.0,
                                 rho_l=2.0, rho_v=0.1)
    rho = f.sum(axis=0)
    assert np.allclose(f, w[:, None, None, None] * rho[None], rtol=1e-15, atol=0)
    # axis at (10, 8): the axis node is liquid, the corner vapour
    assert rho[0, 8, 10] > 1.99 and rho[0, 0, 0] < 0.11
    # at z = 0 the radius is 5.5; at z = 12 (half a wave) it is 4.5
    assert abs(rho[0, 8, 10 + 5] - rho[12, 8, 10 + 4]) < 0.5 * abs(rho[0, 8, 15] - rho[12, 8, 15])
    assert rho[0, 8, 15] > rho[12, 8, 15]
    # interface at r = R: the midpoint density
    g = oracle_mod.init_ligament(16, 16, 8, R0=5.0, amp_rel=0.0, wavelength=8.0,
                                 rho_l=2.0, rho_v=0.1)
    assert g.sum(axis=0)[3, 8, 13] == pytest.approx(1.05, abs=1e-14)
    # noise is bounded by noise_amp and reproducible from the seed
    h = oracle_mod.init_ligament(20, 16, 24, R0=5.0, amp_rel=0.1, wavelength=24.0,
                                 rho_l=2.0, rho_v=0.1, noise_amp=1e-3, seed=5)
    d = h.sum(axis=0) - rho
    assert np.abs(d).max() <= 1e-3 * (1 + 1e-9) and np.abs(d).max() > 9e-4
    i = (3 * 16 + 2) * 20 + 7
    assert d[3, 2, 7] == pytest.approx(1e-3 * (2 * oracle_mod.uniform(5, i) - 1), abs=1e-15)


def test_droplet_labelling(oracle_mod):
    rho = np.zeros((6, 6, 6))
    rho[0, 0, 0] = rho[5, 0, 0] = 1.0      # joined across the z wrap
    rho[2, 2, 2] = rho[2, 2, 3] = 1.0      # one pair
    rho[4, 4, 4] = 1.0                     # isolated
    rho[0, 3, 3] = rho[1, 4, 4] = 1.0      # diagonal only: two components
    n, lab = oracle_mod.label(rho, 0.5)
    assert n == 5
    assert lab[0, 0, 0] == lab[5, 0, 0] != 0
    assert lab[2, 2, 2] == lab[2, 2, 3]
    assert lab[0, 3, 3] != lab[1, 4, 4]


def _flat_interface(oracle_mod, G, tau, steps, n=128):
    """A 1 x 1 x n periodic slab with liquid on [n/4, 3n/4), started from the
    oracle's coexistence densities and run for `steps` steps."""
    co = oracle_mod.coexistence(G, tau)
    z = np.arange(n, dtype=np.float64)
    rho = co.rho_v + (co.rho_l - co.rho_v) * 0.5 * (np.tanh(2 * (z - (n / 4 - 0.5)) / 4)
                                                   - np.tanh(2 * (z - (3 * n / 4 - 0.5)) / 4))
    f = _rest_populations(oracle_mod, rho.reshape(n, 1, 1))
    return oracle_mod.run(f, steps, tau, G)


@pytest.mark.parametrize("tau", [0.8, 1.3])
def test_reported_velocity_vanishes_at_a_static_interface(oracle_mod, tau):
    """The velocity the oracle reports is u = (j + F/2)/rho (Eqs. 4-6 with
    the standard Shan-Chen hydrodynamic velocity).  At a converged flat
    interface nothing moves, so the reported velocity must vanish, while the
    bare j/rho is of order 0.2 there (the pre-collision momentum lags the
    force by half of its effect).

    Measured: max|u| / max|j/rho| = 3.8e-5 (tau 0.8) and 5.7e-5 (tau 1.3),
    unchanged between 60k and 240k steps -- the discrete steady state's
    O(dx^2) residual, not round-off.  The weight c of F in (j + c F)/rho
    that best cancels the flux is 1/2 to that accuracy; a dropped 1/2
    (c = 0), the post-collision momentum (c = 1) or the shift itself
    (c = tau) would leave velocities of 0.1-0.2."""
    f = _flat_interface(oracle_mod, -5.5, tau, 60_000)
    fl = oracle_mod.fields(f, -5.5)
    j, F, rho, u = fl["j"][2, :, 0, 0], fl["F"][2, :, 0, 0], fl["rho"][:, 0, 0], fl["u"][2, :, 0, 0]
    bare = np.abs(j / rho).max()
    assert bare > 0.1
    assert np.abs(u).max() < 1e-4 * bare
    c_best = -np.dot(j, F) / np.dot(F, F)  # least-squares weight making j + c F vanish
    assert abs(c_best - 0.5) < 1e-3
    for c in (0.0, 1.0, tau):
        assert np.abs((j + c * F) / rho).max() > 0.1 * bare


def test_reported_velocity_is_the_mid_collision_momentum(oracle_mod):
    """Under the velocity shift of Eq. (6) a BGK collision changes the
    momentum by exactly F (sum_a c_a f*_a = j + omega (rho u' - j) = j + F),
    so (j + F/2) is the mean of the momenta before and after the collision.
    The post-collision momentum is read back from the next state of the
    oracle's own step (f*_a(x) = f_a(x + c_a, t + 1)), independent of the
    code that reports the velocity."""
    rho = workloads.smooth_density((6, 7, 8), seed=11, mean=1.0, amp=0.8)
    f = workloads.random_populations((6, 7, 8), seed=12, base=1.0, spread=0.2) * 19 \
        * _rest_populations(oracle_mod, rho)
    tau, G = 0.85, -5.5
    fl = oracle_mod.fields(f, G)
    g = oracle_mod.step(f, tau, G)
    cx, cy, cz, _ = oracle_mod.lattice()
    post = np.stack([np.roll(g[a], (-cz[a], -cy[a], -cx[a]), axis=(0, 1, 2)) for a in range(19)])
    jstar = np.stack([np.tensordot(c, post, axes=(0, 0)) for c in (cx, cy, cz)])
    assert np.abs(fl["F"]).max() > 1e-2
    assert np.allclose(jstar, fl["j"] + fl["F"], rtol=0, atol=1e-14)
    assert np.allclose(fl["u"] * fl["rho"], 0.5 * (fl["j"] + jstar), rtol=0, atol=1e-14)
