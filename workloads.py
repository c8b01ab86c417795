"""Seeded synthetic workloads: ligament specifications and random states.

This module is the only code shared by the GPU-side tests/benchmark and the
CPU oracle.  It holds parameters and random numbers only -- none of the
method's arithmetic (no equilibrium, no pseudo-potential, no force): each
side turns a spec into populations with its own code.

Workloads (the paper's Section 3 test case: a liquid cylinder with a
cosine-perturbed radius on a periodic box; Section 4 parameters):

* ``small_fp64``      32 x 32 x 64, tau 1.0, G -5.5, R0 6, one wave along z,
                      amplitude 0.1 R0, interface width 2, no noise.
* ``large_fp32``      256 x 256 x 1024, tau 0.8, G -5.5, R0 24, wavelength
                      1024/5, amplitude 0.05 R0, noise +-1e-4 on rho, seed 1.
* ``convergence(R)``  4R x 4R x L with L = round(2 pi R / 0.7), tau 1, G -5.5,
                      amplitude 0.1 R0, no noise.
* ``batch64``         64 ligaments drawn from numpy ``default_rng(seed)``:
                      R0 ~ U[6,20], kR ~ U[0.3,0.9], tau ~ U[0.6,1.2],
                      G ~ U[-6,-5]; grid (round 4R)^2 x round(2 pi R / kR).
* ``paper_table1(R0)`` the paper's sweep (Section 4, Table 1): G = -5.3,
                      tau from Oh = 0.1, R0 in {7, 14, ..., 84}, grid as for
                      ``convergence``.

``rho_l``/``rho_v`` of None mean "the flat-interface coexistence densities at
this (G, tau)", which each side computes itself.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace

import numpy as np


@dataclass(frozen=True)
class Ligament:
    name: str
    nx: int
    ny: int
    nz: int
    tau: float
    G: float
    R0: float
    wavelength: float
    amp_rel: float
    axis: int = 2
    width: float = 2.0
    noise_amp: float = 0.0
    seed: int = 0
    rho0: float = 1.0
    rho_l: float | None = None
    rho_v: float | None = None
    steps: int = 0

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def center(self):
        plane = [(self.ny, self.nz), (self.nx, self.nz), (self.nx, self.ny)][self.axis]
        return plane[0] / 2.0, plane[1] / 2.0

    def with_densities(self, rho_l: float, rho_v: float) -> "Ligament":
        return replace(self, rho_l=rho_l, rho_v=rho_v)


def round_half_up(v: float) -> int:
    return int(math.floor(v + 0.5))


SMALL_FP64 = Ligament("small_fp64 32x32x64", 32, 32, 64, tau=1.0, G=-5.5, R0=6.0,
                      wavelength=64.0, amp_rel=0.1, steps=2000)

LARGE_FP32 = Ligament("large_fp32 256x256x1024", 256, 256, 1024, tau=0.8, G=-5.5, R0=24.0,
                      wavelength=1024.0 / 5.0, amp_rel=0.05, noise_amp=1e-4, seed=1,
                      steps=20000)


def convergence(R: int) -> Ligament:
    N = round_half_up(4 * R)
    L = round_half_up(2 * math.pi * R / 0.7)
    return Ligament(f"convergence R={R} {N}x{N}x{L}", N, N, L, tau=1.0, G=-5.5, R0=float(R),
                    wavelength=float(L), amp_rel=0.1)


def batch64(seed: int = 2024, count: int = 64) -> list[Ligament]:
    rng = np.random.default_rng(seed)
    R = rng.uniform(6.0, 20.0, count)
    kR = rng.uniform(0.3, 0.9, count)
    tau = rng.uniform(0.6, 1.2, count)
    G = rng.uniform(-6.0, -5.0, count)
    out = []
    for i in range(count):
        N = round_half_up(4 * R[i])
        L = round_half_up(2 * math.pi * R[i] / kR[i])
        out.append(Ligament(f"batch[{i}]", N, N, L, tau=float(tau[i]), G=float(G[i]),
                            R0=float(R[i]), wavelength=float(L), amp_rel=0.1, seed=i))
    return out


# The paper's Table 1 (Section 4): G0 = 5.3 (attractive, G = -5.3), Oh = 0.1.
# Rows (R0, rho_l, rho_v, sigma) as printed.
TABLE1 = (
    (7, 2.112, 0.081, 0.05159),
    (14, 2.117, 0.084, 0.05345),
    (28, 2.125, 0.090, 0.05775),
    (42, 2.135, 0.097, 0.06277),
    (56, 2.145, 0.106, 0.06848),
    (70, 2.156, 0.116, 0.07491),
    (84, 2.167, 0.126, 0.08206),
)
TABLE1_R0 = tuple(r[0] for r in TABLE1)
TABLE1_G = -5.3
TABLE1_OH = 0.1


def table1_tau(R0: int) -> float:
    """tau of a Table 1 row: Oh = nu sqrt(rho_l / (sigma R0)) = 0.1 with the
    row's printed rho_l and sigma, nu = (tau - 1/2) / 3 (Eq. (8) with the
    square root that makes it dimensionless)."""
    _, rho_l, _, sigma = {r[0]: r for r in TABLE1}[R0]
    return 0.5 + 3.0 * TABLE1_OH * math.sqrt(sigma * R0 / rho_l)


def paper_table1(R0: int) -> Ligament:
    """A ligament of the paper's sweep: G = -5.3, tau from Oh = 0.1, radius R0
    perturbed by R0/10 with one cosine wave along a z period of
    round(2 pi R0 / 0.7) (kR = 0.7, inside the unstable band), cross-section
    round(4 R0) squared, interface width 2, no noise."""
    N = round_half_up(4 * R0)
    L = round_half_up(2 * math.pi * R0 / 0.7)
    return Ligament(f"paper R0={R0} {N}x{N}x{L}", N, N, L, tau=table1_tau(R0), G=TABLE1_G,
                    R0=float(R0), wavelength=float(L), amp_rel=0.1)


def random_populations(shape, seed: int, base: float = 1.0, spread: float = 0.1,
                       q: int = 19) -> np.ndarray:
    """Arbitrary positive populations (q, nz, ny, nx): base/q * (1 + spread*(2U-1)).

    Not an equilibrium: used to exercise the update on generic states.
    """
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    u = rng.random((q, nz, ny, nx))
    return (base / q) * (1.0 + spread * (2.0 * u - 1.0))


def smooth_density(shape, seed: int, mean: float = 1.0, amp: float = 0.3, modes: int = 3):
    """A smooth periodic positive density field made of a few random Fourier modes."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    rho = np.full(shape, mean, dtype=np.float64)
    for _ in range(modes):
        kx, ky, kz = rng.integers(0, 3, 3)
        ph = rng.uniform(0, 2 * math.pi)
        a = rng.uniform(0.3, 1.0) * amp / modes
        rho += a * np.cos(2 * math.pi * (kx * x / nx + ky * y / ny + kz * z / nz) + ph)
    return rho
