"""Post-processing of ligament runs: break-up time, droplets, capillary scales.

Host-side analysis of what the GPU library produces (neck-density series from
the diagnostics ring, density fields exported by ``lbm_get_fields``); it does
not take part in the update itself.

* Break-up (the paper's Section 3 asks for the break-up time but does not say
  how it is detected): the ligament is taken as broken at the first time the
  neck density -- the minimum over the axis of the maximum density in the
  cross-section -- falls below rho_mid = (rho_l + rho_v)/2, interpolated
  linearly between samples.
* Droplets: 6-connected components of {rho > rho_mid} on the periodic grid,
  satellites included (Fig. 2 of the paper shows satellite droplets).
* Capillary time and Ohnesorge number, Eq. (8), with the square root the
  printed formula lacks: t_cap = sqrt(rho_l R^3 / sigma),
  Oh = nu sqrt(rho_l / (sigma R)), nu = (tau - 1/2)/3.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def breakup_time(steps, neck, rho_mid: float):
    """First crossing of neck < rho_mid, linearly interpolated; None if none."""
    steps = np.asarray(steps, dtype=np.float64)
    neck = np.asarray(neck, dtype=np.float64)
    below = np.nonzero(neck < rho_mid)[0]
    if below.size == 0:
        return None
    k = int(below[0])
    if k == 0:
        return float(steps[0])
    t0, t1, n0, n1 = steps[k - 1], steps[k], neck[k - 1], neck[k]
    return float(t0 + (n0 - rho_mid) / (n0 - n1) * (t1 - t0))


@dataclass
class Droplets:
    count: int
    volumes: np.ndarray  # nodes per droplet, largest first
    masses: np.ndarray   # sum of rho per droplet, same order


def droplets(rho, rho_mid: float) -> Droplets:
    """6-connected components of rho > rho_mid with periodic wrap in x, y, z."""
    from scipy import ndimage

    rho = np.asarray(rho, dtype=np.float64)
    mask = rho > rho_mid
    lab, n = ndimage.label(mask)  # 6-connectivity, no wrap
    if n == 0:
        return Droplets(0, np.zeros(0, np.int64), np.zeros(0))
    parent = np.arange(n + 1)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    # merge labels that touch across each periodic face
    for axis in range(3):
        lo = np.take(lab, 0, axis=axis)
        hi = np.take(lab, lab.shape[axis] - 1, axis=axis)
        both = (lo > 0) & (hi > 0)
        for a, b in zip(lo[both].ravel(), hi[both].ravel()):
            ra, rb = find(int(a)), find(int(b))
            if ra != rb:
                parent[max(ra, rb)] = min(ra, rb)
    roots = np.array([find(i) for i in range(n + 1)])
    comp = roots[lab]
    ids, inv = np.unique(comp[mask], return_inverse=True)
    vol = np.bincount(inv)
    mass = np.bincount(inv, weights=rho[mask])
    order = np.argsort(-vol, kind="stable")
    return Droplets(len(ids), vol[order], mass[order])


def capillary_time(rho_l: float, R: float, sigma: float) -> float:
    return math.sqrt(rho_l * R ** 3 / sigma)


def ohnesorge(tau: float, rho_l: float, sigma: float, R: float) -> float:
    return (tau - 0.5) / 3.0 * math.sqrt(rho_l / (sigma * R))


def tau_for_ohnesorge(oh: float, rho_l: float, sigma: float, R: float) -> float:
    return 0.5 + 3.0 * oh * math.sqrt(sigma * R / rho_l)


def run_to_breakup(lat, rho_l: float, rho_v: float, max_steps: int, every: int = 1,
                   chunk_records: int = 2000):
    """Advance a Lattice, recording diagnostics every `every` steps in the
    device ring, until the neck density falls below rho_mid or max_steps.

    Returns (t_b or None, steps array, neck array, last diagnostics record).
    """
    rho_mid = 0.5 * (rho_l + rho_v)
    steps, neck = [], []
    lat.record_diag()
    done = 0
    last = None
    while done < max_steps:
        n = min(chunk_records, (max_steps - done + every - 1) // every)
        for _ in range(n):
            lat.step(every)
            lat.record_diag()
        done += n * every
        hist = lat.read_diag_history()
        steps += [h["step"] for h in hist]
        neck += [h["neck_rho"] for h in hist]
        last = hist[-1]
        if last["nonfinite"] or min(h["neck_rho"] for h in hist) < rho_mid:
            break
    return breakup_time(steps, neck, rho_mid), np.array(steps), np.array(neck), last


def laplace_sigma(lbm, G: float, tau: float, rho_l: float, rho_v: float,
                  radii=(10, 14, 18, 22), N: int = 80, steps: int = 8000, storage="f64",
                  width: float = 2.0, mrt: dict | None = None):
    """Surface tension from the Laplace law on quasi-2D cylinders (N x N x 1,
    periodic): fit dp = sigma / R_eq + b over several radii, with
    dp = P(rho_in) - P(rho_out) from the equation of state (Eq. 7) and R_eq
    from the liquid area.  `width` is the initial tanh interface width (a
    wider start is gentler at small tau).  ``mrt``: MRT rates, or None for
    BGK.  Runs on the GPU through the library."""
    inv_r, dps = [], []

    def pressure(r):
        psi = -math.expm1(-r)
        return r / 3.0 + G * psi * psi / 6.0

    for R in radii:
        lat = lbm.Lattice(N, N, 1, tau, G, storage=storage, mrt=mrt)
        lat.init_ligament(R0=float(R), amp_rel=0.0, wavelength=1.0, rho_l=rho_l, rho_v=rho_v,
                          width=width)
        lat.step(steps)
        rho = lat.fields()["rho"].cpu().numpy()[0]
        lat.close()
        if not np.isfinite(rho).all() or rho.min() <= 0.0:
            raise RuntimeError(f"Laplace cylinder R={R} diverged at G={G}, tau={tau}")
        rin, rout = rho[N // 2, N // 2], rho[0, 0]
        area = ((rho - rout) / (rin - rout)).sum()
        inv_r.append(1.0 / math.sqrt(area / math.pi))
        dps.append(pressure(rin) - pressure(rout))
    slope, icpt = np.polyfit(inv_r, dps, 1)
    return float(slope), float(icpt)
