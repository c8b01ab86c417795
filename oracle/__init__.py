"""FP64 CPU oracle for the Shan-Chen D3Q19 lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_1904_11792_amd``) and never imports it.

The arithmetic lives in ``sc_oracle.c`` (plain C, FP64, OpenMP over z); this
module is a ctypes wrapper plus the slow drivers built on it:

* ``step`` / ``run``          -- Eq. (3) with the velocity shift of Eq. (6)
                                 (Section 2 of the paper); with ``mrt=`` the
                                 multiple-relaxation-time collision the
                                 paper's conclusion names (see sc_oracle.c)
* ``mrt_matrix`` / ``mrt_equilibrium`` / ``mrt_rates`` -- its ingredients
* ``fields``                  -- rho, j (Eq. 4), F (Eq. 5), physical velocity
* ``init_ligament``           -- the perturbed cylinder of Section 3 (Fig. 1)
* ``diag``                    -- mass, momentum, rho range, neck density
* ``coexistence``             -- flat-interface run to steady state
* ``label``                   -- 6-connected droplet labelling

Arrays are numpy float64 with shape (19, nz, ny, nx), C-contiguous.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sc_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
# AddressSanitizer + UndefinedBehaviorSanitizer build of the same source,
# loaded instead when ORACLE_SANITIZED=1 (the process must then preload the
# ASan runtime, see tests/test_oracle_sanitized.py)
_SO_SAN = os.path.join(_HERE, "liboracle_san.so")
_lib = None

Q = 19


def build(sanitize: bool = False) -> str:
    """Compile sc_oracle.c with gcc into oracle/liboracle.so (always rebuilds);
    with sanitize=True into oracle/liboracle_san.so, instrumented with
    AddressSanitizer and UndefinedBehaviorSanitizer (every report fatal)."""
    out = _SO_SAN if sanitize else _SO
    tmp = out + ".tmp"
    extra = (["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]
             if sanitize else [])
    cmd = ["gcc", "-O2", "-fopenmp", "-std=c11", "-Wall", "-shared", "-fPIC", *extra,
           _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def lib():
    """Load the oracle library, compiling it first if it has never been built."""
    global _lib
    if _lib is not None:
        return _lib
    sanitized = os.environ.get("ORACLE_SANITIZED") == "1"
    path = _SO_SAN if sanitized else _SO
    if not os.path.exists(path):
        build(sanitize=sanitized)
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    i32p = ctypes.POINTER(ctypes.c_int32)
    ci, cd, cl, cu64 = ctypes.c_int, ctypes.c_double, ctypes.c_long, ctypes.c_uint64
    L.orc_num_threads.argtypes = []
    L.orc_num_threads.restype = ci
    L.orc_lattice.argtypes = [ip, ip, ip, dp]
    L.orc_lattice.restype = None
    L.orc_psi.argtypes = [cd, cd]
    L.orc_psi.restype = cd
    L.orc_pressure.argtypes = [cd, cd, cd]
    L.orc_pressure.restype = cd
    L.orc_feq.argtypes = [cd, cd, cd, cd, dp]
    L.orc_feq.restype = None
    L.orc_step.argtypes = [ci, ci, ci, cd, cd, cd, dp, dp]
    L.orc_step.restype = ci
    L.orc_run.argtypes = [ci, ci, ci, cd, cd, cd, cl, dp, dp]
    L.orc_run.restype = ci
    L.orc_mrt_matrix.argtypes = [dp]
    L.orc_mrt_matrix.restype = None
    L.orc_mrt_equilibrium.argtypes = [cd, cd, cd, cd, dp]
    L.orc_mrt_equilibrium.restype = None
    L.orc_run_mrt.argtypes = [ci, ci, ci, dp, cd, cd, cl, dp, dp]
    L.orc_run_mrt.restype = ci
    L.orc_fields.argtypes = [ci, ci, ci, cd, cd, dp, dp, dp, dp, dp]
    L.orc_fields.restype = ci
    L.orc_splitmix64.argtypes = [cu64]
    L.orc_splitmix64.restype = cu64
    L.orc_uniform.argtypes = [cu64, cu64]
    L.orc_uniform.restype = cd
    L.orc_init_ligament.argtypes = [ci, ci, ci, ci, cd, cd, cd, cd, cd, cd, cd, cd, cd,
                                     cu64, dp]
    L.orc_init_ligament.restype = ci
    L.orc_diag.argtypes = [ci, ci, ci, ci, dp, dp]
    L.orc_diag.restype = ci
    L.orc_label.argtypes = [ci, ci, ci, dp, cd, i32p]
    L.orc_label.restype = cl
    _lib = L
    return L


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _shape(f: np.ndarray):
    if f.ndim != 4 or f.shape[0] != Q:
        raise ValueError("populations must have shape (19, nz, ny, nx)")
    _, nz, ny, nx = f.shape
    return nx, ny, nz


def num_threads() -> int:
    """OpenMP threads the oracle runs on."""
    return int(lib().orc_num_threads())


def lattice():
    """(cx, cy, cz, w) of the D3Q19 set in the oracle's direction order."""
    L = lib()
    cx = (ctypes.c_int * Q)()
    cy = (ctypes.c_int * Q)()
    cz = (ctypes.c_int * Q)()
    w = (ctypes.c_double * Q)()
    L.orc_lattice(cx, cy, cz, w)
    return (np.array(cx[:]), np.array(cy[:]), np.array(cz[:]), np.array(w[:]))


def psi(rho: float, rho0: float = 1.0) -> float:
    return lib().orc_psi(float(rho), float(rho0))


def pressure(rho: float, G: float, rho0: float = 1.0) -> float:
    """Eq. (7) of the paper."""
    return lib().orc_pressure(float(rho), float(G), float(rho0))


def feq(rho: float, u) -> np.ndarray:
    out = np.zeros(Q)
    lib().orc_feq(float(rho), float(u[0]), float(u[1]), float(u[2]), _dp(out))
    return out


# Rates of d'Humieres et al. (2002) for the non-hydrodynamic moments.
MRT_DEFAULT = {"s_e": 1.19, "s_eps": 1.4, "s_q": 1.2, "s_pi": 1.4, "s_m": 1.98}


def mrt_matrix() -> np.ndarray:
    """The 19 x 19 moment matrix M (rows: rho, e, eps, jx, qx, jy, qy, jz, qz,
    3pxx, 3pixx, pww, piww, pxy, pyz, pxz, mx, my, mz)."""
    M = np.empty((Q, Q))
    lib().orc_mrt_matrix(_dp(M))
    return M


def mrt_equilibrium(rho: float, j) -> np.ndarray:
    out = np.empty(Q)
    lib().orc_mrt_equilibrium(float(rho), float(j[0]), float(j[1]), float(j[2]), _dp(out))
    return out


def mrt_rates(tau: float, mrt: dict) -> np.ndarray:
    """Rate of every moment: the viscous moments (3pxx, pww, pxy, pyz, pxz)
    relax at 1/tau; the others as given in ``mrt`` (keys s_e, s_eps, s_q,
    s_pi, s_m, s_j; defaults MRT_DEFAULT and s_j = 1/tau)."""
    r = dict(MRT_DEFAULT)
    r["s_j"] = 1.0 / tau
    r.update(mrt)
    nu = 1.0 / tau
    return np.array([0.0, r["s_e"], r["s_eps"], r["s_j"], r["s_q"], r["s_j"], r["s_q"], r["s_j"],
                     r["s_q"], nu, r["s_pi"], nu, r["s_pi"], nu, nu, nu, r["s_m"], r["s_m"], r["s_m"]])


def step(f: np.ndarray, tau: float, G: float, rho0: float = 1.0, mrt: dict | None = None) -> np.ndarray:
    """One update; returns a new array."""
    if mrt is not None:
        return run(f, 1, tau, G, rho0, mrt)
    f = np.ascontiguousarray(f, dtype=np.float64)
    nx, ny, nz = _shape(f)
    out = np.empty_like(f)
    if lib().orc_step(nx, ny, nz, tau, G, rho0, _dp(f), _dp(out)) != 0:
        raise MemoryError("oracle step failed")
    return out


def run(f: np.ndarray, nsteps: int, tau: float, G: float, rho0: float = 1.0,
        mrt: dict | None = None) -> np.ndarray:
    """nsteps updates; returns a new array (the input is left untouched).
    ``mrt``: None for BGK, else the rates of the MRT collision (``mrt_rates``)."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    nx, ny, nz = _shape(f)
    scratch = np.empty_like(f)
    if mrt is None:
        rc = lib().orc_run(nx, ny, nz, tau, G, rho0, int(nsteps), _dp(f), _dp(scratch))
    else:
        s = mrt_rates(tau, mrt)
        rc = lib().orc_run_mrt(nx, ny, nz, _dp(s), G, rho0, int(nsteps), _dp(f), _dp(scratch))
    if rc != 0:
        raise MemoryError("oracle run failed")
    return f


def fields(f: np.ndarray, G: float, rho0: float = 1.0) -> dict:
    """rho (nz,ny,nx); j, F, u (3,nz,ny,nx); u is the physical (j + F/2)/rho."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    nx, ny, nz = _shape(f)
    rho = np.empty((nz, ny, nx))
    j = np.empty((3, nz, ny, nx))
    F = np.empty((3, nz, ny, nx))
    u = np.empty((3, nz, ny, nx))
    if lib().orc_fields(nx, ny, nz, G, rho0, _dp(f), _dp(rho), _dp(j), _dp(F), _dp(u)) != 0:
        raise MemoryError("oracle fields failed")
    return {"rho": rho, "j": j, "F": F, "u": u}


def splitmix64(s: int) -> int:
    return int(lib().orc_splitmix64(ctypes.c_uint64(s & (2**64 - 1))))


def uniform(seed: int, index: int) -> float:
    return float(lib().orc_uniform(seed & (2**64 - 1), index & (2**64 - 1)))


def init_ligament(nx: int, ny: int, nz: int, *, axis: int = 2, R0: float,
                  amp_rel: float, wavelength: float, c1: float | None = None,
                  c2: float | None = None, width: float = 2.0, rho_l: float,
                  rho_v: float, noise_amp: float = 0.0, seed: int = 0) -> np.ndarray:
    """Perturbed liquid cylinder at rest (Section 3); see sc_oracle.c."""
    plane = [(ny, nz), (nx, nz), (nx, ny)][axis]
    c1 = plane[0] / 2.0 if c1 is None else c1
    c2 = plane[1] / 2.0 if c2 is None else c2
    f = np.empty((Q, nz, ny, nx))
    rc = lib().orc_init_ligament(nx, ny, nz, axis, R0, amp_rel, wavelength, c1, c2, width,
                                 rho_l, rho_v, noise_amp, seed & (2**64 - 1), _dp(f))
    if rc != 0:
        raise ValueError("bad ligament spec")
    return f


def diag(f: np.ndarray, axis: int = 2) -> dict:
    f = np.ascontiguousarray(f, dtype=np.float64)
    nx, ny, nz = _shape(f)
    out = np.zeros(8)
    if lib().orc_diag(nx, ny, nz, axis, _dp(f), _dp(out)) != 0:
        raise MemoryError("oracle diag failed")
    return {"mass": out[0], "mom": out[1:4].copy(), "rho_min": out[4], "rho_max": out[5],
            "neck_rho": out[6], "nonfinite": int(out[7])}


def label(rho: np.ndarray, thresh: float):
    """6-connected periodic components of rho > thresh: (count, labels int32)."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    nz, ny, nx = rho.shape
    lab = np.zeros(rho.shape, dtype=np.int32)
    cnt = lib().orc_label(nx, ny, nz, _dp(rho), thresh,
                          lab.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if cnt < 0:
        raise MemoryError("oracle label failed")
    return int(cnt), lab


@dataclass
class Coexistence:
    rho_l: float
    rho_v: float
    steps: int
    residual: float
    converged: bool


def equal_area(G: float, rho0: float = 1.0):
    """Liquid/vapour densities of the Shan-Chen mechanical-stability
    construction for the EOS of Eq. (7): P(rho_v) = P(rho_l) = p and
    integral_{rho_v}^{rho_l} (p - P) psi'/psi^2 drho = 0.  The spinodals are
    closed-form (psi psi' = rho0 e (1 - e) with e = exp(-rho/rho0)); the
    roots and the pressure are found by bracketing (scipy brentq, quad)."""
    from scipy import integrate, optimize

    if not G < -4.0 / rho0:
        raise ValueError("no coexistence above the critical point")
    P = lambda r: pressure(r, G, rho0)
    root = math.sqrt(1.0 + 4.0 / (G * rho0))
    s_lo = -rho0 * math.log(0.5 * (1.0 + root))   # spinodal on the vapour side
    s_hi = -rho0 * math.log(0.5 * (1.0 - root))   # spinodal on the liquid side

    def branches(p):
        rv = optimize.brentq(lambda r: P(r) - p, 0.0, s_lo, xtol=1e-15)
        top = 3.0 * (p - G * rho0 * rho0 / 6.0) + 10.0
        rl = optimize.brentq(lambda r: P(r) - p, s_hi, top, xtol=1e-15)
        return rv, rl

    def area(p):
        rv, rl = branches(p)
        f = lambda r: (p - P(r)) * math.exp(-r / rho0) / psi(r, rho0) ** 2
        return integrate.quad(f, rv, rl, epsabs=1e-13, epsrel=1e-10, limit=400)[0]

    # the vapour branch exists only for p > 0 = P(0)
    lo, hi = max(P(s_hi), 0.0), P(s_lo)
    eps = 1e-12 * (hi - lo)
    p = optimize.brentq(area, lo + eps, hi - eps, xtol=1e-15)
    rv, rl = branches(p)
    return rl, rv


def coexistence(G: float, tau: float, rho0: float = 1.0, n: int = 128,
                tol: float = 1e-12, chunk: int = 1000, max_steps: int = 200_000,
                rho_hi: float | None = None, rho_lo: float | None = None,
                width: float = 4.0, tau_step: float = 0.05,
                mrt: dict | None = None) -> Coexistence:
    """Coexisting densities from a flat interface on a 1 x 1 x n periodic slab.

    Start: densities hi/lo of the equal-area construction (``equal_area``)
    unless given, profile
    rho = lo + (hi - lo)/2 [tanh(2(z - z1)/W) - tanh(2(z - z2)/W)] with
    z1 = n/4 - 1/2 and z2 = 3n/4 - 1/2 (liquid on [n/4, 3n/4)), populations at
    rest equilibrium.

    For tau < 1 the slab is first relaxed at tau = 1 and then at tau lowered
    in steps of ``tau_step`` (each of these stages until the largest density
    change over a chunk is below 1e-8, at most 100 chunks): starting a
    low-tau run directly from the construction's densities can blow up in
    the initial transient, while each stage starts close to its own steady
    state.

    The final stage at the requested tau runs in chunks; the residual of a
    chunk is the largest density change over it.  It stops when the residual
    is below ``tol``, when it has grown 100-fold above the smallest residual
    seen once that one is below 1e-8 (the quasi-1D slab at tau = 1 develops a
    slowly growing counter-flow drift seeded by round-off), or at
    ``max_steps``.  The state with the smallest residual is reported: liquid
    density at z = n/2, vapour at z = 0.  The velocity-shift forcing makes
    these depend on tau as well as on G.

    ``mrt``: run the slab with the MRT collision at these rates (the stages
    then change only the viscous rate 1/tau).
    """
    if rho_hi is None or rho_lo is None:
        rho_hi, rho_lo = equal_area(G, rho0)
    z = np.arange(n, dtype=np.float64)
    z1, z2 = n / 4 - 0.5, 3 * n / 4 - 0.5
    rho = rho_lo + (rho_hi - rho_lo) * 0.5 * (np.tanh(2.0 * (z - z1) / width)
                                             - np.tanh(2.0 * (z - z2) / width))
    _, _, _, w = lattice()
    f = np.empty((Q, n, 1, 1))
    for a in range(Q):
        f[a, :, 0, 0] = w[a] * rho
    stages = []
    if tau < 1.0:
        t = 1.0
        while t > tau + 1e-12:
            stages.append(t)
            t = round(t - tau_step, 12)
    diverged = Coexistence(float("nan"), float("nan"), 0, float("inf"), False)
    prev = rho.copy()
    for t in stages:  # relaxation stages
        for _ in range(100):
            f = run(f, chunk, t, G, rho0, mrt)
            cur = f.sum(axis=0)[:, 0, 0]
            if not np.all(np.isfinite(cur)):
                return diverged
            res = float(np.max(np.abs(cur - prev)))
            prev = cur
            if res < 1e-8:
                break
    best = (np.inf, 0, float(prev[n // 2]), float(prev[0]))
    steps = 0
    while steps < max_steps:
        f = run(f, chunk, tau, G, rho0, mrt)
        steps += chunk
        cur = f.sum(axis=0)[:, 0, 0]
        if not np.all(np.isfinite(cur)):
            if best[0] == np.inf:
                return diverged
            break
        res = float(np.max(np.abs(cur - prev)))
        prev = cur
        if res < best[0]:
            best = (res, steps, float(cur[n // 2]), float(cur[0]))
        if res < tol or (best[0] < 1e-8 and res > 100.0 * best[0]):
            break
    return Coexistence(best[2], best[3], best[1], best[0], best[0] < tol)


def breakup_time(steps, neck, rho_mid: float):
    """First sample where the neck density drops below rho_mid, with linear
    interpolation between that sample and the one before it; None if never."""
    prev = None
    for t, v in zip(steps, neck):
        if v < rho_mid:
            if prev is None:
                return float(t)
            t0, v0 = prev
            return float(t0) + (v0 - rho_mid) / (v0 - v) * (float(t) - float(t0))
        prev = (t, v)
    return None


def droplets(rho: np.ndarray, rho_mid: float):
    """(count, volumes, masses) of the 6-connected periodic components of
    rho > rho_mid, largest volume first."""
    count, lab = label(rho, rho_mid)
    vols = np.zeros(count, dtype=np.int64)
    mass = np.zeros(count)
    flat_l = lab.ravel()
    flat_r = np.asarray(rho, dtype=np.float64).ravel()
    for i in range(flat_l.size):
        c = flat_l[i]
        if c:
            vols[c - 1] += 1
            mass[c - 1] += flat_r[i]
    order = np.argsort(-vols, kind="stable")
    return count, vols[order], mass[order]


def run_to_breakup(f: np.ndarray, tau: float, G: float, rho_mid: float, max_steps: int,
                   every: int = 1, rho0: float = 1.0, axis: int = 2, mrt: dict | None = None):
    """Step the oracle, sampling the neck density every `every` steps, until it
    falls below rho_mid or max_steps.  Returns (t_b or None, steps, necks, f)."""
    steps, necks = [0], [diag(f, axis)["neck_rho"]]
    t = 0
    while t < max_steps and necks[-1] >= rho_mid:
        f = run(f, every, tau, G, rho0, mrt)
        t += every
        steps.append(t)
        necks.append(diag(f, axis)["neck_rho"])
    return breakup_time(steps, necks, rho_mid), steps, necks, f
