"""ctypes binding of liblbm (include/liblbm.h).

Argument marshalling only: every step of the update runs in the HIP kernels
of ``liblbm.so``.  PyTorch supplies device memory (the workspace and field
tensors) and the HIP stream.  There is no CPU fallback: if the library is
not built, importing this module raises.

Module-level functions carry the C names (``lbm_create``, ``lbm_step``, ...);
``Lattice`` and ``Batch`` wrap them for convenience.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# LBM_LIBRARY names another build of the same library (the host-sanitized
# one of build.py), else the in-tree liblbm.so
LIB_PATH = os.environ.get("LBM_LIBRARY") or os.path.join(_HERE, "liblbm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python paper_1904_11792_amd/build.py` "
        "(the HIP library is the only implementation)")

_lib = ctypes.CDLL(LIB_PATH)

# ---- constants (include/liblbm.h) -------------------------------------------
LBM_OK = 0
LBM_ERR_INVALID_ARG = -1
LBM_ERR_UNSUPPORTED = -2
LBM_ERR_DEVICE = -3
LBM_ERR_STATE = -4
LBM_ERR_DIVERGED = -5
LBM_ERR_BUFFER_TOO_SMALL = -6
LBM_PSI_EXP = 0
LBM_F64, LBM_F32, LBM_F16S, LBM_BF16S, LBM_F16M, LBM_BF16M = 0, 1, 2, 3, 4, 5
LBM_FIELD_RHO, LBM_FIELD_U, LBM_FIELD_FORCE, LBM_FIELD_POP = 1, 2, 4, 8
LBM_DIAG_RING = 4096
LBM_NOALLOC_MAX_RUNS = 64

STORAGE = {"f64": LBM_F64, "f32": LBM_F32, "f16s": LBM_F16S, "bf16s": LBM_BF16S,
           "f16m": LBM_F16M, "bf16m": LBM_BF16M}
Q = 19


class lbm_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("tau", ctypes.c_double), ("G", ctypes.c_double), ("psi", ctypes.c_int32),
                ("rho0", ctypes.c_double), ("storage", ctypes.c_int32),
                ("rho_ref", ctypes.c_double)]


class lbm_ligament(ctypes.Structure):
    _fields_ = [("axis", ctypes.c_int32), ("R0", ctypes.c_double), ("amp_rel", ctypes.c_double),
                ("wavelength", ctypes.c_double), ("c1", ctypes.c_double), ("c2", ctypes.c_double),
                ("width", ctypes.c_double), ("rho_l", ctypes.c_double), ("rho_v", ctypes.c_double),
                ("noise_amp", ctypes.c_double), ("seed", ctypes.c_uint64)]


class lbm_diag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("mass", ctypes.c_double), ("mom", ctypes.c_double * 3),
                ("rho_min", ctypes.c_double), ("rho_max", ctypes.c_double),
                ("neck_rho", ctypes.c_double), ("nonfinite", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {"step": int(self.step), "mass": self.mass, "mom": list(self.mom),
                "rho_min": self.rho_min, "rho_max": self.rho_max, "neck_rho": self.neck_rho,
                "nonfinite": int(self.nonfinite)}


class lbm_mrt(ctypes.Structure):
    _fields_ = [("s_e", ctypes.c_double), ("s_eps", ctypes.c_double), ("s_q", ctypes.c_double),
                ("s_pi", ctypes.c_double), ("s_m", ctypes.c_double), ("s_j", ctypes.c_double)]


# Rates of the non-hydrodynamic moments suggested by d'Humieres et al. (2002).
MRT_DEFAULT = {"s_e": 1.19, "s_eps": 1.4, "s_q": 1.2, "s_pi": 1.4, "s_m": 1.98, "s_j": 0.0}


def make_mrt(**rates) -> lbm_mrt:
    """MRT rates; missing ones from MRT_DEFAULT (s_j = 0 selects 1/tau)."""
    r = dict(MRT_DEFAULT)
    unknown = set(rates) - set(r)
    if unknown:
        raise ValueError(f"unknown MRT rates {sorted(unknown)}")
    r.update(rates)
    return lbm_mrt(*(float(r[k]) for k in ("s_e", "s_eps", "s_q", "s_pi", "s_m", "s_j")))


class lbm_droplet(ctypes.Structure):
    _fields_ = [("volume", ctypes.c_int64), ("mass", ctypes.c_double), ("first_node", ctypes.c_int64)]


class lbm_launch(ctypes.Structure):
    _fields_ = [("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32), ("zchunk", ctypes.c_int32)]


_P = ctypes.POINTER
_vp, _sz, _i32, _i64, _u32, _d = (ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32,
                                  ctypes.c_int64, ctypes.c_uint32, ctypes.c_double)
_SIGS = {
    "lbm_workspace_bytes": (_sz, [_P(lbm_params)]),
    "lbm_create": (ctypes.c_int, [_P(lbm_params), _vp, _sz, _vp, _P(_vp)]),
    "lbm_destroy": (ctypes.c_int, [_vp]),
    "lbm_coexistence": (ctypes.c_int, [_d, _d, _i32, _d, _P(_d), _P(_d)]),
    "lbm_equal_area": (ctypes.c_int, [_d, _i32, _d, _P(_d), _P(_d)]),
    "lbm_coexistence_mrt": (ctypes.c_int, [_d, _d, _P(lbm_mrt), _i32, _d, _P(_d), _P(_d)]),
    "lbm_coexistence_many": (ctypes.c_int, [_i32, _P(_d), _P(_d), _P(lbm_mrt), _i32, _d, _P(_d), _P(_d),
                                            _P(_i32)]),
    "lbm_coexistence_many_noalloc": (ctypes.c_int, [_i32, _P(_d), _P(_d), _P(lbm_mrt), _i32, _d, _P(_d),
                                                    _P(_d), _P(_i32)]),
    "lbm_set_mrt": (ctypes.c_int, [_vp, _P(lbm_mrt)]),
    "lbm_init_ligament": (ctypes.c_int, [_vp, _P(lbm_ligament)]),
    "lbm_step": (ctypes.c_int, [_vp, _i64]),
    "lbm_get_fields": (ctypes.c_int, [_vp, _u32, _vp, _vp, _vp, _vp, _i32]),
    "lbm_set_populations": (ctypes.c_int, [_vp, _vp, _i32]),
    "lbm_diagnostics": (ctypes.c_int, [_vp, _P(lbm_diag)]),
    "lbm_set_axis": (ctypes.c_int, [_vp, _i32]),
    "lbm_record_diag": (ctypes.c_int, [_vp]),
    "lbm_read_diag_history": (ctypes.c_int, [_vp, _P(lbm_diag), _i32, _P(_i32)]),
    "lbm_get_step": (ctypes.c_int, [_vp, _P(_i64)]),
    "lbm_set_step": (ctypes.c_int, [_vp, _i64]),
    "lbm_droplets": (ctypes.c_int, [_vp, _d, _P(lbm_droplet), _i32, _P(_i64)]),
    "lbm_set_launch": (ctypes.c_int, [_vp, _P(lbm_launch)]),
    "lbm_get_launch": (ctypes.c_int, [_vp, _P(lbm_launch)]),
    "lbm_list_tiles": (ctypes.c_int, [_P(lbm_launch), _i32, _P(_i32)]),
    "lbm_default_launch": (ctypes.c_int, [_P(lbm_params), _P(lbm_launch), _P(_i32), _P(_i32)]),
    "lbm_lattice_layout": (ctypes.c_int, [_P(lbm_params), _P(_i32), _P(_i64)]),
    "lbm_autotune": (ctypes.c_int, [_vp, _i32, _P(lbm_launch), _P(_d)]),
    "lbm_set_graph_chunk": (ctypes.c_int, [_vp, _i32]),
    "lbm_last_error": (ctypes.c_char_p, []),
    "lbm_version": (ctypes.c_char_p, []),
    "lbm_device_copy": (ctypes.c_int, [_vp, _vp, _sz, _vp]),
    "lbm_batch_workspace_bytes": (_sz, [_i32, _P(lbm_params)]),
    "lbm_batch_create": (ctypes.c_int, [_i32, _P(lbm_params), _vp, _sz, _vp, _P(_vp)]),
    "lbm_batch_init": (ctypes.c_int, [_vp, _P(lbm_ligament)]),
    "lbm_batch_step": (ctypes.c_int, [_vp, _i64]),
    "lbm_batch_diagnostics": (ctypes.c_int, [_vp, _P(lbm_diag)]),
    "lbm_batch_get_fields": (ctypes.c_int, [_vp, _i32, _u32, _vp, _vp, _vp, _vp, _i32]),
    "lbm_batch_set_launch": (ctypes.c_int, [_vp, _P(lbm_launch)]),
    "lbm_batch_set_graph_chunk": (ctypes.c_int, [_vp, _i32]),
    "lbm_batch_set_chunking": (ctypes.c_int, [_vp, _i32]),
    "lbm_batch_autotune": (ctypes.c_int, [_vp, _i32, _P(lbm_launch), _P(_d)]),
    "lbm_batch_destroy": (ctypes.c_int, [_vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class LbmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"liblbm status {status}: {message}")
        self.status = status
        self.message = message


def _check(status: int, ok=(LBM_OK,)):
    if status not in ok:
        raise LbmError(status, lbm_last_error())
    return status


# ---- thin wrappers with the C names -----------------------------------------
def lbm_last_error() -> str:
    return _lib.lbm_last_error().decode()


def lbm_version() -> str:
    return _lib.lbm_version().decode()


def lbm_workspace_bytes(p: lbm_params) -> int:
    return int(_lib.lbm_workspace_bytes(ctypes.byref(p)))


def lbm_create(p: lbm_params, workspace_ptr: int, ws_bytes: int, stream_handle: int):
    ctx = _vp()
    _check(_lib.lbm_create(ctypes.byref(p), _vp(workspace_ptr), ws_bytes, _vp(stream_handle),
                           ctypes.byref(ctx)))
    return ctx


def lbm_destroy(ctx) -> None:
    _check(_lib.lbm_destroy(ctx))


def lbm_coexistence(G: float, tau: float, psi: int = LBM_PSI_EXP, rho0: float = 1.0,
                    mrt: dict | None = None):
    """Flat-interface coexistence densities; mrt: None (BGK) or MRT rates (make_mrt keys)."""
    rl, rv = _d(), _d()
    if mrt is None:
        _check(_lib.lbm_coexistence(G, tau, psi, rho0, ctypes.byref(rl), ctypes.byref(rv)))
    else:
        m = make_mrt(**mrt)
        _check(_lib.lbm_coexistence_mrt(G, tau, ctypes.byref(m), psi, rho0, ctypes.byref(rl),
                                        ctypes.byref(rv)))
    return rl.value, rv.value


def lbm_coexistence_many(G, tau, psi: int = LBM_PSI_EXP, rho0: float = 1.0, mrt: dict | None = None):
    """lbm_coexistence for each (G[j], tau[j]), all runs advanced together.

    Returns (rho_l, rho_v, status) as numpy arrays; a diverged run has status
    LBM_ERR_DIVERGED and NaN densities (no exception for that)."""
    return _coexistence_many(_lib.lbm_coexistence_many, G, tau, psi, rho0, mrt)


def lbm_coexistence_many_noalloc(G, tau, psi: int = LBM_PSI_EXP, rho0: float = 1.0,
                                 mrt: dict | None = None):
    """lbm_coexistence_many on the library's fixed device array (no device
    allocation; at most LBM_NOALLOC_MAX_RUNS runs)."""
    return _coexistence_many(_lib.lbm_coexistence_many_noalloc, G, tau, psi, rho0, mrt)


def _coexistence_many(fn, G, tau, psi, rho0, mrt):
    G = np.ascontiguousarray(G, dtype=np.float64)
    tau = np.ascontiguousarray(tau, dtype=np.float64)
    if G.shape != tau.shape or G.ndim != 1:
        raise ValueError("G and tau must be 1-D arrays of one length")
    m = G.size
    rl, rv = np.empty(m), np.empty(m)
    st = np.empty(m, dtype=np.int32)
    dp = lambda a: a.ctypes.data_as(_P(_d))
    mp = ctypes.byref(make_mrt(**mrt)) if mrt is not None else None
    _check(fn(m, dp(G), dp(tau), mp, psi, rho0, dp(rl), dp(rv), st.ctypes.data_as(_P(_i32))),
           ok=(LBM_OK, LBM_ERR_DIVERGED))
    return rl, rv, st


def lbm_set_mrt(ctx, mrt: dict | None) -> None:
    if mrt is None:
        _check(_lib.lbm_set_mrt(ctx, None))
    else:
        m = make_mrt(**mrt)
        _check(_lib.lbm_set_mrt(ctx, ctypes.byref(m)))


def lbm_equal_area(G: float, psi: int = LBM_PSI_EXP, rho0: float = 1.0):
    rl, rv = _d(), _d()
    _check(_lib.lbm_equal_area(G, psi, rho0, ctypes.byref(rl), ctypes.byref(rv)))
    return rl.value, rv.value


def lbm_init_ligament(ctx, spec: lbm_ligament) -> None:
    _check(_lib.lbm_init_ligament(ctx, ctypes.byref(spec)))


def lbm_step(ctx, nsteps: int) -> None:
    _check(_lib.lbm_step(ctx, int(nsteps)))


def lbm_get_fields(ctx, mask, rho=0, u=0, force=0, pop=0, on_device=1) -> None:
    _check(_lib.lbm_get_fields(ctx, mask, _vp(rho), _vp(u), _vp(force), _vp(pop), on_device))


def lbm_set_populations(ctx, pop_ptr: int, on_device: int = 1) -> None:
    _check(_lib.lbm_set_populations(ctx, _vp(pop_ptr), on_device))


def lbm_diagnostics(ctx) -> tuple[int, lbm_diag]:
    d = lbm_diag()
    st = _check(_lib.lbm_diagnostics(ctx, ctypes.byref(d)), ok=(LBM_OK, LBM_ERR_DIVERGED))
    return st, d


def lbm_droplets(ctx, rho_mid: float, max_out: int = 1024) -> tuple[int, list[lbm_droplet]]:
    buf = (lbm_droplet * max(max_out, 1))()
    cnt = _i64()
    _check(_lib.lbm_droplets(ctx, float(rho_mid), buf, int(max_out), ctypes.byref(cnt)))
    return int(cnt.value), [buf[i] for i in range(min(int(cnt.value), max_out))]


def lbm_set_axis(ctx, axis: int) -> None:
    _check(_lib.lbm_set_axis(ctx, axis))


def lbm_record_diag(ctx) -> None:
    _check(_lib.lbm_record_diag(ctx))


def lbm_read_diag_history(ctx, max_records: int = LBM_DIAG_RING) -> list[lbm_diag]:
    buf = (lbm_diag * max_records)()
    cnt = _i32()
    _check(_lib.lbm_read_diag_history(ctx, buf, max_records, ctypes.byref(cnt)))
    return [buf[i] for i in range(cnt.value)]


def lbm_get_step(ctx) -> int:
    s = _i64()
    _check(_lib.lbm_get_step(ctx, ctypes.byref(s)))
    return s.value


def lbm_set_step(ctx, step: int) -> None:
    _check(_lib.lbm_set_step(ctx, int(step)))


def lbm_set_launch(ctx, tile_x: int, tile_y: int, zchunk: int) -> None:
    _check(_lib.lbm_set_launch(ctx, ctypes.byref(lbm_launch(tile_x, tile_y, zchunk))))


def lbm_get_launch(ctx) -> tuple[int, int, int]:
    l = lbm_launch()
    _check(_lib.lbm_get_launch(ctx, ctypes.byref(l)))
    return l.tile_x, l.tile_y, l.zchunk


def lbm_list_tiles() -> list[tuple[int, int]]:
    buf = (lbm_launch * 64)()
    cnt = _i32()
    _check(_lib.lbm_list_tiles(buf, 64, ctypes.byref(cnt)))
    return [(buf[i].tile_x, buf[i].tile_y) for i in range(min(cnt.value, 64))]


def lbm_default_launch(params: lbm_params):
    """((tile_x, tile_y, zchunk), (tile_w, tile_h)): the default launch and its run-time tile."""
    l, tw, th = lbm_launch(), _i32(), _i32()
    _check(_lib.lbm_default_launch(ctypes.byref(params), ctypes.byref(l), ctypes.byref(tw), ctypes.byref(th)))
    return (l.tile_x, l.tile_y, l.zchunk), (tw.value, th.value)


def lbm_lattice_layout(params: lbm_params) -> tuple[int, int]:
    """(rows per record, bytes of one lattice) of the HBM layout for these parameters."""
    k, nbytes = _i32(), _i64()
    _check(_lib.lbm_lattice_layout(ctypes.byref(params), ctypes.byref(k), ctypes.byref(nbytes)))
    return k.value, nbytes.value


def lbm_autotune(ctx, steps_per_candidate: int = 5):
    l = lbm_launch()
    m = _d()
    _check(_lib.lbm_autotune(ctx, steps_per_candidate, ctypes.byref(l), ctypes.byref(m)))
    return (l.tile_x, l.tile_y, l.zchunk), m.value


def lbm_set_graph_chunk(ctx, chunk_steps: int) -> None:
    _check(_lib.lbm_set_graph_chunk(ctx, chunk_steps))


def lbm_device_copy(dst_ptr: int, src_ptr: int, nbytes: int, stream_handle: int) -> None:
    _check(_lib.lbm_device_copy(_vp(dst_ptr), _vp(src_ptr), nbytes, _vp(stream_handle)))


# ---- convenience wrappers ----------------------------------------------------
def make_params(nx, ny, nz, tau, G, rho0=1.0, storage="f32", rho_ref=0.0) -> lbm_params:
    st = STORAGE[storage] if isinstance(storage, str) else int(storage)
    return lbm_params(int(nx), int(ny), int(nz), float(tau), float(G), LBM_PSI_EXP, float(rho0),
                      st, float(rho_ref))


def make_ligament(nx, ny, nz, *, axis=2, R0, amp_rel, wavelength, c1=None, c2=None, width=2.0,
                  rho_l=None, rho_v=None, noise_amp=0.0, seed=0) -> lbm_ligament:
    plane = [(ny, nz), (nx, nz), (nx, ny)][axis]
    c1 = plane[0] / 2.0 if c1 is None else c1
    c2 = plane[1] / 2.0 if c2 is None else c2
    return lbm_ligament(int(axis), float(R0), float(amp_rel), float(wavelength), float(c1),
                        float(c2), float(width), float(rho_l or 0.0), float(rho_v or 0.0),
                        float(noise_amp), int(seed) & (2 ** 64 - 1))


def _stream_handle(stream) -> int:
    return int(stream.cuda_stream) if stream is not None else 0


class Lattice:
    """One periodic grid behind an lbm_ctx; device memory from torch."""

    def __init__(self, nx, ny, nz, tau, G, rho0=1.0, storage="f32", rho_ref=0.0,
                 device="cuda", stream=None, mrt: dict | None = None):
        self.params = make_params(nx, ny, nz, tau, G, rho0, storage, rho_ref)
        nbytes = lbm_workspace_bytes(self.params)
        if nbytes == 0:
            raise LbmError(LBM_ERR_INVALID_ARG, lbm_last_error())
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        # the library works on the workspace on self.stream: the caching
        # allocator must not hand it out again before that work is done
        self.workspace.record_stream(self.stream)
        self.ctx = lbm_create(self.params, self.workspace.data_ptr(), nbytes,
                              _stream_handle(self.stream))
        self.shape = (nz, ny, nx)
        self.n = nx * ny * nz
        if mrt is not None:
            lbm_set_mrt(self.ctx, mrt)

    def set_mrt(self, mrt: dict | None) -> None:
        """Select the collision: None for BGK, else MRT rates (make_mrt keys)."""
        lbm_set_mrt(self.ctx, mrt)

    def close(self):
        if getattr(self, "ctx", None):
            self.stream.synchronize()  # queued steps still use the workspace
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_ligament(self, **kw) -> None:
        nz, ny, nx = self.shape
        lbm_init_ligament(self.ctx, make_ligament(nx, ny, nz, **kw))

    def step(self, n: int = 1) -> None:
        lbm_step(self.ctx, n)

    @property
    def step_count(self) -> int:
        return lbm_get_step(self.ctx)

    def set_step(self, step: int) -> None:
        lbm_set_step(self.ctx, step)

    def fields(self, rho=True, u=False, force=False, pop=False) -> dict:
        """FP64 device tensors: rho (nz,ny,nx), u/force (3,nz,ny,nx), pop (19,nz,ny,nx)."""
        nz, ny, nx = self.shape
        out = {}
        mask = 0
        opt = dict(dtype=torch.float64, device=self.device)
        if rho:
            out["rho"] = torch.empty((nz, ny, nx), **opt)
            mask |= LBM_FIELD_RHO
        if u:
            out["u"] = torch.empty((3, nz, ny, nx), **opt)
            mask |= LBM_FIELD_U
        if force:
            out["force"] = torch.empty((3, nz, ny, nx), **opt)
            mask |= LBM_FIELD_FORCE
        if pop:
            out["pop"] = torch.empty((Q, nz, ny, nx), **opt)
            mask |= LBM_FIELD_POP
        p = lambda k: out[k].data_ptr() if k in out else 0
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        lbm_get_fields(self.ctx, mask, p("rho"), p("u"), p("force"), p("pop"), 1)
        cur.wait_stream(self.stream)
        return out

    def populations(self) -> torch.Tensor:
        return self.fields(rho=False, pop=True)["pop"]

    def set_populations(self, pop) -> None:
        nz, ny, nx = self.shape
        t = torch.as_tensor(pop, dtype=torch.float64).to(self.device).contiguous()
        if tuple(t.shape) != (Q, nz, ny, nx):
            raise ValueError(f"populations must have shape {(Q, nz, ny, nx)}")
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        lbm_set_populations(self.ctx, t.data_ptr(), 1)
        self.stream.synchronize()  # t may be freed when this returns

    def diagnostics(self) -> dict:
        st, d = lbm_diagnostics(self.ctx)
        r = d.as_dict()
        r["diverged"] = st == LBM_ERR_DIVERGED
        return r

    def set_axis(self, axis: int) -> None:
        lbm_set_axis(self.ctx, axis)

    def droplets(self, rho_mid: float, max_out: int = 1024) -> dict:
        """Components of rho > rho_mid labelled on the device: count, and for
        the max_out largest their volumes, masses and first nodes."""
        count, items = lbm_droplets(self.ctx, rho_mid, max_out)
        return {"count": count,
                "volumes": np.array([d.volume for d in items], dtype=np.int64),
                "masses": np.array([d.mass for d in items], dtype=np.float64),
                "first_nodes": np.array([d.first_node for d in items], dtype=np.int64)}

    def record_diag(self) -> None:
        lbm_record_diag(self.ctx)

    def read_diag_history(self) -> list[dict]:
        return [d.as_dict() for d in lbm_read_diag_history(self.ctx)]

    def set_launch(self, tile_x, tile_y, zchunk) -> None:
        lbm_set_launch(self.ctx, tile_x, tile_y, zchunk)

    def get_launch(self):
        return lbm_get_launch(self.ctx)

    def autotune(self, steps_per_candidate: int = 5):
        return lbm_autotune(self.ctx, steps_per_candidate)

    def set_graph_chunk(self, chunk_steps: int) -> None:
        lbm_set_graph_chunk(self.ctx, chunk_steps)


class Batch:
    """Many independent ligaments advanced by one launch per step."""

    def __init__(self, params_list, device="cuda", stream=None):
        n = len(params_list)
        arr = (lbm_params * n)(*params_list)
        nbytes = int(_lib.lbm_batch_workspace_bytes(n, arr))
        if nbytes == 0:
            raise LbmError(LBM_ERR_INVALID_ARG, lbm_last_error())
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self.workspace.record_stream(self.stream)  # as in Lattice
        h = _vp()
        _check(_lib.lbm_batch_create(n, arr, _vp(self.workspace.data_ptr()), nbytes,
                                     _vp(_stream_handle(self.stream)), ctypes.byref(h)))
        self.handle = h
        self.params = list(params_list)
        self.count = n

    def close(self):
        if getattr(self, "handle", None):
            self.stream.synchronize()
            _check(_lib.lbm_batch_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, specs) -> None:
        arr = (lbm_ligament * self.count)(*specs)
        _check(_lib.lbm_batch_init(self.handle, arr))

    def step(self, n: int = 1) -> None:
        _check(_lib.lbm_batch_step(self.handle, int(n)))

    def diagnostics(self) -> list[dict]:
        arr = (lbm_diag * self.count)()
        _check(_lib.lbm_batch_diagnostics(self.handle, arr))
        return [arr[i].as_dict() for i in range(self.count)]

    def fields(self, index: int, rho=True, pop=False) -> dict:
        p = self.params[index]
        nz, ny, nx = p.nz, p.ny, p.nx
        opt = dict(dtype=torch.float64, device=self.device)
        out, mask = {}, 0
        if rho:
            out["rho"] = torch.empty((nz, ny, nx), **opt)
            mask |= LBM_FIELD_RHO
        if pop:
            out["pop"] = torch.empty((Q, nz, ny, nx), **opt)
            mask |= LBM_FIELD_POP
        ptr = lambda k: out[k].data_ptr() if k in out else 0
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        _check(_lib.lbm_batch_get_fields(self.handle, index, mask, _vp(ptr("rho")), None, None,
                                         _vp(ptr("pop")), 1))
        cur.wait_stream(self.stream)
        return out

    def set_launch(self, tile_x, tile_y, zchunk) -> None:
        _check(_lib.lbm_batch_set_launch(self.handle, ctypes.byref(lbm_launch(tile_x, tile_y, zchunk))))

    def set_graph_chunk(self, chunk_steps: int) -> None:
        _check(_lib.lbm_batch_set_graph_chunk(self.handle, chunk_steps))

    def set_chunking(self, rounds: int) -> None:
        """0: uniform z chunks of the launch; > 0: equal-cost chunks, about `rounds` rounds."""
        _check(_lib.lbm_batch_set_chunking(self.handle, int(rounds)))

    def autotune(self, steps_per_candidate: int = 3):
        l = lbm_launch()
        m = _d()
        _check(_lib.lbm_batch_autotune(self.handle, steps_per_candidate, ctypes.byref(l), ctypes.byref(m)))
        return (l.tile_x, l.tile_y, l.zchunk), m.value
