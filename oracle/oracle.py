"""Python face of the FP64 CPU oracle (``tlb_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of ``bench.py``. The GPU library and its binding never
import, call or link anything in this directory.

The oracle follows the scheme of Sec. 2 of the paper step by step in double
precision; see the header of ``tlb_oracle.c`` for the order of operations and
the readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tlb_oracle.c")
_LIB = os.path.join(_HERE, "libtlb_oracle.so")

# Plain FP64: no contraction into FMA, no fast-math. Node loops are OpenMP
# parallel; each node's update reads only the previous state, so results do
# not depend on the thread count.
CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/libtlb_oracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("lx", ctypes.c_int32),
        ("ly", ctypes.c_int32),
        ("periodic_y", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("tau_g", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("g12", ctypes.c_double),
        ("g_a", ctypes.c_double * 2),
        ("g_r", ctypes.c_double * 2),
        ("alpha_g", ctypes.c_double),
        ("t_top", ctypes.c_double),
        ("rho_wall", ctypes.c_double * 2),
        ("dt_nominal", ctypes.c_double),
        ("u_wall", ctypes.c_double * 2),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        lib.ora_create.restype = ctypes.c_void_p
        lib.ora_create.argtypes = [ctypes.POINTER(_Params), dp, dp, dp, dp, dp,
                                   ctypes.POINTER(ctypes.c_uint8), dp]
        lib.ora_destroy.argtypes = [ctypes.c_void_p]
        lib.ora_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        lib.ora_time.argtypes = [ctypes.c_void_p]
        lib.ora_time.restype = ctypes.c_int64
        lib.ora_fields.argtypes = [ctypes.c_void_p, dp, dp, dp, dp, dp]
        lib.ora_populations.argtypes = [ctypes.c_void_p, dp, dp, dp]
        lib.ora_post_collision.argtypes = [ctypes.c_void_p, dp, dp, dp]
        lib.ora_observables.argtypes = [ctypes.c_void_p, dp]
        lib.ora_load_post_collision.argtypes = [ctypes.c_void_p, dp, dp, dp, ctypes.c_int64]
        lib.ora_stress.argtypes = [ctypes.c_void_p, dp, dp]
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.ora_droplets.restype = ctypes.c_int64
        lib.ora_droplets.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int64, i64p, i64p,
                                     dp, dp, dp, dp, ctypes.POINTER(ctypes.c_int32)]
        lib.ora_threads.restype = ctypes.c_int
        lib.ora_threads.argtypes = [ctypes.c_void_p]
        lib.ora_set_threads.argtypes = [ctypes.c_void_p, ctypes.c_int]
        _lib = lib
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class ModelParams:
    """Model constants (Sec. 2 and the tables of Appendix A)."""

    tau: float = 1.0
    tau_g: float = 1.0
    rho0: float = 0.83
    g12: float = 0.405
    g_a: tuple = (-9.0, -8.0)
    g_r: tuple = (8.1, 7.1)
    alpha_g: float = 0.0
    t_top: float = 0.0
    rho_wall: tuple = (0.612, 0.612)
    dt_nominal: float = 1.0
    u_wall: tuple = (0.0, 0.0)   # x-velocity of the bottom and top walls


OBS_NAMES = ("mass_a", "mass_b", "sum_t", "nu", "nu_top", "ke")



class Oracle:
    """One oracle run: a lattice state advanced step by step in FP64."""

    def __init__(self, params: ModelParams, rho_a, rho_b, temp, *, solid=None,
                 t_bottom=None, ux0=None, uy0=None, periodic_y=False, threads=None):
        rho_a = np.ascontiguousarray(rho_a, dtype=np.float64)
        ly, lx = rho_a.shape
        self.shape = (ly, lx)
        rho_b = np.ascontiguousarray(rho_b, dtype=np.float64).reshape(ly, lx)
        temp = np.ascontiguousarray(temp, dtype=np.float64).reshape(ly, lx)
        ux0 = None if ux0 is None else np.ascontiguousarray(ux0, np.float64).reshape(ly, lx)
        uy0 = None if uy0 is None else np.ascontiguousarray(uy0, np.float64).reshape(ly, lx)
        if solid is None:
            solid = np.zeros((ly, lx), np.uint8)
        solid = np.ascontiguousarray(solid, dtype=np.uint8).reshape(ly, lx)
        if t_bottom is None:
            t_bottom = np.ones(lx)
        t_bottom = np.ascontiguousarray(np.broadcast_to(np.asarray(t_bottom, np.float64), (lx,)))
        p = _Params()
        p.lx, p.ly, p.periodic_y = lx, ly, int(bool(periodic_y))
        p.tau, p.tau_g, p.rho0, p.g12 = params.tau, params.tau_g, params.rho0, params.g12
        p.g_a[0], p.g_a[1] = params.g_a
        p.g_r[0], p.g_r[1] = params.g_r
        p.alpha_g, p.t_top = params.alpha_g, params.t_top
        p.rho_wall[0], p.rho_wall[1] = params.rho_wall
        p.dt_nominal = params.dt_nominal
        p.u_wall[0], p.u_wall[1] = params.u_wall
        self._p = p
        lib = _load()
        self._h = lib.ora_create(ctypes.byref(p), _dp(rho_a), _dp(rho_b), _dp(temp),
                                 _dp(ux0), _dp(uy0),
                                 solid.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                 _dp(t_bottom))
        if not self._h:
            raise MemoryError("oracle state allocation failed")
        if threads is not None:
            lib.ora_set_threads(self._h, int(threads))
        self._keep = (solid, t_bottom)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().ora_destroy(h)
            self._h = None

    @property
    def threads(self) -> int:
        """Threads of the parallel node loops (results do not depend on it)."""
        return int(_load().ora_threads(self._h))

    @property
    def t(self) -> int:
        return int(_load().ora_time(self._h))

    def step(self, n: int = 1) -> "Oracle":
        _load().ora_step(self._h, int(n))
        return self

    def fields(self) -> dict:
        ly, lx = self.shape
        out = {k: np.empty((ly, lx)) for k in ("rho_a", "rho_b", "ux", "uy", "temp")}
        _load().ora_fields(self._h, *(_dp(out[k]) for k in ("rho_a", "rho_b", "ux", "uy", "temp")))
        return out

    def populations(self) -> np.ndarray:
        """Pre-collision f_A, f_B, g stacked as [27, ly, lx]."""
        ly, lx = self.shape
        out = np.empty((27, ly, lx))
        _load().ora_populations(self._h, _dp(out[0:9]), _dp(out[9:18]), _dp(out[18:27]))
        return out

    def post_collision(self) -> np.ndarray:
        """Post-collision f*_A, f*_B, g* stacked as [27, ly, lx]."""
        ly, lx = self.shape
        out = np.empty((27, ly, lx))
        _load().ora_post_collision(self._h, _dp(out[0:9]), _dp(out[9:18]), _dp(out[18:27]))
        return out

    def load_post_collision(self, pop, t: int) -> "Oracle":
        """Set the state to the streaming of post-collision populations
        ``pop`` ([27, ly, lx]: f*_A, f*_B, g*) and the time to ``t``."""
        pop = np.ascontiguousarray(pop, dtype=np.float64)
        if pop.shape != (27, *self.shape):
            raise ValueError("populations must be [27, ly, lx]")
        _load().ora_load_post_collision(self._h, _dp(pop[0:9]), _dp(pop[9:18]), _dp(pop[18:27]), int(t))
        return self

    def stress(self) -> dict:
        """xy stress of the current time, (ly, lx) each: the viscous part
        ``sxy_visc`` and the interaction pressure tensor ``pxy_int``; the
        total stress is their difference (zero at solid cells)."""
        ly, lx = self.shape
        out = {k: np.empty((ly, lx)) for k in ("sxy_visc", "pxy_int")}
        _load().ora_stress(self._h, _dp(out["sxy_visc"]), _dp(out["pxy_int"]))
        return out

    def droplets(self, threshold: float = 0.8) -> dict:
        """Droplets of the current time (bulk rho_A > threshold, 4-connected,
        numbered by smallest node index): arrays root, size, mass, x, y, nu
        and the node labels (ly, lx), -1 outside droplets."""
        ly, lx = self.shape
        lib = _load()
        label = np.empty((ly, lx), np.int32)
        n = lib.ora_droplets(self._h, float(threshold), 0, None, None, None, None, None, None,
                             label.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        if n < 0:
            raise MemoryError("oracle droplet buffers")
        out = {"root": np.empty(n, np.int64), "size": np.empty(n, np.int64)}
        for k in ("mass", "x", "y", "nu"):
            out[k] = np.empty(n)
        i64 = ctypes.POINTER(ctypes.c_int64)
        lib.ora_droplets(self._h, float(threshold), n, out["root"].ctypes.data_as(i64),
                         out["size"].ctypes.data_as(i64), _dp(out["mass"]), _dp(out["x"]),
                         _dp(out["y"]), _dp(out["nu"]), None)
        out["label"] = label
        return out

    def observables(self) -> dict:
        out = np.empty(6)
        _load().ora_observables(self._h, _dp(out))
        return dict(zip(OBS_NAMES, out.tolist()))
