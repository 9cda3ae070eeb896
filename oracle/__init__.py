"""FP64 CPU reference checker for the shallow-water RK3 step (test infrastructure).

Only the test-suite, the smoke check and the bench's CPU-baseline leg may
import this package.  The product library never loads it and shares no code
with it; see ``swe_oracle.c`` for the paper passages each routine follows and
the readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "swe_oracle.c"
_LIB = _HERE / "libswe_oracle.so"

BC_REFLECT = 0
BC_FIXED = 1


def build(force: bool = True) -> Path:
    """Compile the checker with gcc (plain C11, OpenMP, no FMA contraction)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp")
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", str(tmp), str(_SRC), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("g", ctypes.c_double), ("cfl", ctypes.c_double),
                ("dt_fixed", ctypes.c_double), ("h_dry", ctypes.c_double),
                ("weno_eps", ctypes.c_double), ("kappa_cap", ctypes.c_double),
                ("bc", ctypes.c_int32 * 4)]


_lib = None


def load(path) -> ctypes.CDLL:
    """Load a checker library from ``path`` and declare its entry points."""
    L = ctypes.CDLL(str(path))
    _declare(L)
    return L


def lib():
    global _lib
    if _lib is None:
        if not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
            build(force=True)
        _lib = load(_LIB)
    return _lib


def _declare(L):
    P = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    L.oracle_create.restype = P
    L.oracle_create.argtypes = [ctypes.POINTER(_Params), dp, dp, dp, dp, dp]
    L.oracle_step.restype = ctypes.c_int
    L.oracle_step.argtypes = [P, ctypes.c_int]
    L.oracle_read.restype = None
    L.oracle_read.argtypes = [P, dp, dp, dp]
    L.oracle_scalars.restype = None
    L.oracle_scalars.argtypes = [P, dp]
    L.oracle_rhs.restype = None
    L.oracle_rhs.argtypes = [P, dp, dp, dp]
    L.oracle_stage1.restype = ctypes.c_double
    L.oracle_stage1.argtypes = [P, dp, dp, dp]
    L.oracle_weno5.restype = ctypes.c_double
    L.oracle_weno5.argtypes = [dp, ctypes.c_double, dp]
    L.oracle_destroy.restype = None
    L.oracle_destroy.argtypes = [P]
    L.oracle_num_threads.restype = ctypes.c_int
    L.oracle_num_threads.argtypes = []
    L.oracle_set_friction.restype = None
    L.oracle_set_friction.argtypes = [P, ctypes.c_int]
    L.oracle_set_split.restype = None
    L.oracle_set_split.argtypes = [P, ctypes.c_int]


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def weno5(v, eps: float = 1e-6, L=None):
    """WENO5-JS reconstruction of a five-point stencil -> (value, weights)."""
    v = _f64(v)
    assert v.shape == (5,)
    w = np.zeros(3)
    r = (L or lib()).oracle_weno5(_dp(v), float(eps), _dp(w))
    return r, w


class Oracle:
    """One FP64 scenario.  Fields are row-major [ny][nx]."""

    def __init__(self, params, b, n, h, hu, hv, L=None):
        self._L = L or lib()
        p = _Params()
        p.nx, p.ny = int(params.nx), int(params.ny)
        p.dx, p.dy, p.g = float(params.dx), float(params.dy), float(params.g)
        p.cfl, p.dt_fixed = float(params.cfl), float(params.dt_fixed)
        p.h_dry, p.weno_eps = float(params.h_dry), float(params.weno_eps)
        p.kappa_cap = float(params.kappa_cap)
        for k in range(4):
            p.bc[k] = int(params.bc[k])
        self.nx, self.ny = p.nx, p.ny
        arrs = [_f64(a) for a in (b, n, h, hu, hv)]
        for a in arrs:
            if a.shape != (self.ny, self.nx):
                raise ValueError(f"field shape {a.shape} != ({self.ny}, {self.nx})")
        self._ptr = self._L.oracle_create(ctypes.byref(p), *[_dp(a) for a in arrs])
        if not self._ptr:
            raise ValueError("oracle_create rejected the inputs")

    @classmethod
    def from_scenario(cls, sc, L=None):
        return cls(sc.params, *sc.fields(), L=L)

    def step(self, nsteps: int) -> int:
        return int(self._L.oracle_step(self._ptr, int(nsteps)))

    def set_friction(self, implicit: bool):
        """Point-implicit friction per stage (reading R10) or the explicit term."""
        self._L.oracle_set_friction(self._ptr, 1 if implicit else 0)

    def set_split(self, local: bool):
        """Local Lax-Friedrichs splitting per face (reading R11) or the global speed."""
        self._L.oracle_set_split(self._ptr, 1 if local else 0)

    def state(self):
        h = np.empty((self.ny, self.nx))
        hu = np.empty_like(h)
        hv = np.empty_like(h)
        self._L.oracle_read(self._ptr, _dp(h), _dp(hu), _dp(hv))
        return h, hu, hv

    def scalars(self) -> dict:
        out = np.zeros(8)
        self._L.oracle_scalars(self._ptr, _dp(out))
        keys = ("t", "step", "mass", "clamp_mass", "runup", "alpha_x", "alpha_y", "dt")
        d = dict(zip(keys, out.tolist()))
        d["step"] = int(d["step"])
        return d

    def rhs(self):
        L = [np.empty((self.ny, self.nx)) for _ in range(3)]
        self._L.oracle_rhs(self._ptr, *[_dp(a) for a in L])
        return tuple(L)

    def stage1(self):
        out = [np.empty((self.ny, self.nx)) for _ in range(3)]
        dt = self._L.oracle_stage1(self._ptr, *[_dp(a) for a in out])
        return tuple(out), float(dt)

    def run_with_outputs(self, nsteps: int, times=(), max_depth: bool = False):
        """Advance nsteps steps one at a time, taking the run's outputs.

        The paper's runs write the state at chosen output times (Section 3,
        host orchestration).  Output k is the state at the end of the first
        step whose time reaches times[k] (times non-decreasing); one step may
        serve several outputs.  The maximum-depth map is, per cell, the
        maximum of h over the starting state and the state after every step.
        Returns (outputs, hmax): outputs[k] = (h, hu, hv, t, step) or None if
        the run does not reach times[k]; hmax is None unless max_depth.
        """
        times = [float(x) for x in times]
        outs = [None] * len(times)
        hmax = self.state()[0].copy() if max_depth else None
        k = 0
        for _ in range(int(nsteps)):
            rc = self.step(1)
            if rc != 0:
                raise RuntimeError(f"oracle step failed ({rc})")
            h, hu, hv = self.state()
            if max_depth:
                np.maximum(hmax, h, out=hmax)
            sc = self.scalars()
            while k < len(times) and sc["t"] >= times[k]:
                outs[k] = (h, hu, hv, sc["t"], sc["step"])
                k += 1
        return outs, hmax

    def close(self):
        if getattr(self, "_ptr", None):
            self._L.oracle_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
