"""CPU oracle for the swept rule -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or runs it, and shares no code with
it.

The numbers come from ``oracle.c``: the plain full-grid, step-by-step
definition of what the swept rule computes (paper, Sections 2-3: the swept
decomposition only reorders the per-point sub-timestep updates, so its result
is that of plain time stepping).  This module only builds that file with gcc
and marshals numpy arrays to it.

Pins: each function here is checked in ``tests/test_oracle_pins.py`` against
closed forms (Fourier decay of the heat scheme, linearised KS growth, the
second-harmonic term of u u_x), exact rational brute force on small integer
data, conservation of the grid sum, and exact symmetries.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# -ffp-contract=off: no fused multiply-add anywhere; -fno-fast-math: IEEE
# semantics (no reassociation, denormals kept).
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
          "-shared", "-std=c99", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc and return the path."""
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        i64, i32, dbl, flt = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_float
        vp = ctypes.c_void_p
        L.oracle_heat_f64.argtypes = [vp, i64, i64, dbl, i32]
        L.oracle_heat_f32.argtypes = [vp, i64, i64, flt, i32]
        L.oracle_ks_f64.argtypes = [vp, i64, i64, dbl, dbl, i32]
        L.oracle_heat_f64_points.argtypes = [vp, i64, i64, dbl, vp, i64, vp]
        L.oracle_heat_f32_points.argtypes = [vp, i64, i64, flt, vp, i64, vp]
        L.oracle_ks_f64_points.argtypes = [vp, i64, i64, dbl, dbl, vp, i64, vp]
        L.oracle_heat_f64_adjoint.argtypes = [vp, i64, i64, dbl, i64, dbl, vp, vp, i32]
        L.oracle_ks_f64_adjoint.argtypes = [vp, i64, i64, dbl, dbl, i64, dbl, vp, vp, i32]
        L.oracle_euler_f64.argtypes = [vp, i64, i64, dbl, dbl, dbl, i32]
        L.oracle_ks_f64_tlm.argtypes = [vp, i64, i64, dbl, dbl, i64, dbl, vp, vp, i64, vp, i32]
        L.oracle_heat_fma_f64.argtypes = [vp, i64, i64, dbl, i32]
        L.oracle_heat_fma_f32.argtypes = [vp, i64, i64, flt, i32]
        L.oracle_ks_fma_f64.argtypes = [vp, i64, i64, dbl, dbl, i32]
        for name in ("oracle_heat_f64", "oracle_heat_f32", "oracle_ks_f64",
                     "oracle_heat_fma_f64", "oracle_heat_fma_f32", "oracle_ks_fma_f64",
                     "oracle_ks_f64_tlm",
                     "oracle_heat_f64_points", "oracle_heat_f32_points",
                     "oracle_ks_f64_points", "oracle_max_threads", "oracle_heat_f64_adjoint",
                     "oracle_ks_f64_adjoint", "oracle_euler_f64"):
            getattr(L, name).restype = i32
        _lib = L
    return _lib


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise RuntimeError("%s failed with code %d" % (what, rc))


def heat(u0: np.ndarray, nsteps: int, r: float, threads: int = 0) -> np.ndarray:
    """Heat FTCS, paper Section 4 ("3 FLOPs" finite-difference sub-timestep):
    u' = u + r*((u[i-1]+u[i+1]) - 2u), periodic.  float64 or float32 in/out;
    the arithmetic is done in the array's precision."""
    u = np.array(u0, copy=True, order="C")
    if u.dtype == np.float64:
        _check(lib().oracle_heat_f64(u.ctypes.data, u.size, int(nsteps), float(r),
                                     int(threads)), "oracle_heat_f64")
    elif u.dtype == np.float32:
        _check(lib().oracle_heat_f32(u.ctypes.data, u.size, int(nsteps),
                                     float(np.float32(r)), int(threads)), "oracle_heat_f32")
    else:
        raise TypeError("heat oracle takes float64 or float32")
    return u


def ks(u0: np.ndarray, nsteps: int, dt: float, dx: float, threads: int = 0) -> np.ndarray:
    """Kuramoto-Sivashinsky, paper Section 6 (finite differences + explicit
    RK2), as four radius-1 sub-timesteps per step (Section 2).  float64."""
    u = np.array(u0, dtype=np.float64, copy=True, order="C")
    _check(lib().oracle_ks_f64(u.ctypes.data, u.size, int(nsteps), float(dt), float(dx),
                               int(threads)), "oracle_ks_f64")
    return u


def heat_fma(u0: np.ndarray, nsteps: int, r: float, threads: int = 0) -> np.ndarray:
    """The heat scheme with its multiply-adds fused (Section 4's 3-FLOP
    form): u' = fma(r, fma(-2, u, u[i-1] + u[i+1]), u).  float64 or float32."""
    u = np.array(u0, copy=True, order="C")
    if u.dtype == np.float64:
        _check(lib().oracle_heat_fma_f64(u.ctypes.data, u.size, int(nsteps), float(r),
                                         int(threads)), "oracle_heat_fma_f64")
    elif u.dtype == np.float32:
        _check(lib().oracle_heat_fma_f32(u.ctypes.data, u.size, int(nsteps),
                                         float(np.float32(r)), int(threads)), "oracle_heat_fma_f32")
    else:
        raise TypeError("heat oracle takes float64 or float32")
    return u


def ks_fma(u0: np.ndarray, nsteps: int, dt: float, dx: float, threads: int = 0) -> np.ndarray:
    """The KS scheme with its multiply-adds fused: D2(a) = fma(-2, a,
    a[i-1] + a[i+1]) c2, F(a,b) = -(fma(a, D1 a, b) + D2 b), v = fma(h, F, u),
    u' = fma(dt, F, u).  float64."""
    u = np.array(u0, dtype=np.float64, copy=True, order="C")
    _check(lib().oracle_ks_fma_f64(u.ctypes.data, u.size, int(nsteps), float(dt), float(dx),
                                   int(threads)), "oracle_ks_fma_f64")
    return u


def euler(q0: np.ndarray, nsteps: int, dt: float, dx: float, gamma: float,
          threads: int = 0) -> np.ndarray:
    """1D Euler equations, paper Section 7 (second-order finite volume, minmod
    limiter, scalar dissipation by the Roe spectral radius, midpoint RK2) as
    four radius-1 sub-timesteps (Section 2).  q0 has shape (N, 3): rho, m, E
    per cell; float64."""
    q = np.array(q0, dtype=np.float64, copy=True, order="C")
    if q.ndim != 2 or q.shape[1] != 3:
        raise ValueError("q0 must have shape (N, 3)")
    _check(lib().oracle_euler_f64(q.ctypes.data, q.shape[0], int(nsteps), float(dt), float(dx),
                                  float(gamma), int(threads)), "oracle_euler_f64")
    return q


def heat_points(u0: np.ndarray, nsteps: int, r: float, idx) -> np.ndarray:
    """Selected outputs of heat(u0, nsteps, r), each from its cone of dependence."""
    u0 = np.ascontiguousarray(u0)
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    out = np.empty(idx.size, dtype=u0.dtype)
    if u0.dtype == np.float64:
        rc = lib().oracle_heat_f64_points(u0.ctypes.data, u0.size, int(nsteps), float(r),
                                          idx.ctypes.data, idx.size, out.ctypes.data)
    elif u0.dtype == np.float32:
        rc = lib().oracle_heat_f32_points(u0.ctypes.data, u0.size, int(nsteps),
                                          float(np.float32(r)), idx.ctypes.data, idx.size,
                                          out.ctypes.data)
    else:
        raise TypeError("heat oracle takes float64 or float32")
    _check(rc, "oracle_heat_points")
    return out


def ks_points(u0: np.ndarray, nsteps: int, dt: float, dx: float, idx) -> np.ndarray:
    """Selected outputs of ks(u0, nsteps, dt, dx), each from its cone of dependence."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    out = np.empty(idx.size, dtype=np.float64)
    _check(lib().oracle_ks_f64_points(u0.ctypes.data, u0.size, int(nsteps), float(dt),
                                      float(dx), idx.ctypes.data, idx.size, out.ctypes.data),
           "oracle_ks_points")
    return out


def _adjoint_args(u0, cot_final):
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    grad = np.empty_like(u0)
    cot = None if cot_final is None else np.ascontiguousarray(cot_final, dtype=np.float64)
    return u0, grad, cot


def heat_adjoint(u0, nsteps, r, n0, wgt, cot_final=None, threads=0):
    """dJ/du0 for J = wgt*sum_{j=n0}^{nsteps} |u^j|^2 + <cot_final, u^nsteps>, by
    the discrete adjoint (transposed sub-timestep Jacobians in reverse order)."""
    u0, grad, cot = _adjoint_args(u0, cot_final)
    _check(lib().oracle_heat_f64_adjoint(u0.ctypes.data, u0.size, int(nsteps), float(r), int(n0),
                                         float(wgt), None if cot is None else cot.ctypes.data,
                                         grad.ctypes.data, int(threads)), "oracle_heat_f64_adjoint")
    return grad


def ks_adjoint(u0, nsteps, dt, dx, n0, wgt, cot_final=None, threads=0):
    """dJ/du0 for the KS scheme, same objective as heat_adjoint."""
    u0, grad, cot = _adjoint_args(u0, cot_final)
    _check(lib().oracle_ks_f64_adjoint(u0.ctypes.data, u0.size, int(nsteps), float(dt), float(dx),
                                       int(n0), float(wgt), None if cot is None else cot.ctypes.data,
                                       grad.ctypes.data, int(threads)), "oracle_ks_f64_adjoint")
    return grad


def ks_tlm(u0, nsteps, dt, dx, n0, wgt, dirs, cot_final=None, threads=0):
    """<dJ/du0, v> for each row v of dirs (same objective as ks_adjoint), by
    forward-mode stepping of the KS scheme with its tangent-linear model."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    dirs = np.ascontiguousarray(np.atleast_2d(dirs), dtype=np.float64)
    if dirs.shape[1] != u0.size:
        raise ValueError("directions must have the field's length")
    cot = None if cot_final is None else np.ascontiguousarray(cot_final, dtype=np.float64)
    out = np.empty(dirs.shape[0])
    _check(lib().oracle_ks_f64_tlm(u0.ctypes.data, u0.size, int(nsteps), float(dt), float(dx),
                                   int(n0), float(wgt), None if cot is None else cot.ctypes.data,
                                   dirs.ctypes.data, dirs.shape[0], out.ctypes.data,
                                   int(threads)), "oracle_ks_f64_tlm")
    return out


def window_objective(u_steps, wgt):
    """J from a list of fields (test helper)."""
    return wgt * sum(float(np.dot(u, u)) for u in u_steps)
