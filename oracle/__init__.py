"""Plain FP64 CPU oracle for AIDW (arXiv 1511.02186) -- TEST INFRASTRUCTURE.

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this module.  The product path (the HIP library and its Python
binding) never imports it, and it imports nothing from the product path.

The arithmetic lives in ``aidw_oracle.c`` (plain C, FP64, no FMA contraction);
this file only marshals numpy arrays through ctypes.  See the C file's header
for the definition followed (Eq. 1-6 of the paper and the readings of the
points the paper leaves open).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "aidw_oracle.c")
_LIB = os.path.join(_HERE, "libaidw_oracle.so")
_lib = None

OK = 0
EINVAL = -1
ENOMEM = -2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, -ffp-contract=off) into oracle/."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-fPIC",
               "-shared", _SRC, "-o", tmp, "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_int64)
        lib.aidw_oracle_r_exp.restype = ctypes.c_double
        lib.aidw_oracle_r_exp.argtypes = [ctypes.c_int64, ctypes.c_double]
        lib.aidw_oracle_mu.restype = ctypes.c_double
        lib.aidw_oracle_mu.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
        lib.aidw_oracle_alpha.restype = ctypes.c_double
        lib.aidw_oracle_alpha.argtypes = [ctypes.c_double, dp]
        lib.aidw_oracle_run.restype = ctypes.c_int
        lib.aidw_oracle_run.argtypes = [dp, dp, dp, ctypes.c_int64, dp, dp, ctypes.c_int64,
                                        ctypes.c_int, dp, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, dp, dp, dp, lp, ctypes.c_int]
        lib.aidw_oracle_idw.restype = ctypes.c_int
        lib.aidw_oracle_idw.argtypes = [dp, dp, dp, ctypes.c_int64, dp, dp, ctypes.c_int64,
                                        ctypes.c_double, dp, ctypes.c_int]
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a, ty=ctypes.c_double):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ty))


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


class OracleError(RuntimeError):
    pass


def r_exp(m: int, area: float) -> float:
    """Eq. 2: expected nearest-neighbour distance for m points on area A."""
    return _load().aidw_oracle_r_exp(int(m), float(area))


def mu(R: float, R_min: float = 0.0, R_max: float = 2.0) -> float:
    """Eq. 5: fuzzy normalisation of the nearest-neighbour statistic."""
    return _load().aidw_oracle_mu(float(R), float(R_min), float(R_max))


def alpha(mu_R: float, levels) -> float:
    """Eq. 6: triangular membership from mu_R to the decay power."""
    lv = _f64(levels)
    assert lv.shape == (5,)
    return _load().aidw_oracle_alpha(float(mu_R), _ptr(lv))


def run(data_x, data_y, data_z, query_x, query_y, k, alpha_levels=(1, 2, 3, 4, 5),
        R_min=0.0, R_max=2.0, area=None, diag=False, threads=None):
    """AIDW of every query over all data points, in FP64.

    Inputs are promoted to float64 (so FP32 inputs are seen exactly).  ``area``
    is the study-area A of Eq. 2 and must be given.  Returns ``out`` or, with
    ``diag=True``, ``(out, r_obs, alpha, knn_idx)`` where ``knn_idx`` is
    ``[n, k]`` sorted by (squared distance, index).
    """
    if area is None:
        raise ValueError("area (A in Eq. 2) must be given")
    x, y, z = _f64(data_x), _f64(data_y), _f64(data_z)
    qx, qy = _f64(query_x), _f64(query_y)
    m, n = x.shape[0], qx.shape[0]
    assert y.shape == (m,) and z.shape == (m,) and qy.shape == (n,)
    lv = _f64(alpha_levels)
    assert lv.shape == (5,)
    out = np.empty(n, dtype=np.float64)
    r_obs = np.empty(n, dtype=np.float64) if diag else None
    al = np.empty(n, dtype=np.float64) if diag else None
    knn = np.empty((n, max(int(k), 1)), dtype=np.int64) if diag else None
    st = _load().aidw_oracle_run(_ptr(x), _ptr(y), _ptr(z), m, _ptr(qx), _ptr(qy), n, int(k),
                                 _ptr(lv), float(R_min), float(R_max), float(area), _ptr(out),
                                 _ptr(r_obs), _ptr(al), _ptr(knn, ctypes.c_int64),
                                 int(threads or default_threads()))
    if st != OK:
        raise OracleError("aidw_oracle_run returned %d" % st)
    if diag:
        return out, r_obs, al, knn
    return out


def idw(data_x, data_y, data_z, query_x, query_y, power, threads=None):
    """Standard IDW (Eq. 1) with a constant power, in FP64."""
    x, y, z = _f64(data_x), _f64(data_y), _f64(data_z)
    qx, qy = _f64(query_x), _f64(query_y)
    m, n = x.shape[0], qx.shape[0]
    out = np.empty(n, dtype=np.float64)
    st = _load().aidw_oracle_idw(_ptr(x), _ptr(y), _ptr(z), m, _ptr(qx), _ptr(qy), n,
                                 float(power), _ptr(out), int(threads or default_threads()))
    if st != OK:
        raise OracleError("aidw_oracle_idw returned %d" % st)
    return out
