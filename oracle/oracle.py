"""ctypes front end of the plain C oracle (oracle/vlasov_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark.  The solver package never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vlasov_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# R8: sin and cos are called on their own (no merging into sincos)
CFLAGS = ["-O2", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-fno-builtin-sin", "-fno-builtin-cos", "-fno-builtin-sincos",
          "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP contraction off, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


class _P(C.Structure):
    _fields_ = [("model", C.c_int32), ("storage", C.c_int32), ("bc_x", C.c_int32), ("bc_p", C.c_int32),
                ("spline", C.c_int32), ("splitting", C.c_int32), ("filter_every", C.c_int32), ("pad", C.c_int32),
                ("nx", C.c_int64), ("np", C.c_int64),
                ("xmin", C.c_double), ("xmax", C.c_double), ("pmin", C.c_double), ("pmax", C.c_double),
                ("dt", C.c_double), ("ring_eps", C.c_double), ("sheet_G", C.c_double),
                ("filter_strength", C.c_double)]


_lib = None
_D = C.POINTER(C.c_double)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        lib = C.CDLL(LIB)
        PP = C.POINTER(_P)
        lib.oracle_run.argtypes = [PP, _D, C.c_int64, _D, _D]
        lib.oracle_run.restype = C.c_int
        lib.oracle_sweep_x.argtypes = [PP, _D, _D, C.c_double]
        lib.oracle_sweep_p.argtypes = [PP, _D, _D, _D, C.c_double]
        lib.oracle_density.argtypes = [PP, _D, _D]
        lib.oracle_force.argtypes = [PP, _D, _D, _D, _D]
        lib.oracle_moments.argtypes = [PP, _D, _D]
        lib.oracle_second_difference.argtypes = [_D, C.c_int64, C.c_int64, C.c_int]
        lib.oracle_second_difference.restype = C.c_double
        lib.oracle_foot.argtypes = [C.c_double, C.POINTER(C.c_int64), _D]
        lib.oracle_interpolate_line.argtypes = [_D, _D, C.c_int64, C.c_double, C.c_int, C.c_int]
        lib.oracle_interpolate_line_gs.argtypes = [_D, _D, C.c_int64, C.c_double, C.c_int, C.c_int]
        lib.oracle_ring_dV.argtypes = [PP, C.c_int64]
        lib.oracle_ring_dV.restype = C.c_double
        lib.oracle_ring_V.argtypes = [PP, C.c_int64]
        lib.oracle_ring_V.restype = C.c_double
        lib.oracle_filter_p.argtypes = [PP, _D, _D]
        lib.oracle_split_weights.argtypes = [C.c_int, _D]
        lib.oracle_split_weights.restype = C.c_int
        lib.oracle_set_threads.argtypes = [C.c_int]
        lib.oracle_set_threads.restype = None
        lib.oracle_get_threads.argtypes = []
        lib.oracle_get_threads.restype = C.c_int
        _lib = lib
    return _lib


def _params(p) -> _P:
    return _P(int(p.model), int(p.storage), int(p.bc_x), int(p.bc_p), int(getattr(p, "spline", 0)),
              int(getattr(p, "splitting", 0)), int(getattr(p, "filter_every", 0)), 0,
              int(p.nx), int(p.np_),
              float(p.xmin), float(p.xmax), float(p.pmin), float(p.pmax), float(p.dt),
              float(p.ring_eps), float(p.sheet_G), float(getattr(p, "filter_strength", 0.0)))


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (the results do not depend on it)."""
    _load().oracle_set_threads(int(n))


def threads() -> int:
    return int(_load().oracle_get_threads())


def split_weights(scheme: int) -> list[float]:
    """Sizes w_k (in units of dt) of the substeps of one step."""
    w = np.zeros(8)
    n = _load().oracle_split_weights(int(scheme), _ptr(w))
    return [float(v) for v in w[:n]]


def run(p, f0: np.ndarray, nsteps: int, F_ext=None, history: bool = False):
    """nsteps time steps from f0; returns f (and the magnetization history of
    the drifted distributions, one (Mx, My) row per force evaluation, i.e.
    nsteps times the number of substeps, if history=True)."""
    lib = _load()
    f = _f64(f0).copy()
    assert f.shape == (p.np_, p.nx)
    nev = nsteps * len(split_weights(getattr(p, "splitting", 0)))
    hist = np.zeros((max(nev, 1), 2)) if history else None
    fe = _f64(F_ext) if F_ext is not None else None
    rc = lib.oracle_run(C.byref(_params(p)), _ptr(f), int(nsteps), _ptr(fe) if fe is not None else None,
                        _ptr(hist) if hist is not None else None)
    if rc != 0:
        raise MemoryError("oracle_run failed")
    return (f, hist[:nev]) if history else f


def filter_p(p, f: np.ndarray) -> np.ndarray:
    """The filter along p (one application with p.filter_strength)."""
    lib = _load()
    f = _f64(f)
    out = np.empty_like(f)
    lib.oracle_filter_p(C.byref(_params(p)), _ptr(f), _ptr(out))
    return out


def sweep_x(p, f: np.ndarray, tau: float) -> np.ndarray:
    lib = _load()
    f = _f64(f)
    out = np.empty_like(f)
    lib.oracle_sweep_x(C.byref(_params(p)), _ptr(f), _ptr(out), float(tau))
    return out


def sweep_p(p, f: np.ndarray, F: np.ndarray, dt: float) -> np.ndarray:
    lib = _load()
    f = _f64(f)
    F = _f64(F)
    out = np.empty_like(f)
    lib.oracle_sweep_p(C.byref(_params(p)), _ptr(f), _ptr(out), _ptr(F), float(dt))
    return out


def density(p, f: np.ndarray) -> np.ndarray:
    lib = _load()
    f = _f64(f)
    rho = np.empty(p.nx)
    lib.oracle_density(C.byref(_params(p)), _ptr(f), _ptr(rho))
    return rho


def force(p, rho: np.ndarray, F_ext=None):
    """Returns (F, (mx, my))."""
    lib = _load()
    rho = _f64(rho)
    F = np.empty(p.nx)
    mm = np.zeros(2)
    fe = _f64(F_ext) if F_ext is not None else None
    lib.oracle_force(C.byref(_params(p)), _ptr(rho), _ptr(fe) if fe is not None else None, _ptr(F), _ptr(mm))
    return F, (float(mm[0]), float(mm[1]))


MOMENT_NAMES = ("mass", "momentum", "kinetic", "potential", "energy", "mx", "my", "l2", "entropy", "neg_mass")


def moments(p, f: np.ndarray) -> dict:
    lib = _load()
    f = _f64(f)
    out = np.zeros(len(MOMENT_NAMES))
    lib.oracle_moments(C.byref(_params(p)), _ptr(f), _ptr(out))
    return dict(zip(MOMENT_NAMES, out.tolist()))


def second_difference(line: np.ndarray, l: int, bc: int = 0) -> float:
    lib = _load()
    line = _f64(line)
    return lib.oracle_second_difference(_ptr(line), line.size, int(l), int(bc))


def foot(shift: float):
    """(m, alpha, beta, gamma, delta) of a shift in cells."""
    lib = _load()
    m = C.c_int64()
    w = np.zeros(4)
    lib.oracle_foot(float(shift), C.byref(m), _ptr(w))
    return (m.value, *w.tolist())


def interpolate_line(line: np.ndarray, shift: float, bc: int = 0, storage: int = 0) -> np.ndarray:
    lib = _load()
    line = _f64(line)
    out = np.empty_like(line)
    lib.oracle_interpolate_line(_ptr(line), _ptr(out), line.size, float(shift), int(bc), int(storage))
    return out


def interpolate_line_gs(line: np.ndarray, shift: float, bc: int = 0, storage: int = 0) -> np.ndarray:
    """One line moved by `shift` cells with the global spline (eq. tridiagsys)."""
    lib = _load()
    line = _f64(line)
    out = np.empty_like(line)
    lib.oracle_interpolate_line_gs(_ptr(line), _ptr(out), line.size, float(shift), int(bc), int(storage))
    return out


def ring_tables(p):
    lib = _load()
    P = _params(p)
    dV = np.array([lib.oracle_ring_dV(C.byref(P), s) for s in range(p.nx)])
    V = np.array([lib.oracle_ring_V(C.byref(P), s) for s in range(p.nx)])
    return dV, V
