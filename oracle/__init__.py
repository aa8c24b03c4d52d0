"""FP64 CPU oracle (test infrastructure only).

A thin ctypes wrapper around ``oracle.c``: the plain, slow reference that the
GPU library is checked against.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg import this package; the product library never
does.  It shares no code with the HIP path.

Arrays follow the C side: ``m`` is ``(N,)``, ``x`` and ``v`` are ``(3, N)``
structure-of-arrays float64, results for an active list are ``(3, n_act)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "oracle.c"
_LIB = _HERE / "liboracle.so"

OK = 0
E_INVAL = -1
E_DTMIN = -5
E_NONFINITE = -6

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC", "-std=c11"]


def build(force: bool = True) -> Path:
    """Compile liboracle.so with gcc (no FMA contraction)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp")
        subprocess.run(["gcc", *CFLAGS, "-o", str(tmp), str(_SRC), "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_lib_path: Path | None = None


def use_library(path) -> None:
    """Load the oracle from another build of oracle.c (the mutation tests use
    this to check that deliberately broken builds fail the pins)."""
    global _lib, _lib_path
    _lib, _lib_path = None, Path(path)


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        path = _lib_path
        if path is None:
            if not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
                build(force=True)
            path = _LIB
        L = ctypes.CDLL(str(path))
        i64, f64, p = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        L.oracle_threads.argtypes = []
        L.oracle_threads.restype = ctypes.c_int
        L.oracle_force.argtypes = [i64, p, p, p, f64, i64, p, p, p, p]
        L.oracle_force.restype = None
        L.oracle_force_sliced.argtypes = [i64, p, p, p, f64, i64, i64, p, p, p, p]
        L.oracle_force_sliced.restype = None
        L.oracle_force_abs.argtypes = [i64, p, p, p, f64, i64, p, p]
        L.oracle_force_abs.restype = None
        L.oracle_perturbers.argtypes = [i64, p, p, f64, f64, i64, p, ctypes.c_int32, p, p]
        L.oracle_perturbers.restype = None
        L.oracle_predict.argtypes = [i64, p, p, p, p, p, f64, p, p]
        L.oracle_predict.restype = None
        L.oracle_correct_one.argtypes = [f64, p, p, p, p, p, p, p, p, p, p]
        L.oracle_correct_one.restype = None
        L.oracle_aarseth_dt.argtypes = [f64, p, p, p, p, f64]
        L.oracle_aarseth_dt.restype = f64
        L.oracle_pow2_floor.argtypes = [f64]
        L.oracle_pow2_floor.restype = f64
        L.oracle_quantize.argtypes = [f64, f64, f64, f64, f64, ctypes.POINTER(ctypes.c_int)]
        L.oracle_quantize.restype = f64
        L.oracle_initial_dt.argtypes = [f64, p, p, f64, f64, ctypes.POINTER(ctypes.c_int)]
        L.oracle_initial_dt.restype = f64
        L.oracle_start.argtypes = [i64, p, p, p, f64, f64, f64, f64, p, p, p, p]
        L.oracle_start.restype = ctypes.c_int
        L.oracle_select.argtypes = [i64, p, p, ctypes.POINTER(f64), p]
        L.oracle_select.restype = i64
        L.oracle_block_step.argtypes = [i64, p, p, p, p, p, p, p, f64, f64, f64, f64, p, p,
                                        ctypes.POINTER(f64)]
        L.oracle_block_step.restype = i64
        L.oracle_run.argtypes = [i64, p, p, p, p, p, p, p, f64, f64, f64, f64, f64, i64,
                                 ctypes.POINTER(f64), ctypes.POINTER(f64)]
        L.oracle_run.restype = i64
        L.oracle_diagnostics.argtypes = [i64, p, p, p, f64, p]
        L.oracle_diagnostics.restype = None
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = None
        _lib = L
    return _lib


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().oracle_threads())


def set_threads(n: int) -> None:
    """Number of OpenMP threads for the oracle's parallel loops."""
    lib().oracle_set_threads(int(n))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def force(m, x, v, eps: float, active=None, slices: int | None = None):
    """Acceleration, jerk, potential on ``active`` (default: all) from all particles.

    Returns ``(acc, jerk, pot)`` with shapes ``(3, n_act), (3, n_act), (n_act,)``.
    With ``slices=p`` the j range is summed in p contiguous slices added in
    slice order (the paper's j-parallel partition, emulated)."""
    m, x, v = _f64(m), _f64(x), _f64(v)
    n = m.shape[0]
    assert x.shape == (3, n) and v.shape == (3, n)
    act = np.arange(n, dtype=np.int32) if active is None else np.ascontiguousarray(active, dtype=np.int32)
    na = act.shape[0]
    acc = np.zeros((3, na))
    jerk = np.zeros((3, na))
    pot = np.zeros(na)
    if slices is None:
        lib().oracle_force(n, _ptr(m), _ptr(x), _ptr(v), float(eps), na, _ptr(act), _ptr(acc),
                           _ptr(jerk), _ptr(pot))
    else:
        lib().oracle_force_sliced(n, _ptr(m), _ptr(x), _ptr(v), float(eps), int(slices), na,
                                  _ptr(act), _ptr(acc), _ptr(jerk), _ptr(pot))
    return acc, jerk, pot


def force_abs(m, x, v, eps: float, active=None) -> np.ndarray:
    """(3, n_act): sums of |acceleration term|, |jerk term| and |potential
    term| over j -- the scale that rounding errors are measured against."""
    m, x, v = _f64(m), _f64(x), _f64(v)
    n = m.shape[0]
    act = np.arange(n, dtype=np.int32) if active is None else np.ascontiguousarray(active, dtype=np.int32)
    out = np.zeros((3, act.shape[0]))
    lib().oracle_force_abs(n, _ptr(m), _ptr(x), _ptr(v), float(eps), act.shape[0], _ptr(act), _ptr(out))
    return out


def perturbers(m, x, eps: float, thr: float, active=None, cap: int = 256):
    """Perturber lists (Sect. 3.1): for each active i the j != i with
    m_j / (|x_j - x_i|^2 + eps^2) > thr, in ascending j, at most ``cap`` of
    them.  Returns ``(lists, counts)``: lists (n_act, cap) int32 padded with
    -1, counts (n_act,) the number of j that pass (also beyond cap)."""
    m, x = _f64(m), _f64(x)
    n = m.shape[0]
    act = np.arange(n, dtype=np.int32) if active is None else np.ascontiguousarray(active, dtype=np.int32)
    na = act.shape[0]
    lists = np.empty((na, cap), dtype=np.int32)
    counts = np.empty(na, dtype=np.int32)
    lib().oracle_perturbers(n, _ptr(m), _ptr(x), float(eps), float(thr), na, _ptr(act), int(cap), _ptr(lists),
                            _ptr(counts))
    return lists, counts


def predict(x, v, a, k, t, t_pred: float):
    x, v, a, k, t = _f64(x), _f64(v), _f64(a), _f64(k), _f64(t)
    n = t.shape[0]
    xp = np.empty((3, n))
    vp = np.empty((3, n))
    lib().oracle_predict(n, _ptr(x), _ptr(v), _ptr(a), _ptr(k), _ptr(t), float(t_pred), _ptr(xp), _ptr(vp))
    return xp, vp


def correct_one(h: float, a0, k0, a1, k1, xp, vp):
    """Corrector for one particle; returns (x, v, a2, a3)."""
    args = [_f64(u).reshape(3) for u in (a0, k0, a1, k1, xp, vp)]
    outs = [np.empty(3) for _ in range(4)]
    lib().oracle_correct_one(float(h), *[_ptr(a) for a in args], *[_ptr(o) for o in outs])
    return tuple(outs)


def aarseth_dt(eta: float, a1, k1, a2, a3, h: float) -> float:
    args = [_f64(u).reshape(3) for u in (a1, k1, a2, a3)]
    return lib().oracle_aarseth_dt(float(eta), *[_ptr(a) for a in args], float(h))


def pow2_floor(x: float) -> float:
    return lib().oracle_pow2_floor(float(x))


def quantize(dt_raw: float, dt_old: float, t_now: float, dt_max: float, dt_min: float):
    """Returns ``(dt_new, status)``."""
    st = ctypes.c_int(0)
    r = lib().oracle_quantize(float(dt_raw), float(dt_old), float(t_now), float(dt_max),
                              float(dt_min), ctypes.byref(st))
    return r, st.value


def initial_dt(eta_s: float, a, k, dt_max: float, dt_min: float):
    st = ctypes.c_int(0)
    a, k = _f64(a).reshape(3), _f64(k).reshape(3)
    r = lib().oracle_initial_dt(float(eta_s), _ptr(a), _ptr(k), float(dt_max), float(dt_min), ctypes.byref(st))
    return r, st.value


def diagnostics(m, x, v, eps: float) -> dict:
    """Softened energy, linear and angular momentum (FP64)."""
    m, x, v = _f64(m), _f64(x), _f64(v)
    out = np.empty(8)
    lib().oracle_diagnostics(m.shape[0], _ptr(m), _ptr(x), _ptr(v), float(eps), _ptr(out))
    return {"KE": out[0], "PE": out[1], "E": out[0] + out[1], "P": out[2:5].copy(), "L": out[5:8].copy()}


class Sim:
    """A single cluster advanced by the oracle's block-step Hermite integrator."""

    def __init__(self, m, x, v, eps: float, eta: float = 0.01, eta_s: float = 0.01,
                 dt_max: float = 2.0**-3, dt_min: float = 2.0**-40):
        self.m = _f64(m).copy()
        self.x = _f64(x).copy()
        self.v = _f64(v).copy()
        self.n = self.m.shape[0]
        self.eps, self.eta, self.eta_s = float(eps), float(eta), float(eta_s)
        self.dt_max, self.dt_min = float(dt_max), float(dt_min)
        n = self.n
        self.a = np.zeros((3, n))
        self.k = np.zeros((3, n))
        self.t = np.zeros(n)
        self.dt = np.zeros(n)
        self.work = np.zeros(13 * n)
        self.act = np.zeros(n, dtype=np.int32)
        self.steps = 0
        self.interactions = 0.0
        self.time = 0.0
        st = lib().oracle_start(n, _ptr(self.m), _ptr(self.x), _ptr(self.v), self.eps, self.eta_s,
                                self.dt_max, self.dt_min, _ptr(self.a), _ptr(self.k), _ptr(self.t),
                                _ptr(self.dt))
        if st != OK:
            raise RuntimeError(f"oracle start failed: {st}")

    def block_step(self) -> np.ndarray:
        """One block step; returns the block (ascending particle indices)."""
        ts = ctypes.c_double(0.0)
        nb = lib().oracle_block_step(self.n, _ptr(self.m), _ptr(self.x), _ptr(self.v), _ptr(self.a),
                                     _ptr(self.k), _ptr(self.t), _ptr(self.dt), self.eps, self.eta,
                                     self.dt_max, self.dt_min, _ptr(self.work), _ptr(self.act),
                                     ctypes.byref(ts))
        if nb < 0:
            raise RuntimeError(f"oracle block step failed: {nb}")
        self.steps += 1
        self.interactions += nb * self.n
        self.time = ts.value
        return self.act[:nb].copy()

    def run(self, t_end: float, max_steps: int = 1 << 40) -> int:
        """Block steps until every particle reaches t_end (a multiple of dt_max)."""
        ni = ctypes.c_double(0.0)
        tr = ctypes.c_double(0.0)
        s = lib().oracle_run(self.n, _ptr(self.m), _ptr(self.x), _ptr(self.v), _ptr(self.a),
                             _ptr(self.k), _ptr(self.t), _ptr(self.dt), self.eps, self.eta,
                             self.dt_max, self.dt_min, float(t_end), int(max_steps),
                             ctypes.byref(ni), ctypes.byref(tr))
        if s < 0:
            raise RuntimeError(f"oracle run failed: {s}")
        self.steps += s
        self.interactions += ni.value
        self.time = tr.value
        return s

    def diagnostics(self) -> dict:
        return diagnostics(self.m, self.x, self.v, self.eps)
