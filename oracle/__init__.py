"""CPU oracle for the pseudo-projection sweep -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never imports, links or calls it, and it
shares no code with the GPU library.

The arithmetic lives in ``modap_oracle.c`` (plain loops, FP64 data,
extended-precision accumulation); this module only builds it with gcc and
marshals numpy arrays.  ``brute`` holds exhaustive checks for n <= 3.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "modap_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_DT = {"f64": 0, "f32": 1, "bf16": 2}

STATUS = {0: "converged", 1: "step_limit", 2: "no_direction", 3: "bad_row"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE semantics: no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    """The compiled oracle.  MODAP_ORACLE_LIB may name another build of the same
    source (the sanitizer test runs the pins against an ASan/UBSan build)."""
    global _lib
    if _lib is None:
        alt = os.environ.get("MODAP_ORACLE_LIB")
        if alt:
            L = C.CDLL(alt)
        else:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            L = C.CDLL(_LIB)
        i64, dp, vp, ip = C.c_int64, C.POINTER(C.c_double), C.c_void_p, C.POINTER(C.c_int64)
        L.oracle_norms.argtypes = [i64, i64, C.c_int, vp, i64, dp]
        L.oracle_norms.restype = i64
        L.oracle_translate.argtypes = [i64, i64, C.c_int, vp, i64, dp, dp]
        L.oracle_translate.restype = None
        L.oracle_sweep.argtypes = [i64, i64, C.c_int, vp, i64, dp, dp, dp, dp, dp, dp, ip, dp, dp]
        L.oracle_sweep.restype = None
        L.oracle_step.argtypes = [i64, dp, i64, C.c_int, C.c_double, dp]
        L.oracle_step.restype = C.c_int
        L.oracle_solve.argtypes = [i64, i64, C.c_int, vp, i64, dp, dp, C.c_double, C.c_double,
                                   C.c_int, C.c_int, i64, dp, i64, i64, ip, dp, ip, dp, dp]
        L.oracle_solve.restype = C.c_int
        L.oracle_replace_rows.argtypes = [i64, C.c_int, vp, i64, dp, i64, ip, vp, dp]
        L.oracle_replace_rows.restype = None
        _lib = L
    return _lib


def _d(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, n=None):
    out = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None:
        assert out.shape == (n,), (out.shape, n)
    return out


def _A(A):
    A = np.ascontiguousarray(A)
    assert A.ndim == 2
    return A


@dataclass
class Sweep:
    r: np.ndarray       # [m] residuals <a_i,x> - b_i
    t: np.ndarray       # [m] rounding scale sum_j |a_ij x_j| + |b_i|
    y: np.ndarray       # [n] sum of positive slices
    h: int              # number of violated rows
    dmax: float         # max distance to a violated half-space
    binf: float         # max |b_i|
    nu: np.ndarray      # [m] ||a_i||^2


def norms(A, dtype):
    A = _A(A)
    m, n = A.shape
    nu = np.empty(m)
    bad = lib().oracle_norms(m, n, _DT[dtype], A.ctypes.data, n, _d(nu))
    return nu, int(bad)


def translate(A, dtype, b, v):
    """b + A v (returns a new array)."""
    A = _A(A)
    m, n = A.shape
    bb = _f64(b, m).copy()
    vv = _f64(v, n)
    lib().oracle_translate(m, n, _DT[dtype], A.ctypes.data, n, _d(vv), _d(bb))
    return bb


def sweep(A, dtype, b, x, nu=None) -> Sweep:
    """One sweep at x on (A, b): residuals, positive-slice sum, h, max violation."""
    A = _A(A)
    m, n = A.shape
    bb, xx = _f64(b, m), _f64(x, n)
    if nu is None:
        nu, _ = norms(A, dtype)
    nu = _f64(nu, m)
    r, t, y = np.empty(m), np.empty(m), np.empty(n)
    h = C.c_int64(0)
    dmax, binf = C.c_double(0), C.c_double(0)
    lib().oracle_sweep(m, n, _DT[dtype], A.ctypes.data, n, _d(bb), _d(nu), _d(xx),
                       _d(r), _d(t), _d(y), C.byref(h), C.byref(dmax), C.byref(binf))
    return Sweep(r, t, y, int(h.value), float(dmax.value), float(binf.value), nu)


def sweep_rows(A, dtype, b, x, rows):
    """Residuals and scales for a subset of rows only (for sampled checks at full size)."""
    A = _A(A)
    rows = np.asarray(rows, dtype=np.int64)
    sub = np.ascontiguousarray(A[rows])
    s = sweep(sub, dtype, np.asarray(b)[rows], x)
    return s


def step(y, h, rule, lam, x):
    """x - lambda*y/||y|| (rule 0) or x - (lambda/h)*y (rule 1); returns (x', status)."""
    xx = _f64(x).copy()
    yy = _f64(y, xx.shape[0])
    st = lib().oracle_step(xx.shape[0], _d(yy), int(h), int(rule), float(lam), _d(xx))
    return xx, int(st)


@dataclass
class Solve:
    status: int
    iters: int
    x: np.ndarray
    b: np.ndarray
    dmax: float
    h: int
    dmax_trace: np.ndarray | None
    x_trace: np.ndarray | None


def solve(A, dtype, b, x0, lam=1.0, eps=1e-6, eps_relative=True, rule=0,
          max_steps=10000, V=None, trace=False, x_trace=False) -> Solve:
    """ModAP (rule 0) or relaxed Algorithm 1 (rule 1) to eps-feasibility."""
    A = _A(A)
    m, n = A.shape
    bb = _f64(b, m).copy()
    xx = _f64(x0, n).copy()
    Vp, T, ldv = None, 0, n
    if V is not None:
        Vp = np.ascontiguousarray(V, dtype=np.float64)
        assert Vp.ndim == 2 and Vp.shape[1] == n
        T = Vp.shape[0]
    it, hh = C.c_int64(0), C.c_int64(0)
    dm = C.c_double(0)
    dtr = np.zeros(max_steps + 1) if trace else None
    xtr = np.zeros((max_steps + 1, n)) if x_trace else None
    st = lib().oracle_solve(m, n, _DT[dtype], A.ctypes.data, n, _d(bb), _d(xx), float(lam),
                            float(eps), int(bool(eps_relative)), int(rule), int(max_steps),
                            _d(Vp), T, ldv, C.byref(it), C.byref(dm), C.byref(hh),
                            _d(dtr), None if xtr is None else _d(xtr))
    k = int(it.value)
    return Solve(int(st), k, xx, bb, float(dm.value), int(hh.value),
                 None if dtr is None else dtr[:k + 1],
                 None if xtr is None else xtr[:k + 1])


def replace_rows(A, dtype, b, rows, new_rows, new_b):
    """Row replacement; returns new (A, b) copies."""
    A2 = _A(A).copy()
    b2 = _f64(b).copy()
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    nr = np.ascontiguousarray(new_rows, dtype=A2.dtype)
    nb = _f64(new_b)
    lib().oracle_replace_rows(A2.shape[1], _DT[dtype], A2.ctypes.data, A2.shape[1], _d(b2),
                              rows.shape[0], rows.ctypes.data_as(C.POINTER(C.c_int64)),
                              nr.ctypes.data, _d(nb))
    return A2, b2
