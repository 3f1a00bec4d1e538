"""Python binding of libmodap (the MI355X pseudo-projection sweep library).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  Arrays may be numpy arrays (host memory) or torch tensors on the
context's GPU (device memory); all arrays of one call must be on the same
side.  PyTorch supplies device memory and the stream; it computes nothing here.

There is no CPU fallback: if the compiled library is missing, importing
``lib()`` raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmodap.so")

F64, F32, BF16 = 0, 1, 2
DTYPES = {"f64": F64, "f32": F32, "bf16": BF16}
STEP_FIXED, STEP_AVG = 0, 1

OK = 0
STATUS_NAMES = {0: "OK", 1: "E_INVAL", 2: "E_ZERO_ROW", 3: "E_NOMEM", 4: "E_DEVICE", 5: "E_STATE",
                6: "E_NOT_CONVERGED", 7: "E_INFEASIBLE", 8: "E_NUMERIC"}
STATE_NAMES = {0: "running", 1: "converged", 2: "no_direction", 3: "numeric", 4: "step_limit", 5: "bad_row",
               6: "uncertified"}

# every symbol declared in include/modap.h
EXPORTS = ["modap_create", "modap_destroy", "modap_set_system", "modap_set_x", "modap_update_coeffs",
           "modap_set_drift", "modap_iterate", "modap_solve", "modap_eval_sweep", "modap_query",
           "modap_set_tile", "modap_get_tile", "modap_autotune", "modap_strerror", "modap_last_error",
           "modap_batch_create", "modap_batch_destroy", "modap_batch_add", "modap_batch_remove",
           "modap_batch_set_drift", "modap_batch_update", "modap_batch_iterate", "modap_batch_solve",
           "modap_batch_query", "modap_batch_set_tile", "modap_batch_get_tile", "modap_batch_autotune",
           "modap_batch_last_error", "modap_server_create", "modap_server_destroy", "modap_server_submit",
           "modap_server_update", "modap_server_round", "modap_server_info", "modap_server_result",
           "modap_server_totals", "modap_server_last_error", "modap_server_set_max_live",
           "modap_server_set_max_long", "modap_server_release",
           "modap_eval_sweep_static"]


class Params(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("eps", C.c_double), ("eps_relative", C.c_int32),
                ("step", C.c_int32), ("max_iters", C.c_int64), ("profile", C.c_int32),
                ("track", C.c_int32), ("certify", C.c_int32), ("pad", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int64), ("sweeps", C.c_int64), ("converged", C.c_int32),
                ("state", C.c_int32), ("max_viol", C.c_double), ("h", C.c_int64),
                ("y_norm", C.c_double), ("b_inf", C.c_double), ("eps_abs", C.c_double),
                ("seconds", C.c_double), ("hbm_bytes", C.c_double), ("sweep_ms", C.c_double),
                ("reduce_ms", C.c_double), ("profiled", C.c_int64), ("certified", C.c_int32),
                ("resident", C.c_int32), ("b_drift", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}
        d["state_name"] = STATE_NAMES.get(self.state, "?")
        return d


class Tile(C.Structure):
    _fields_ = [("kind", C.c_int32), ("block", C.c_int32), ("lanes_per_row", C.c_int32),
                ("chunks", C.c_int32), ("grid", C.c_int32), ("rows_per_step", C.c_int32),
                ("depth", C.c_int32), ("interleave", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchStats(C.Structure):
    _fields_ = [("iters", C.c_int64), ("running", C.c_int64), ("systems", C.c_int64),
                ("seconds", C.c_double), ("hbm_bytes", C.c_double), ("sweep_ms", C.c_double),
                ("reduce_ms", C.c_double), ("profiled", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchTile(C.Structure):
    _fields_ = [("item_kib", C.c_int32 * 4), ("grid", C.c_int32), ("min_items", C.c_int32)]

    def as_dict(self):
        return {"item_kib": list(self.item_kib), "grid": self.grid, "min_items": self.min_items}


class RequestInfo(C.Structure):
    _fields_ = [("state", C.c_int32), ("status", C.c_int32), ("batched", C.c_int32), ("pad", C.c_int32),
                ("iters", C.c_int64), ("sweeps", C.c_int64), ("max_viol", C.c_double), ("eps_abs", C.c_double),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("hbm_bytes", C.c_double), ("footprint", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}
        d["state_name"] = ("queued", "live", "done", "failed")[self.state]
        return d


class ModapError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def lib():
    """Load libmodap.so (raises when it has not been built).

    PyTorch, when it is installed, is imported first: its wheel carries a HIP
    runtime of its own, which it loads by path.  Loaded after the library
    (whose runtime is found by soname), it would map a second HIP runtime into
    the process, and the two would not share devices, streams or memory.
    Imported first, its runtime is the one the library's dependency resolves to.
    """
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              f"`python -m paper_2003_09956_amd._build` (no CPU fallback exists)")
        try:
            import torch  # noqa: F401  (one HIP runtime in the process: see above)
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, dp = C.c_void_p, C.c_int64, C.c_int, C.c_void_p
        L.modap_create.argtypes = [i32, vp, C.POINTER(vp)]
        L.modap_destroy.argtypes = [vp]
        L.modap_destroy.restype = None
        L.modap_set_system.argtypes = [vp, i64, i64, i32, vp, i64, dp, dp, i32]
        L.modap_set_x.argtypes = [vp, dp, i32]
        L.modap_update_coeffs.argtypes = [vp, i64, vp, vp, dp, dp, i32]
        L.modap_set_drift.argtypes = [vp, i64, dp, i64, i32]
        L.modap_iterate.argtypes = [vp, C.POINTER(Params), i64, C.POINTER(Stats)]
        L.modap_solve.argtypes = [vp, C.POINTER(Params), C.POINTER(Stats)]
        L.modap_eval_sweep.argtypes = [vp, dp, dp, dp, C.POINTER(C.c_int64), C.POINTER(C.c_double), i32]
        L.modap_query.argtypes = [vp, dp, dp, C.POINTER(Stats), i32]
        L.modap_set_tile.argtypes = [vp, C.POINTER(Tile)]
        L.modap_get_tile.argtypes = [vp, C.POINTER(Tile)]
        L.modap_autotune.argtypes = [vp, i32, C.POINTER(Tile)]
        L.modap_strerror.argtypes = [i32]
        L.modap_strerror.restype = C.c_char_p
        L.modap_last_error.argtypes = [vp]
        L.modap_last_error.restype = C.c_char_p
        L.modap_batch_create.argtypes = [i32, vp, i32, C.POINTER(vp)]
        L.modap_batch_destroy.argtypes = [vp]
        L.modap_batch_destroy.restype = None
        L.modap_batch_add.argtypes = [vp, i64, i64, vp, i64, dp, dp, i32, C.POINTER(C.c_int64)]
        L.modap_batch_remove.argtypes = [vp, i64]
        L.modap_batch_set_drift.argtypes = [vp, i64, i64, dp, i64, i32]
        L.modap_batch_update.argtypes = [vp, i64, i64, vp, vp, dp, dp, i32]
        L.modap_batch_iterate.argtypes = [vp, C.POINTER(Params), i64, C.POINTER(BatchStats)]
        L.modap_batch_solve.argtypes = [vp, C.POINTER(Params), C.POINTER(BatchStats)]
        L.modap_batch_query.argtypes = [vp, i64, dp, dp, C.POINTER(Stats), i32]
        L.modap_batch_set_tile.argtypes = [vp, C.POINTER(BatchTile)]
        L.modap_batch_get_tile.argtypes = [vp, C.POINTER(BatchTile)]
        L.modap_batch_autotune.argtypes = [vp, i32, C.POINTER(BatchTile)]
        L.modap_batch_last_error.argtypes = [vp]
        L.modap_batch_last_error.restype = C.c_char_p
        L.modap_server_create.argtypes = [i32, i32, C.c_double, C.POINTER(Params), i32, C.POINTER(vp)]
        L.modap_server_destroy.argtypes = [vp]
        L.modap_server_destroy.restype = None
        L.modap_server_submit.argtypes = [vp, i64, i64, vp, dp, dp, i64, dp, i64, i32, C.c_double,
                                          C.POINTER(C.c_int64)]
        L.modap_server_update.argtypes = [vp, i64, i64, vp, vp, dp, dp, i32]
        L.modap_server_round.argtypes = [vp, C.c_double, C.POINTER(C.c_int64)]
        L.modap_server_info.argtypes = [vp, i64, C.POINTER(RequestInfo)]
        L.modap_server_result.argtypes = [vp, i64, dp]
        L.modap_server_release.argtypes = [vp, i64]
        L.modap_server_totals.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.modap_server_last_error.argtypes = [vp]
        L.modap_server_last_error.restype = C.c_char_p
        L.modap_server_set_max_live.argtypes = [vp, i64]
        L.modap_server_set_max_long.argtypes = [vp, i64]
        L.modap_eval_sweep_static.argtypes = [i32, vp, i64, i64, i32, vp, i64, dp, dp, dp, dp, dp, dp]
        for name in EXPORTS:
            if name not in ("modap_destroy", "modap_strerror", "modap_last_error", "modap_batch_destroy",
                            "modap_batch_last_error", "modap_server_destroy", "modap_server_last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def params(lam=1.0, eps=1e-6, eps_relative=True, step=STEP_FIXED, max_iters=100000, profile=0,
           track=False, certify=True):
    """profile: 0 = no timing, k = time every k-th iteration (True = every iteration).
    certify: confirm every stop at eps-feasibility with the library's FP64 certificate."""
    return Params(float(lam), float(eps), int(bool(eps_relative)), int(step), int(max_iters),
                  int(profile), int(bool(track)), int(bool(certify)), 0)


def eval_sweep_static(A, b, x, y, dtype="f32", r=None, h=None, max_viol=None, lda=None, device=0, stream=None):
    """modap_eval_sweep_static: one sweep with no allocation.  Every array is a
    torch tensor on `device` (A [m x lda] zero-padded, b [m], x [n], outputs y [n]
    and optionally r [m], h (int64 [1]) and max_viol (float64 [1])); the work is
    queued on `stream` (default: torch's current stream) and not waited for."""
    code = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    m = int(A.shape[0])
    n = int(x.shape[0])
    lda = int(A.shape[1]) if lda is None else int(lda)
    if stream is None:
        import torch
        stream = torch.cuda.current_stream(device).cuda_stream
    g = _Args(device)
    pa = g.ptr(A, _NP_STORE[code], m * lda)
    pb = g.ptr(b, np.float64, m)
    px = g.ptr(x, np.float64, n)
    py = g.ptr(y, np.float64, n)
    pr = g.ptr(r, np.float64, m)
    ph = g.ptr(h, np.int64, 1)
    pd = g.ptr(max_viol, np.float64, 1)
    if g.on_dev != 1:
        raise ValueError("eval_sweep_static takes device tensors only")
    st = lib().modap_eval_sweep_static(int(device), C.c_void_p(int(stream)) if stream else None, m, n, code, pa, lda,
                                       pb, px, pr, py, ph, pd)
    if st != OK:
        raise ModapError(st, lib().modap_strerror(st).decode())


def _is_torch(a):
    return type(a).__module__.startswith("torch")


class _Args:
    """Collects the pointers of one call and checks they are all host or all device."""

    def __init__(self, device):
        self.device = device
        self.side = None
        self.keep = []

    def ptr(self, a, np_dtype, count=None):
        if a is None:
            return None
        if _is_torch(a):
            if a.is_cuda:
                side = 1
                if a.device.index != self.device:
                    raise ValueError(f"tensor on cuda:{a.device.index}, context on device {self.device}")
                if not a.is_contiguous():
                    raise ValueError("device tensors must be contiguous")
                want = {np.float64: "torch.float64", np.float32: "torch.float32",
                        np.uint16: ("torch.int16", "torch.uint16", "torch.bfloat16"),
                        np.int64: "torch.int64"}[np_dtype]
                if str(a.dtype) not in (want if isinstance(want, tuple) else (want,)):
                    raise TypeError(f"tensor dtype {a.dtype} does not match {np_dtype}")
                if count is not None and a.numel() < count:
                    raise ValueError(f"tensor has {a.numel()} elements, {count} needed")
                self.keep.append(a)
                p = a.data_ptr()
            else:
                side = 0
                a = a.numpy()
        if not _is_torch(a):
            side = 0
            arr = np.ascontiguousarray(a)
            if arr.dtype != np_dtype:
                if np_dtype == np.uint16:
                    raise TypeError("bf16 data must be uint16 bit patterns")
                arr = arr.astype(np_dtype)
            if count is not None and arr.size < count:
                raise ValueError(f"array has {arr.size} elements, {count} needed")
            self.keep.append(arr)
            p = arr.ctypes.data
        if self.side is None:
            self.side = side
        elif self.side != side:
            raise ValueError("all arrays of one call must be host arrays or all device tensors")
        return p

    @property
    def on_dev(self):
        return int(self.side or 0)


_NP_STORE = {F64: np.float64, F32: np.float32, BF16: np.uint16}


@dataclass
class SweepResult:
    y: object
    r: object
    h: int
    max_viol: float


class Solver:
    """One library context: a system A x <= b on one GPU and its iteration state."""

    def __init__(self, device: int = 0, stream=None):
        L = lib()
        self.device = int(device)
        if stream is None:
            try:
                import torch
                stream = torch.cuda.current_stream(self.device).cuda_stream
            except Exception:
                stream = None
        ctx = C.c_void_p()
        st = L.modap_create(self.device, C.c_void_p(int(stream)) if stream else None, C.byref(ctx))
        if st != OK:
            raise ModapError(st, L.modap_strerror(st).decode())
        self._ctx = ctx
        self.m = self.n = 0
        self.dtype = None

    # ------------------------------------------------------------- plumbing
    def close(self):
        if getattr(self, "_ctx", None):
            lib().modap_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st):
        if st != OK:
            raise ModapError(st, lib().modap_last_error(self._ctx).decode())

    # ------------------------------------------------------------- API
    def set_system(self, A, b, x0=None, dtype="f32"):
        code = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        m, n = int(A.shape[0]), int(A.shape[1])
        g = _Args(self.device)
        pa = g.ptr(A, _NP_STORE[code], m * n)
        pb = g.ptr(b, np.float64, m)
        px = g.ptr(x0, np.float64, n)
        self._check(lib().modap_set_system(self._ctx, m, n, code, pa, n, pb, px, g.on_dev))
        self.m, self.n, self.dtype = m, n, code

    def set_x(self, x=None):
        g = _Args(self.device)
        self._check(lib().modap_set_x(self._ctx, g.ptr(x, np.float64, self.n), g.on_dev))

    def update_coeffs(self, rows=None, new_rows=None, new_b=None, translate=None):
        g = _Args(self.device)
        k = 0 if rows is None else int(len(rows))
        pr = g.ptr(rows, np.int64, k) if k else None
        pn = g.ptr(new_rows, _NP_STORE[self.dtype], k * self.n) if k else None
        pb = g.ptr(new_b, np.float64, k) if k else None
        pv = g.ptr(translate, np.float64, self.n)
        self._check(lib().modap_update_coeffs(self._ctx, k, pr, pn, pb, pv, g.on_dev))

    def set_drift(self, V=None):
        g = _Args(self.device)
        T = 0 if V is None else int(V.shape[0])
        pv = g.ptr(V, np.float64, T * self.n) if T else None
        self._check(lib().modap_set_drift(self._ctx, T, pv, self.n, g.on_dev))

    def iterate(self, k, prm=None, stats=True):
        prm = prm or params()
        out = Stats() if stats else None
        st = lib().modap_iterate(self._ctx, C.byref(prm), int(k), C.byref(out) if stats else None)
        self._check(st)
        return out

    def solve(self, prm=None, raise_on_stop=True):
        prm = prm or params()
        out = Stats()
        st = lib().modap_solve(self._ctx, C.byref(prm), C.byref(out))
        if raise_on_stop:
            self._check(st)
        return out, st

    def eval_sweep(self, x, want_r=True, y_out=None, r_out=None):
        """One stateless sweep at x (host or device) on the current data."""
        dev = _is_torch(x) and x.is_cuda
        if dev:
            import torch
            y_out = y_out if y_out is not None else torch.empty(self.n, dtype=torch.float64, device=x.device)
            if want_r:
                r_out = r_out if r_out is not None else torch.empty(self.m, dtype=torch.float64, device=x.device)
        else:
            y_out = np.empty(self.n) if y_out is None else y_out
            if want_r:
                r_out = np.empty(self.m) if r_out is None else r_out
        g = _Args(self.device)
        px = g.ptr(x, np.float64, self.n)
        py = g.ptr(y_out, np.float64, self.n)
        pr = g.ptr(r_out, np.float64, self.m) if want_r else None
        h = C.c_int64(0)
        dm = C.c_double(0)
        self._check(lib().modap_eval_sweep(self._ctx, px, pr, py, C.byref(h), C.byref(dm), g.on_dev))
        return SweepResult(y_out, r_out if want_r else None, int(h.value), float(dm.value))

    def query(self, want_x=True, want_b=False):
        x = np.empty(self.n) if want_x else None
        b = np.empty(self.m) if want_b else None
        out = Stats()
        g = _Args(self.device)
        px = g.ptr(x, np.float64) if want_x else None
        pb = g.ptr(b, np.float64) if want_b else None
        self._check(lib().modap_query(self._ctx, px, pb, C.byref(out), 0))
        return x, b, out

    def set_tile(self, block=None, lanes_per_row=None, chunks=None, grid=0, rows_per_step=1, kind=0, depth=0,
                 interleave=0):
        if block is None:
            self._check(lib().modap_set_tile(self._ctx, None))
            return
        t = Tile(int(kind), int(block), int(lanes_per_row), int(chunks), int(grid), int(rows_per_step), int(depth),
                 int(interleave))
        self._check(lib().modap_set_tile(self._ctx, C.byref(t)))

    def autotune(self, reps=5):
        """Time every compiled sweep shape for the loaded system and keep the fastest."""
        t = Tile()
        self._check(lib().modap_autotune(self._ctx, int(reps), C.byref(t)))
        return t.as_dict()

    def get_tile(self):
        t = Tile()
        self._check(lib().modap_get_tile(self._ctx, C.byref(t)))
        return t.as_dict()


class Batch:
    """Many independent systems of one storage type advanced together: one
    persistent sweep launch and one reduction launch per iteration for all of
    them (modap_batch_* of the C ABI)."""

    def __init__(self, dtype="f32", device: int = 0, stream=None):
        L = lib()
        self.device = int(device)
        self.dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        if stream is None:
            try:
                import torch
                stream = torch.cuda.current_stream(self.device).cuda_stream
            except Exception:
                stream = None
        h = C.c_void_p()
        st = L.modap_batch_create(self.device, C.c_void_p(int(stream)) if stream else None, self.dtype, C.byref(h))
        if st != OK:
            raise ModapError(st, L.modap_strerror(st).decode())
        self._h = h
        self.shapes = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().modap_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st):
        if st != OK:
            raise ModapError(st, lib().modap_batch_last_error(self._h).decode())

    def add(self, A, b, x0=None):
        """Add a system; returns its id."""
        m, n = int(A.shape[0]), int(A.shape[1])
        g = _Args(self.device)
        pa = g.ptr(A, _NP_STORE[self.dtype], m * n)
        pb = g.ptr(b, np.float64, m)
        px = g.ptr(x0, np.float64, n)
        i = C.c_int64()
        self._check(lib().modap_batch_add(self._h, m, n, pa, n, pb, px, g.on_dev, C.byref(i)))
        self.shapes[i.value] = (m, n)
        return i.value

    def remove(self, sid):
        self._check(lib().modap_batch_remove(self._h, int(sid)))
        self.shapes.pop(int(sid), None)

    def set_drift(self, sid, V=None):
        n = self.shapes.get(int(sid), (0, 0))[1]
        g = _Args(self.device)
        T = 0 if V is None else int(V.shape[0])
        pv = g.ptr(V, np.float64, T * n) if T else None
        self._check(lib().modap_batch_set_drift(self._h, int(sid), T, pv, n, g.on_dev))

    def update(self, sid, rows=None, new_rows=None, new_b=None, translate=None):
        n = self.shapes.get(int(sid), (0, 0))[1]
        g = _Args(self.device)
        k = 0 if rows is None else int(len(rows))
        pr = g.ptr(rows, np.int64, k) if k else None
        pn = g.ptr(new_rows, _NP_STORE[self.dtype], k * n) if k else None
        pb = g.ptr(new_b, np.float64, k) if k else None
        pv = g.ptr(translate, np.float64, n)
        self._check(lib().modap_batch_update(self._h, int(sid), k, pr, pn, pb, pv, g.on_dev))

    def iterate(self, k, prm=None, stats=True):
        prm = prm or params()
        out = BatchStats() if stats else None
        self._check(lib().modap_batch_iterate(self._h, C.byref(prm), int(k), C.byref(out) if stats else None))
        return out

    def solve(self, prm=None):
        prm = prm or params()
        out = BatchStats()
        self._check(lib().modap_batch_solve(self._h, C.byref(prm), C.byref(out)))
        return out

    def query(self, sid, want_x=True, want_b=False):
        m, n = self.shapes.get(int(sid), (0, 0))   # an unknown id is reported by the library
        x = np.empty(n) if want_x else None
        b = np.empty(m) if want_b else None
        out = Stats()
        g = _Args(self.device)
        px = g.ptr(x, np.float64) if want_x else None
        pb = g.ptr(b, np.float64) if want_b else None
        self._check(lib().modap_batch_query(self._h, int(sid), px, pb, C.byref(out), 0))
        return x, b, out

    def set_tile(self, item_kib=None, grid=0, min_items=0):
        if item_kib is None:
            # the library's built-in item sizes, with the grid and item count asked for
            self._check(lib().modap_batch_set_tile(self._h, None))
            if grid == 0 and min_items == 0:
                return
            item_kib = self.get_tile()["item_kib"]
        kib = list(item_kib)
        t = BatchTile((C.c_int32 * 4)(*[int(v) for v in kib]), int(grid), int(min_items))
        self._check(lib().modap_batch_set_tile(self._h, C.byref(t)))

    def get_tile(self):
        t = BatchTile()
        self._check(lib().modap_batch_get_tile(self._h, C.byref(t)))
        return t.as_dict()

    def autotune(self, reps=3):
        t = BatchTile()
        self._check(lib().modap_batch_autotune(self._h, int(reps), C.byref(t)))
        return t.as_dict()


class Server:
    """Continuous-batching solve server (modap_server_* of the C ABI).  The
    caller drives it with round(now); the library copies a request's inputs
    when it is submitted."""

    def __init__(self, dtype="bf16", budget_bytes=64e9, prm=None, iters_per_round=8, device: int = 0):
        L = lib()
        self.device = int(device)
        self.dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        prm = prm or params()
        h = C.c_void_p()
        st = L.modap_server_create(self.device, self.dtype, float(budget_bytes), C.byref(prm), int(iters_per_round),
                                   C.byref(h))
        if st != OK:
            raise ModapError(st, L.modap_strerror(st).decode())
        self._h = h
        self.shapes = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().modap_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st):
        if st != OK:
            raise ModapError(st, lib().modap_server_last_error(self._h).decode())

    def submit(self, A, b, x0=None, V=None, now=0.0):
        m, n = int(A.shape[0]), int(A.shape[1])
        g = _Args(self.device)
        pa = g.ptr(A, _NP_STORE[self.dtype], m * n)
        pb = g.ptr(b, np.float64, m)
        px = g.ptr(x0, np.float64, n)
        T = 0 if V is None else int(V.shape[0])
        pv = g.ptr(V, np.float64, T * n) if T else None
        t = C.c_int64()
        self._check(lib().modap_server_submit(self._h, m, n, pa, pb, px, T, pv, n, g.on_dev, float(now),
                                              C.byref(t)))
        self.shapes[t.value] = (m, n)
        return t.value

    def update(self, ticket, rows=None, new_rows=None, new_b=None, translate=None):
        n = self.shapes.get(int(ticket), (0, 0))[1]
        g = _Args(self.device)
        k = 0 if rows is None else int(len(rows))
        pr = g.ptr(rows, np.int64, k) if k else None
        pn = g.ptr(new_rows, _NP_STORE[self.dtype], k * n) if k else None
        pb = g.ptr(new_b, np.float64, k) if k else None
        pv = g.ptr(translate, np.float64, n)
        self._check(lib().modap_server_update(self._h, int(ticket), k, pr, pn, pb, pv, g.on_dev))

    def round(self, now=0.0):
        out = C.c_int64()
        self._check(lib().modap_server_round(self._h, float(now), C.byref(out)))
        return out.value

    def info(self, ticket):
        r = RequestInfo()
        self._check(lib().modap_server_info(self._h, int(ticket), C.byref(r)))
        return r.as_dict()

    def result(self, ticket):
        x = np.empty(self.shapes[int(ticket)][1])
        self._check(lib().modap_server_result(self._h, int(ticket), x.ctypes.data_as(C.c_void_p)))
        return x

    def release(self, ticket):
        """Free the stored result of a finished request (its info stays)."""
        self._check(lib().modap_server_release(self._h, int(ticket)))

    def set_max_live(self, k):
        self._check(lib().modap_server_set_max_live(self._h, int(k)))

    def set_max_long(self, k):
        self._check(lib().modap_server_set_max_long(self._h, int(k)))

    def totals(self):
        b, r, u = C.c_double(), C.c_int64(), C.c_double()
        self._check(lib().modap_server_totals(self._h, C.byref(b), C.byref(r), C.byref(u)))
        return {"hbm_bytes": b.value, "rounds": r.value, "memory_in_use": u.value}
