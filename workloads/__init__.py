"""Seeded synthetic inputs for the pseudo-projection sweep.

This module builds systems ``A x <= b`` and drift schedules and nothing else:
it holds none of the method's arithmetic (no residuals, no positive slices, no
norms of stored rows, no steps).  Both the CPU oracle and the GPU library read
exactly the bytes produced here, so every precision solves the same system.

Workload families (paper section 5 uses its own scalable test system, which is
not reproduced in the text we have; these synthetic families stand in for it):

* ``box_sum`` -- a box ``0 <= x_j <= 200`` plus one aggregate row
  ``sum_j x_j <= 200 (n - 1)``; rows ordered ``[x_j <= 200 ; -x_j <= 0 ; sum]``
  (m = 2n + 1, the same family shape as the paper's m = 2n + 2 system).
  ``x0_j = 400 + U(0, 100)``.
* ``gaussian`` -- rows ``a_i ~ N(0, 1)^n`` normalised to unit length in FP64
  and then rounded (round-to-nearest-even) to the storage type; a hidden point
  ``z ~ U(-1, 1)^n``; ``b = A_stored z + s`` with slack ``s_i ~ U(0, 1)``,
  computed in FP64 from the stored values, so ``z`` is strictly feasible for
  the stored system.  ``x0 = 0``.
* drift -- a per-iteration translation ``v ~ N(0, sigma^2)^n`` (the
  non-stationarity of section 5: the polytope is moved by a translation).

Storage types: ``"f64"``, ``"f32"`` and ``"bf16"`` (BF16 is held as ``uint16``
bit patterns; ``bf16(fp32(a))`` with RNE at each rounding).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

DTYPE_CODES = {"f64": 0, "f32": 1, "bf16": 2}
ELEM_BYTES = {"f64": 8, "f32": 4, "bf16": 2}


# ---------------------------------------------------------------- encodings
def f32_to_bf16_bits(a32: np.ndarray) -> np.ndarray:
    """Round FP32 values to BF16 (round-to-nearest-even); return uint16 bits.

    NaN inputs keep a quiet NaN pattern.  Pure storage encoding.
    """
    a32 = np.ascontiguousarray(a32, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    rounded = (u + 0x7FFF + lsb) >> 16
    nan = np.isnan(a32)
    out = rounded.astype(np.uint16)
    if nan.any():
        out[nan] = ((u[nan] >> 16) | 0x40).astype(np.uint16)
    return out


def bf16_bits_to_f64(bits: np.ndarray) -> np.ndarray:
    """Widen BF16 bit patterns to FP64 exactly (a BF16 is the top half of an FP32)."""
    u32 = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return u32.view(np.float32).astype(np.float64)


def stored_to_f64(A: np.ndarray, dtype: str) -> np.ndarray:
    """Exact FP64 view of a stored matrix (for test-side bookkeeping only)."""
    if dtype == "bf16":
        return bf16_bits_to_f64(A)
    return np.asarray(A, dtype=np.float64)


def encode(A64: np.ndarray, dtype: str) -> np.ndarray:
    """FP64 values -> storage array (RNE; BF16 via FP32)."""
    if dtype == "f64":
        return np.ascontiguousarray(A64, dtype=np.float64)
    a32 = np.ascontiguousarray(A64, dtype=np.float32)
    if dtype == "f32":
        return a32
    if dtype == "bf16":
        return f32_to_bf16_bits(a32)
    raise ValueError(f"unknown storage dtype {dtype!r}")


# ---------------------------------------------------------------- systems
@dataclass
class System:
    """One system ``A x <= b`` in its storage encoding, plus its provenance."""

    A: np.ndarray            # [m, n] storage dtype (uint16 bits for bf16), C-contiguous
    b: np.ndarray            # [m] float64
    x0: np.ndarray           # [n] float64
    dtype: str
    z: np.ndarray | None = None      # a known feasible point (hidden point), if any
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.A.shape[0])

    @property
    def n(self) -> int:
        return int(self.A.shape[1])

    @property
    def nbytes_A(self) -> int:
        return self.m * self.n * ELEM_BYTES[self.dtype]


def _streams(seed: int, family: int):
    ss = np.random.SeedSequence([int(seed), int(family)])
    return [np.random.default_rng(s) for s in ss.spawn(4)]


def box_sum(n: int = 256, seed: int = 0, dtype: str = "f64", upper: float = 200.0) -> System:
    """Box plus aggregate row; m = 2n + 1 (see module docstring)."""
    rng_x = _streams(seed, 1)[0]
    m = 2 * n + 1
    A = np.zeros((m, n), dtype=np.float64)
    A[np.arange(n), np.arange(n)] = 1.0
    A[n + np.arange(n), np.arange(n)] = -1.0
    A[2 * n, :] = 1.0
    b = np.empty(m, dtype=np.float64)
    b[:n] = upper
    b[n:2 * n] = 0.0
    b[2 * n] = upper * (n - 1)
    x0 = 400.0 + rng_x.uniform(0.0, 100.0, size=n)
    z = np.full(n, upper / 2.0)
    return System(encode(A, dtype), b, x0, dtype, z=z,
                  meta={"family": "box_sum", "n": n, "m": m, "seed": seed,
                        "interior_center": upper / 2.0, "interior_radius": upper / 2.0})


def gaussian(n: int, m: int, seed: int = 0, dtype: str = "f32",
             chunk_rows: int = 4096, slack: float = 1.0) -> System:
    """Gaussian system with a hidden strictly feasible point (module docstring).

    Rows are drawn in chunks (the generator stream is identical for any chunk
    size), normalised in FP64 and rounded to the storage type.  ``b`` is formed
    in FP64 from the *stored* values so that the stored system is the system.
    """
    rng_a, rng_z, rng_s, _ = _streams(seed, 2)
    z = rng_z.uniform(-1.0, 1.0, size=n)
    s = rng_s.uniform(0.0, slack, size=m)
    store_np = {"f64": np.float64, "f32": np.float32, "bf16": np.uint16}[dtype]
    A = np.empty((m, n), dtype=store_np)
    b = np.empty(m, dtype=np.float64)
    for r0 in range(0, m, chunk_rows):
        r1 = min(m, r0 + chunk_rows)
        g = rng_a.standard_normal((r1 - r0, n))
        g /= np.sqrt(np.einsum("ij,ij->i", g, g))[:, None]
        enc = encode(g, dtype)
        A[r0:r1] = enc
        b[r0:r1] = stored_to_f64(enc, dtype) @ z + s[r0:r1]
    return System(A, b, np.zeros(n), dtype, z=z,
                  meta={"family": "gaussian", "n": n, "m": m, "seed": seed})


def replacement_rows(sys_: System, k: int, seed: int, z: np.ndarray | None = None):
    """k fresh normalised Gaussian rows with ``b_i = a_i . z + U(0, 1)``.

    Returns (row indices [k] int64, rows [k, n] storage dtype, b [k] float64).
    Keeps ``z`` (default: the system's hidden point) feasible.
    """
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 7, sys_.m, sys_.n]))
    zz = sys_.z if z is None else z
    idx = np.sort(rng.choice(sys_.m, size=k, replace=False)).astype(np.int64)
    g = rng.standard_normal((k, sys_.n))
    g /= np.sqrt(np.einsum("ij,ij->i", g, g))[:, None]
    enc = encode(g, sys_.dtype)
    bb = stored_to_f64(enc, sys_.dtype) @ zz + rng.uniform(0.0, 1.0, size=k)
    return idx, enc, bb


def drift(n: int, steps: int, sigma: float, seed: int = 0) -> np.ndarray:
    """Translation schedule ``V[k] ~ N(0, sigma^2)^n`` (FP64, [steps, n])."""
    rng = _streams(seed, 3)[0]
    return rng.normal(0.0, sigma, size=(steps, n))


def line_drift(n: int, steps: int, per_coord: float) -> np.ndarray:
    """Straight-line translation along (1, ..., 1): ``per_coord`` per step."""
    return np.full((steps, n), float(per_coord))


# ---------------------------------------------------------------- named configurations
def c1(seed: int = 0) -> System:
    """Plain FP64 stationary: n=256, m=513 box-plus-sum, lambda=1, eps=1e-6*||b||inf."""
    return box_sum(256, seed, "f64")


def c2(seed: int = 0, n: int = 8192, m: int = 16384) -> System:
    """FP32 non-stationary Gaussian: n=8192, m=16384 (drift sigma 1e-2 headline)."""
    return gaussian(n, m, seed, "f32")


def c3(seed: int = 0, n: int = 16384, m: int = 65536) -> System:
    """BF16-stored Gaussian: n=16384, m=65536 (2 GiB of A)."""
    return gaussian(n, m, seed, "bf16")


def batch_shapes(count: int = 512, seed: int = 0, n_lo: int = 64, n_hi: int = 2048):
    """Shapes of the batched family: n ~ U{n_lo..n_hi}, m ~ U{2n..8n}."""
    rng = _streams(seed, 4)[0]
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    ms = np.array([rng.integers(2 * k, 8 * k + 1) for k in ns])
    return [(int(a), int(b)) for a, b in zip(ns, ms)]


def serving_arrivals(rate: float, horizon_s: float, seed: int = 0,
                     n_lo: int = 128, n_hi: int = 16384):
    """Poisson arrivals over [0, horizon): list of (t_arrival, n, m=4n, seed)."""
    rng = _streams(seed, 5)[0]
    t, out, k = 0.0, [], 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= horizon_s:
            return out
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        out.append((t, n, 4 * n, int(seed) * 1_000_003 + k))
        k += 1


def gaussian_device(n: int, m: int, seed: int = 0, dtype: str = "f32", device: str = "cuda"):
    """The ``gaussian`` construction generated on the GPU with torch's seeded
    generator (for workloads too large to build on the host quickly; its
    random numbers differ from ``gaussian``'s): rows ~ N(0,1) normalised in
    FP64 and rounded (RNE) to the storage type, ``z ~ U(-1,1)``, and
    ``b = A_stored z + U(0,1)`` in FP64.  Returns (A, b, z) device tensors; a
    BF16 A is a ``torch.bfloat16`` tensor (its bits are the storage)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 7919 + 104729)
    A = torch.randn((m, n), generator=g, device=device, dtype=torch.float64)
    A /= torch.linalg.vector_norm(A, dim=1, keepdim=True)
    A = A.to({"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dtype])
    z = torch.rand(n, generator=g, device=device, dtype=torch.float64) * 2.0 - 1.0
    b = A.to(torch.float64) @ z + torch.rand(m, generator=g, device=device, dtype=torch.float64)
    return A.contiguous(), b.contiguous(), z


def box_sum_device(n: int, dtype: str = "f64", offset: float = 0.0, upper: float = 200.0, device: str = "cuda"):
    """The ``box_sum`` rows built on the GPU (dense; for the large sizes of the
    translation experiment), the polytope translated by ``offset`` along
    (1, ..., 1): rows ``[I; -I; 1^T]``, ``b = [upper + offset; -offset;
    upper (n - 1) + n offset]``.  Returns (A, b) device tensors."""
    import torch
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dtype]
    m = 2 * n + 1
    A = torch.zeros((m, n), device=device, dtype=tdt)
    idx = torch.arange(n, device=device)
    A[idx, idx] = 1
    A[n + idx, idx] = -1
    A[2 * n] = 1
    b = torch.empty(m, device=device, dtype=torch.float64)
    b[:n] = upper + offset
    b[n:2 * n] = -offset
    b[2 * n] = upper * (n - 1) + n * offset
    return A, b
