"""The no-allocation entry point modap_eval_sweep_static against modap_eval_sweep.

Both run the same one-pass sweep in the same built-in launch shape and row
mapping, so their results are equal bit for bit; both are also held to the
oracle's tolerances (tests/parity.py).  Two calls in a row, the second on a
smaller system, show that the shared scratch array carries nothing from one
call to the next.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from parity import check_sweep

pytestmark = pytest.mark.gpu

VEC = {"f64": 2, "f32": 4, "bf16": 8}
TORCH_STORE = {"f64": "float64", "f32": "float32", "bf16": "int16"}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "these tests need the GPU"
    import paper_2003_09956_amd as P
    P.lib()
    return P


def padded_device(A, dtype):
    """A on the device with lda rounded up to 16 bytes and zero padding."""
    import torch
    m, n = A.shape
    lda = (n + VEC[dtype] - 1) // VEC[dtype] * VEC[dtype]
    host = np.zeros((m, lda), dtype=A.dtype)
    host[:, :n] = A
    if dtype == "bf16":
        host = host.view(np.int16)
    return torch.from_numpy(host).to("cuda:0"), lda


def static_sweep(P, sys_, dtype, x):
    import torch
    Ad, lda = padded_device(sys_.A, dtype)
    dev = torch.device("cuda:0")
    b = torch.from_numpy(sys_.b).to(dev)
    xd = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    y = torch.full((sys_.n,), float("nan"), dtype=torch.float64, device=dev)
    r = torch.full((sys_.m,), float("nan"), dtype=torch.float64, device=dev)
    h = torch.full((1,), -1, dtype=torch.int64, device=dev)
    dm = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
    P.eval_sweep_static(Ad, b, xd, y, dtype=dtype, r=r, h=h, max_viol=dm, lda=lda)
    torch.cuda.synchronize()
    return y.cpu().numpy(), r.cpu().numpy(), int(h.item()), float(dm.item())


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f64"])
def test_static_sweep_equals_context_sweep_twice(P, dtype):
    for call, (n, m) in enumerate([(1003, 3000), (301, 700)]):
        sys_ = W.gaussian(n, m, seed=11 + call, dtype=dtype)
        x = sys_.z + np.random.default_rng(call).normal(scale=0.3, size=n)
        say(f"static sweep call {call} dtype={dtype} n={n} m={m}")
        ys, rs, hs, ds = static_sweep(P, sys_, dtype, x)
        with P.Solver() as s:
            s.set_system(sys_.A, sys_.b, dtype=dtype)
            g = s.eval_sweep(x)
        assert np.array_equal(ys, g.y) and np.array_equal(rs, g.r)
        assert hs == g.h and ds == g.max_viol
        o = oracle.sweep(sys_.A, dtype, sys_.b, x)
        check_sweep(sys_.A, dtype, o, ys, hs, ds, rs, label=f"static {dtype} {n}x{m}")


def test_static_sweep_rejects_what_it_cannot_hold(P):
    import torch
    dev = torch.device("cuda:0")
    # rows longer than the one-pass sweep covers (FP32: 16384 elements)
    A = torch.zeros((4, 16388), dtype=torch.float32, device=dev)
    b = torch.zeros(4, dtype=torch.float64, device=dev)
    x = torch.zeros(16388, dtype=torch.float64, device=dev)
    y = torch.zeros(16388, dtype=torch.float64, device=dev)
    with pytest.raises(P.ModapError, match="E_INVAL"):
        P.eval_sweep_static(A, b, x, y, dtype="f32")
    # a system whose row norms alone need more than the 32 MiB scratch
    m = 4_500_000
    A = torch.zeros((m, 4), dtype=torch.float32, device=dev)
    b = torch.zeros(m, dtype=torch.float64, device=dev)
    x = torch.zeros(4, dtype=torch.float64, device=dev)
    y = torch.zeros(4, dtype=torch.float64, device=dev)
    with pytest.raises(P.ModapError, match="E_INVAL"):
        P.eval_sweep_static(A, b, x, y, dtype="f32")
    # a leading dimension that is not a whole number of 16-byte vectors
    A = torch.zeros((8, 6), dtype=torch.float32, device=dev)
    with pytest.raises(P.ModapError, match="E_INVAL"):
        P.eval_sweep_static(A, torch.zeros(8, dtype=torch.float64, device=dev),
                            torch.zeros(6, dtype=torch.float64, device=dev),
                            torch.zeros(6, dtype=torch.float64, device=dev), dtype="f32")
