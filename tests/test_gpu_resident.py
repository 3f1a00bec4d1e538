"""The resident iteration of small systems (one launch of many iterations,
rows held in LDS, one grid barrier per iteration) against the two-kernel
iteration and the oracle.

The two paths take the same steps from the same data; only the order in which
the partial sums of y over row bands are added differs, so they agree to the
rounding of that sum (and, in FP64 on the box-plus-sum system, in the step
count).  Launch boundaries do not matter to the resident path: queued and
one-per-call iterations give the same bits.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from parity import TOL, weighted_abs_rows

pytestmark = pytest.mark.gpu


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


def two_kernel(s):
    """Force the two-kernel path: the built-in sweep shape, set explicitly."""
    t = s.get_tile()
    s.set_tile(t["block"], t["lanes_per_row"], t["chunks"], 0, t["rows_per_step"], depth=t["depth"])


@pytest.mark.parametrize("seed", [0, 7])
def test_resident_solve_of_box_sum_matches_oracle_and_two_kernel_path(P, seed):
    """The FP64 box-plus-sum system (n=256, m=513): both paths stop after the
    oracle's number of steps at the oracle's point."""
    sys_ = W.c1(seed)
    ores = oracle.solve(sys_.A, "f64", sys_.b, sys_.x0, lam=1.0, eps=1e-6, rule=0, max_steps=20000)
    assert ores.status == 0
    out = {}
    for path in ("resident", "two-kernel"):
        with P.Solver() as s:
            s.set_system(sys_.A, sys_.b, x0=sys_.x0, dtype="f64")
            if path == "two-kernel":
                two_kernel(s)
            say(f"box-sum seed={seed} {path}")
            st, code = s.solve(P.params(lam=1.0, eps=1e-6, max_iters=20000))
            x, _, _ = s.query()
        assert code == 0 and st.converged == 1 and st.certified == 1
        assert st.iters == ores.iters, (path, st.iters, ores.iters)
        np.testing.assert_allclose(x, ores.x, rtol=0, atol=1e-9 * np.abs(ores.x).max())
        out[path] = (x, st.seconds)
    say(f"  seconds: resident {out['resident'][1]:.4f}, two-kernel {out['two-kernel'][1]:.4f}")


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_resident_steps_match_oracle_steps_with_drift(P, dtype):
    """Each resident step against the oracle's step from the GPU's own x_k on
    the oracle's data b_k = b_0 + A (V[0] + ... + V[k-1]) (section 5's moving
    system), with a one-shot translation pending at the start."""
    n, m = 200, 900
    sys_ = W.gaussian(n, m, seed=61, dtype=dtype)
    V = W.drift(n, 40, sigma=1e-3, seed=61)
    v0 = np.random.default_rng(61).normal(scale=1e-2, size=n)
    lam, tol = 0.05, TOL[dtype]
    prm = P.params(lam=lam, eps=1e-9)
    b = oracle.translate(sys_.A, dtype, sys_.b, v0)
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype=dtype)
        s.set_drift(V)
        s.update_coeffs(translate=v0)
        x = sys_.x0.copy()
        for k in range(10):
            say(f"resident step k={k} dtype={dtype}")
            s.iterate(1, prm)
            x1, _, st = s.query()
            o = oracle.sweep(sys_.A, dtype, b, x)
            xo, status = oracle.step(o.y, o.h, 0, lam, x)
            assert status == 0 and st.iters == k + 1
            near = o.r > -tol * o.t
            s_y = np.linalg.norm(weighted_abs_rows(sys_.A, dtype, np.where(near, o.t / o.nu, 0)))
            bound = tol * (np.linalg.norm(x) + lam * s_y / np.linalg.norm(o.y))
            assert np.linalg.norm(x1 - xo) <= bound, (k, np.linalg.norm(x1 - xo), bound)
            b = oracle.translate(sys_.A, dtype, b, V[k])
            x = x1
        _, bq, _ = s.query(want_x=False, want_b=True)
    scale = np.abs(W.stored_to_f64(sys_.A, dtype)) @ (np.abs(V[:10]).sum(axis=0) + np.abs(v0)) + np.abs(sys_.b)
    assert np.max(np.abs(bq - b) / scale) <= 1e-12


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("track", [False, True])
def test_resident_queued_iterations_equal_single_calls(P, dtype, track):
    """The same 30 iterations in one launch, one per call, and in uneven
    chunks: the same bits of x and b, the same counters."""
    n, m = 300, 1000
    sys_ = W.gaussian(n, m, seed=71, dtype=dtype)
    V = W.drift(n, 40, sigma=2e-3, seed=71)
    prm = P.params(lam=0.2, eps=1e-6, track=track)
    x0 = sys_.z + 0.5
    res = []
    for chunks in ([30], [1] * 30, [7, 1, 15, 7]):
        with P.Solver() as s:
            s.set_system(sys_.A, sys_.b, x0=x0, dtype=dtype)
            s.set_drift(V)
            say(f"resident chunks {chunks[:4]} dtype={dtype} track={track}")
            for k in chunks:
                s.iterate(k, prm)
            x, b, st = s.query(want_x=True, want_b=True)
        res.append((x, b, st.sweeps, st.iters))
    assert res[0][2] == res[1][2] == res[2][2] == 30
    assert res[0][3] == res[1][3] == res[2][3] > 0
    for other in res[1:]:
        assert np.array_equal(res[0][0], other[0]) and np.array_equal(res[0][1], other[1])


def test_resident_and_two_kernel_paths_agree_per_step(P):
    """FP32 storage, 15 iterations from the same start on the same moving
    data: the two paths' points agree to the rounding of the band sums."""
    n, m = 500, 1400
    sys_ = W.gaussian(n, m, seed=91, dtype="f32")
    V = W.drift(n, 20, sigma=1e-3, seed=91)
    prm = P.params(lam=0.05, eps=1e-9)
    xs = {}
    for path in ("resident", "two-kernel"):
        with P.Solver() as s:
            s.set_system(sys_.A, sys_.b, dtype="f32")
            if path == "two-kernel":
                two_kernel(s)
            s.set_drift(V)
            say(f"paths agree: {path}")
            st = s.iterate(15, prm)
            xs[path] = s.query()[0]
            assert st.iters == 15
    d = np.linalg.norm(xs["resident"] - xs["two-kernel"])
    assert d <= 15 * TOL["f32"] * (np.linalg.norm(xs["two-kernel"]) + 0.05 * 15), d


# Edge shapes of the resident form: one row and one column; one workgroup;
# the longest row it holds (512 columns, eight per lane, with a ragged last
# lane group at n=449); the most workgroups (32) with full bands (FP64,
# n=512, m=768) and with a ragged last band (m=4097 at n=64, 129 rows a band).
RESIDENT_EDGES = [("f64", 1, 1), ("f32", 1, 1), ("bf16", 1, 1), ("f32", 5, 17), ("bf16", 449, 333),
                  ("f64", 512, 768), ("f32", 64, 4097), ("f64", 63, 130)]


@pytest.mark.parametrize("dtype,n,m", RESIDENT_EDGES)
def test_resident_edge_shapes_step_like_the_oracle(P, dtype, n, m):
    """Six single resident iterations from a point with violated rows, each
    against the oracle's step from the GPU's previous point, and the stats
    report that the resident form ran."""
    sys_ = W.gaussian(n, m, seed=n * 3 + m, dtype=dtype)
    rng = np.random.default_rng(m)
    x = sys_.z + rng.normal(scale=2.0 / np.sqrt(n) + 0.5, size=n)
    lam, tol = 0.7, TOL[dtype]
    prm = P.params(lam=lam, eps=1e-12)
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, x0=x, dtype=dtype)
        for k in range(6):
            say(f"resident edge dtype={dtype} n={n} m={m} k={k}")
            st = s.iterate(1, prm)
            assert st.resident == 1
            x1, _, st = s.query()
            o = oracle.sweep(sys_.A, dtype, sys_.b, x)
            xo, status = oracle.step(o.y, o.h, 0, lam, x)
            if status != 0:      # the oracle's point is feasible: the device stops there too
                assert st.converged == 1 and np.array_equal(x1, x)
                break
            assert st.iters == k + 1
            near = o.r > -tol * o.t
            s_y = np.linalg.norm(weighted_abs_rows(sys_.A, dtype, np.where(near, o.t / o.nu, 0)))
            bound = tol * (np.linalg.norm(x) + lam * s_y / np.linalg.norm(o.y))
            assert np.linalg.norm(x1 - xo) <= bound, (k, np.linalg.norm(x1 - xo), bound)
            x = x1


@pytest.mark.parametrize("dtype,n,m", [("f64", 513, 100), ("f64", 512, 769), ("f32", 64, 12289)])
def test_systems_beyond_the_resident_limits_take_the_two_kernel_form(P, dtype, n, m):
    """A row longer than 512 columns, or rows that do not fit in the LDS of
    32 workgroups, leave the resident form; the step is the oracle's all the
    same."""
    sys_ = W.gaussian(n, m, seed=5, dtype=dtype)
    x = sys_.z + np.random.default_rng(1).normal(scale=0.5, size=n)
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, x0=x, dtype=dtype)
        say(f"beyond resident dtype={dtype} n={n} m={m}")
        st = s.iterate(1, P.params(lam=0.7, eps=1e-12))
        assert st.resident == 0 and st.iters == 1
        x1 = s.query()[0]
    o = oracle.sweep(sys_.A, dtype, sys_.b, x)
    xo, status = oracle.step(o.y, o.h, 0, 0.7, x)
    assert status == 0
    near = o.r > -TOL[dtype] * o.t
    s_y = np.linalg.norm(weighted_abs_rows(sys_.A, dtype, np.where(near, o.t / o.nu, 0)))
    assert np.linalg.norm(x1 - xo) <= TOL[dtype] * (np.linalg.norm(x) + 0.7 * s_y / np.linalg.norm(o.y))


def test_resident_barrier_timeout_is_reported(P, monkeypatch):
    """A wait at the grid barrier that exceeds its bound (here forced from the
    host with a bound of zero clock ticks, so the first workgroup to arrive
    gives up at once) ends every workgroup's loop, and the call reports
    E_DEVICE instead of results."""
    sys_ = W.c1(0)
    monkeypatch.setenv("MODAP_RESIDENT_TIMEOUT_TICKS", "0")
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, x0=sys_.x0, dtype="f64")
        say("forced barrier timeout")
        with pytest.raises(P.ModapError, match="E_DEVICE"):
            s.iterate(5, P.params(lam=1.0, eps=1e-6))
        # the data stay void (the report is sticky) until the system is set again
        monkeypatch.delenv("MODAP_RESIDENT_TIMEOUT_TICKS")
        with pytest.raises(P.ModapError, match="E_DEVICE"):
            s.iterate(5, P.params(lam=1.0, eps=1e-6))
        s.set_system(sys_.A, sys_.b, x0=sys_.x0, dtype="f64")
        st = s.iterate(5, P.params(lam=1.0, eps=1e-6))
        assert st.iters == 5
