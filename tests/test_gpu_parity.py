"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Every comparison takes the same seeded inputs and the same point x on both
sides; tolerances are those of tests/parity.py.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from parity import TOL, TOL_BF16_VS_F64, check_sweep, fejer_gap, weighted_abs_rows

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


def probe_point(sys_, scale, seed):
    rng = np.random.default_rng(seed)
    return sys_.z + rng.normal(scale=scale, size=sys_.n)


SHAPES = [(1, 1), (2, 3), (5, 17), (63, 127), (64, 64), (65, 200), (256, 513), (1000, 700),
          (2049, 300), (4096, 1100), (8192, 600), (12000, 257), (16384, 260), (16390, 70), (40001, 90)]


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n,m", SHAPES)
def test_eval_sweep_matches_oracle(P, dtype, n, m):
    say(f"eval_sweep dtype={dtype} n={n} m={m}")
    sys_ = W.gaussian(n, m, seed=n * 7 + m, dtype=dtype)
    x = probe_point(sys_, 2.0 / np.sqrt(n) + 0.05, seed=m)
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype=dtype)
        g = s.eval_sweep(x)
        say("  tile", s.get_tile())
    o = oracle.sweep(sys_.A, dtype, sys_.b, x)
    check_sweep(sys_.A, dtype, o, g.y, g.h, g.max_viol, g.r, label=f"{dtype} {n}x{m}")


ALL_SHAPES = {  # (block, lanes per row, chunks, rows per step, depth), as compiled
    "f64": [
            (256, 16, 1, 1, 2), (256, 16, 2, 1, 2), (256, 16, 4, 1, 2), (256, 32, 4, 1, 2),
            (256, 64, 1, 1, 2), (256, 64, 2, 1, 2), (256, 64, 4, 1, 2), (256, 64, 1, 2, 2), (256, 64, 2, 2, 2),
            (256, 64, 4, 2, 2), (256, 256, 2, 1, 2), (256, 256, 4, 1, 2), (256, 256, 8, 1, 2), (256, 256, 2, 2, 2),
            (256, 256, 4, 2, 2), (512, 512, 2, 1, 2), (512, 512, 4, 1, 2),
            (512, 512, 2, 2, 2), (512, 512, 4, 2, 2)],
    "f32": [
            (256, 16, 1, 1, 2), (256, 16, 2, 1, 2), (256, 16, 4, 1, 2), (256, 32, 2, 1, 2), (256, 32, 4, 1, 2),
            (256, 64, 1, 1, 2), (256, 64, 2, 1, 2), (256, 64, 4, 1, 2), (256, 64, 1, 2, 2), (256, 64, 2, 2, 2),
            (256, 64, 4, 2, 2), (256, 256, 2, 1, 2), (256, 256, 4, 1, 2), (256, 256, 8, 1, 2), (256, 256, 2, 2, 2),
            (256, 256, 4, 2, 2), (256, 256, 2, 4, 2), (512, 512, 2, 1, 2), (512, 512, 4, 1, 2),
            (512, 512, 8, 1, 2), (512, 512, 2, 2, 2), (512, 512, 4, 2, 2), (512, 512, 2, 4, 2),
            (1024, 1024, 2, 1, 2), (512, 256, 8, 1, 2), (512, 256, 4, 1, 2),
            (512, 512, 4, 1, 3), (512, 512, 4, 1, 4), (1024, 1024, 2, 1, 3)],
    "bf16": [
            (256, 16, 1, 1, 2), (256, 16, 2, 1, 2), (256, 16, 4, 1, 2), (256, 32, 2, 1, 2),
            (256, 64, 1, 1, 2), (256, 64, 2, 1, 2), (256, 64, 4, 1, 2), (256, 64, 1, 2, 2), (256, 64, 2, 2, 2),
            (256, 256, 2, 1, 2), (256, 256, 4, 1, 2), (256, 256, 2, 2, 2), (512, 512, 2, 1, 2),
            (512, 512, 4, 1, 2), (512, 512, 2, 2, 2), (1024, 1024, 1, 1, 2), (1024, 1024, 1, 1, 4),
            (256, 256, 4, 1, 3), (512, 512, 2, 2, 3), (512, 512, 4, 1, 3)],
}
VEC = {"f64": 2, "f32": 4, "bf16": 8}


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_every_kernel_shape_and_grid(P, dtype):
    """Each compiled sweep shape that covers the row, at two grid sizes, gives
    the oracle's sweep; a ragged n and m exercise the masked tails."""
    n, m = 203, 997
    sys_ = W.gaussian(n, m, seed=17, dtype=dtype)
    x = probe_point(sys_, 0.2, seed=3)
    o = oracle.sweep(sys_.A, dtype, sys_.b, x)
    ys = []
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype=dtype)
        for (blk, lpr, ch, rs, pd) in ALL_SHAPES[dtype]:
            if lpr * VEC[dtype] * ch < n:
                continue
            # grids 2 and 3 give a workgroup more rows than its staged row
            # outputs hold, so they are written out inside the row loop too
            for grid, il in ((0, 0), (7, 0), (0, 1), (5, 1), (2, 0), (3, 1)):
                say(f"shape dtype={dtype} block={blk} lpr={lpr} chunks={ch} rows/step={rs} depth={pd} "
                    f"interleave={il} grid={grid}")
                s.set_tile(blk, lpr, ch, grid, rs, depth=pd, interleave=il)
                t = s.get_tile()
                assert t["depth"] == pd and t["interleave"] == il
                g = s.eval_sweep(x)
                check_sweep(sys_.A, dtype, o, g.y, g.h, g.max_viol, g.r,
                            label=f"{dtype} {blk}/{lpr}/{ch}/{rs}/{pd}/{il}/{grid}")
                ys.append(g.y)
    assert len(ys) >= 4


SHORT_ROWS = [("f32", 37, 1999), ("f32", 100, 2003), ("bf16", 90, 1501), ("bf16", 250, 999), ("f64", 29, 2011),
              ("f64", 60, 1500), ("f64", 120, 997)]


@pytest.mark.parametrize("dtype,n,m", SHORT_ROWS)
def test_short_row_shapes_and_grids(P, dtype, n, m):
    """Short rows: every compiled shape that covers the row (16 and 32 lanes
    per row -- four or two rows to a wavefront -- and the wider ones), at
    several grids and in both row orders, gives the oracle's sweep; ragged n
    and m give rows past the band and chunks past the padded row."""
    sys_ = W.gaussian(n, m, seed=n + m, dtype=dtype)
    x = probe_point(sys_, 0.2, seed=5)
    o = oracle.sweep(sys_.A, dtype, sys_.b, x)
    done = 0
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype=dtype)
        for (blk, lpr, ch, rs, pd) in ALL_SHAPES[dtype]:
            if lpr * VEC[dtype] * ch < n or lpr * VEC[dtype] * ch > 4 * 64 * VEC[dtype]:
                continue
            for grid, il in ((0, 0), (7, 0), (3, 1), (2, 0)):
                say(f"short rows dtype={dtype} n={n} m={m} block={blk} lpr={lpr} chunks={ch} grid={grid} il={il}")
                s.set_tile(blk, lpr, ch, grid, rs, depth=pd, interleave=il)
                g = s.eval_sweep(x)
                check_sweep(sys_.A, dtype, o, g.y, g.h, g.max_viol, g.r,
                            label=f"{dtype} n={n} {blk}/{lpr}/{ch}/{rs}/{pd}/{il}/{grid}")
                done += 1
    assert done >= 4


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f64"])
def test_short_row_steps_with_translation(P, monkeypatch, dtype):
    """The built-in shape of a long system of short rows (16 lanes per row),
    on the two-kernel path: each step, with a drift schedule translating the
    data in the same sweep, against the oracle's step from the GPU's x."""
    monkeypatch.setenv("MODAP_RESIDENT", "0")
    n, m = {"f32": 50, "bf16": 100, "f64": 40}[dtype], 20001
    sys_ = W.gaussian(n, m, seed=31, dtype=dtype)
    V = W.drift(n, 10, sigma=1e-3, seed=31)
    lam = 0.3
    prm = P.params(lam=lam, eps=1e-9)
    x = sys_.z + 0.3
    b = sys_.b.copy()
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, x0=x, dtype=dtype)
        assert s.get_tile()["lanes_per_row"] in (16, 32)
        s.set_drift(V)
        for k in range(3):
            say(f"short-row steps dtype={dtype} k={k}")
            s.iterate(1, prm)
            x1, b1, q = s.query(want_b=True)
            o = oracle.sweep(sys_.A, dtype, b, x)
            xo, status = oracle.step(o.y, o.h, 0, lam, x)
            assert status == 0 and q.iters == k + 1
            tol = TOL[dtype]
            near = o.r > -tol * o.t
            s_y = np.linalg.norm(weighted_abs_rows(sys_.A, dtype, np.where(near, o.t / o.nu, 0)))
            assert np.linalg.norm(x1 - xo) <= tol * (np.linalg.norm(x) + lam * s_y / np.linalg.norm(o.y)), k
            b = oracle.translate(sys_.A, dtype, b, V[k])
            scale = np.abs(W.stored_to_f64(sys_.A, dtype)) @ np.abs(V[:k + 1]).sum(axis=0) + np.abs(sys_.b)
            assert np.max(np.abs(b1 - b) / scale) <= tol, k
            x = x1


def test_box_sum_closed_form_on_gpu(P):
    """The box-plus-sum system's sweep has a closed form (independent of the oracle)."""
    sys_ = W.c1(seed=0)
    xs = [sys_.x0, np.random.default_rng(1).uniform(-50, 250, sys_.n), np.full(sys_.n, 100.0)]
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype="f64")
        for x in xs:
            say("box_sum closed form")
            g = s.eval_sweep(x)
            agg = x.sum() - 200.0 * (sys_.n - 1)
            y = np.maximum(x - 200, 0) - np.maximum(-x, 0) + max(agg, 0) / sys_.n
            h = int(np.sum(x > 200) + np.sum(x < 0) + (agg > 0))
            d = max(np.max(np.maximum(x - 200, 0)), np.max(np.maximum(-x, 0)), max(agg, 0) / 16.0)
            assert g.h == h
            np.testing.assert_allclose(g.y, y, rtol=1e-13, atol=1e-12)
            assert g.max_viol == pytest.approx(d, rel=1e-13, abs=1e-12)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_translation_is_fused_into_the_next_sweep(P, dtype):
    """Data update b <- b + A v (section 5's translation) applied by the sweep."""
    n, m = 777, 1500
    sys_ = W.gaussian(n, m, seed=5, dtype=dtype)
    rng = np.random.default_rng(5)
    v1, v2 = rng.normal(scale=0.3, size=n), rng.normal(scale=0.3, size=n)
    x = probe_point(sys_, 0.3, seed=9)
    b2 = oracle.translate(sys_.A, dtype, oracle.translate(sys_.A, dtype, sys_.b, v1), v2)
    o = oracle.sweep(sys_.A, dtype, b2, x)
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype=dtype)
        say(f"translation dtype={dtype}")
        s.update_coeffs(translate=v1)
        s.update_coeffs(translate=v2)
        g = s.eval_sweep(x)
        check_sweep(sys_.A, dtype, o, g.y, g.h, g.max_viol, g.r, label="translated")
        _, bq, _ = s.query(want_x=False, want_b=True)
    # b read back: FP64 flush of the pending translation
    scale = np.abs(W.stored_to_f64(sys_.A, dtype)) @ (np.abs(v1) + np.abs(v2)) + np.abs(sys_.b)
    assert np.max(np.abs(bq - b2) / scale) <= 1e-13


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_row_replacement_in_place(P, dtype):
    """Coefficient updates: rows replaced in place with norms refreshed; a
    translation queued before the replacement does not move the new rows."""
    n, m = 300, 800
    sys_ = W.gaussian(n, m, seed=8, dtype=dtype)
    v = np.random.default_rng(8).normal(scale=0.2, size=n)
    idx, rows, bb = W.replacement_rows(sys_, 40, seed=8)
    A2, b2 = oracle.replace_rows(sys_.A, dtype, oracle.translate(sys_.A, dtype, sys_.b, v), idx, rows, bb)
    x = probe_point(sys_, 0.4, seed=2)
    o = oracle.sweep(A2, dtype, b2, x)
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype=dtype)
        say(f"row replacement dtype={dtype}")
        s.update_coeffs(translate=v)
        s.update_coeffs(idx, rows, bb)
        g = s.eval_sweep(x)
    check_sweep(A2, dtype, o, g.y, g.h, g.max_viol, g.r, label="replaced")


@pytest.mark.parametrize("rule", [0, 1])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_each_step_matches_oracle_step(P, rule, dtype):
    """x_{k+1} from x_k: the GPU's step (eq. 12 or Algorithm 1) against the
    oracle's step from the GPU's own x_k, for several consecutive iterations."""
    n, m = 500, 1400
    sys_ = W.gaussian(n, m, seed=21, dtype=dtype)
    x0 = sys_.z + np.random.default_rng(4).normal(scale=1.0, size=n)
    lam = 0.5
    prm = P.params(lam=lam, eps=1e-9, step=rule)
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, x0=x0, dtype=dtype)
        x = x0.copy()
        for k in range(6):
            say(f"step k={k} rule={rule} dtype={dtype}")
            st = s.iterate(1, prm)
            x1, _, _ = s.query()
            o = oracle.sweep(sys_.A, dtype, sys_.b, x)
            xo, status = oracle.step(o.y, o.h, rule, lam, x)
            assert status == 0 and st.iters == k + 1
            tol = TOL[dtype]
            near = o.r > -tol * o.t
            s_y = np.linalg.norm(weighted_abs_rows(sys_.A, dtype, np.where(near, o.t / o.nu, 0)))
            denom = np.linalg.norm(o.y) if rule == 0 else o.h
            bound = tol * (np.linalg.norm(x) + lam * s_y / denom)
            assert np.linalg.norm(x1 - xo) <= bound, (k, np.linalg.norm(x1 - xo), bound)
            x = x1


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_solve_box_sum_fp64_reaches_feasibility_like_oracle(P, seed):
    """Plain FP64 stationary box-plus-sum system (n=256, m=513, lambda=1,
    eps = 1e-6 * ||b||inf): the GPU solve stops at an eps-feasible point after
    the same number of ModAP steps as the oracle."""
    sys_ = W.c1(seed)
    ores = oracle.solve(sys_.A, "f64", sys_.b, sys_.x0, lam=1.0, eps=1e-6, rule=0, max_steps=20000)
    assert ores.status == 0
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, x0=sys_.x0, dtype="f64")
        say(f"solve c1 seed={seed}")
        st, code = s.solve(P.params(lam=1.0, eps=1e-6, max_iters=20000))
        x, _, _ = s.query()
    assert code == 0 and st.converged == 1
    o = oracle.sweep(sys_.A, "f64", sys_.b, x)
    assert o.dmax <= 1e-6 * o.binf * (1 + 1e-12)
    assert st.iters == ores.iters
    np.testing.assert_allclose(x, ores.x, rtol=0, atol=1e-9 * np.abs(ores.x).max())


@pytest.mark.parametrize("grid", [0, 2])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_drift_schedule_steps_match_oracle(P, dtype, grid):
    """Non-stationary iteration (section 5: the polytope is translated between
    iterations): after step k the system moves by V[k], fused into sweep k+1.
    Each GPU step is compared with the oracle's step from the GPU's own x_k on
    the oracle's data b_k = b_0 + A (V[0] + ... + V[k-1]).  With two
    workgroups each holds 350 rows, more than its staged translated b holds
    at once, so b is also written out inside the row loop."""
    n, m = 256, 700
    sys_ = W.gaussian(n, m, seed=33, dtype=dtype)
    V = W.drift(n, 40, sigma=1e-3, seed=33)
    lam, tol = 0.05, TOL[dtype]
    prm = P.params(lam=lam, eps=1e-9)
    b = sys_.b.copy()
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype=dtype)
        if grid:
            t = s.get_tile()
            s.set_tile(t["block"], t["lanes_per_row"], t["chunks"], grid, t["rows_per_step"], depth=t["depth"])
            assert s.get_tile()["grid"] == grid
        s.set_drift(V)
        x = sys_.x0.copy()
        for k in range(12):
            say(f"drift step k={k} dtype={dtype} grid={grid}")
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
    # query(b) is the exact data in FP64, whatever precision the sweep translates in
    scale = np.abs(W.stored_to_f64(sys_.A, dtype)) @ np.abs(V[:12]).sum(axis=0) + np.abs(sys_.b)
    assert np.max(np.abs(bq - b) / scale) <= 1e-12


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_solve_with_drift_reaches_feasibility(P, dtype):
    """ModAP catches a translating polytope (section 2, eq. 12): the solve stops
    at a point that is eps-feasible for the data current at the stop, and that
    data is the initial system translated by the first `iters` drift vectors.
    (Step counts are not compared: the fixed-length iteration near a moving
    boundary is chaotic -- a 1e-15 change of x0 changes the oracle's own count.)"""
    n, m = 256, 700
    sys_ = W.gaussian(n, m, seed=33, dtype=dtype)
    V = W.drift(n, 400, sigma=1e-3, seed=33)
    ores = oracle.solve(sys_.A, dtype, sys_.b, sys_.x0, lam=0.05, eps=1e-6, rule=0,
                        max_steps=400, V=V)
    assert ores.status == 0
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype=dtype)
        s.set_drift(V)
        say(f"solve with drift dtype={dtype}")
        st, code = s.solve(P.params(lam=0.05, eps=1e-6, max_iters=400))
        x, bq, _ = s.query(want_b=True)
    assert code == 0 and st.converged == 1
    assert 0.5 * ores.iters <= st.iters <= 2 * ores.iters
    b = sys_.b.copy()
    for k in range(st.iters):
        b = oracle.translate(sys_.A, dtype, b, V[k])
    # query(b) returns the exact data (FP64, every translation applied), and
    # the certified stop is eps-feasible on them
    scale = np.abs(W.stored_to_f64(sys_.A, dtype)) @ np.abs(V[:st.iters]).sum(axis=0) + np.abs(sys_.b)
    assert np.max(np.abs(bq - b) / scale) <= 1e-12
    assert st.certified == 1
    o = oracle.sweep(sys_.A, dtype, b, x)
    assert o.dmax <= 1e-6 * o.binf * (1 + 1e-12)
    assert o.dmax <= st.max_viol * (1 + 1e-12)          # the certificate's value is an upper bound


def test_translation_in_wavefront_row_shape(P):
    """The translation path in the one-wavefront-per-row shape (short rows)."""
    n, m = 200, 900
    sys_ = W.gaussian(n, m, seed=44, dtype="f64")
    v = np.random.default_rng(44).normal(scale=0.5, size=n)
    x = probe_point(sys_, 0.3, seed=44)
    o = oracle.sweep(sys_.A, "f64", oracle.translate(sys_.A, "f64", sys_.b, v), x)
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype="f64")
        for shape in [(256, 64, 2, 0, 1), (256, 64, 4, 0, 2), (256, 256, 2, 0, 1)]:
            say(f"wave-shape translation {shape}")
            s.set_tile(*shape)
            s.update_coeffs(translate=v)
            g = s.eval_sweep(x)
            check_sweep(sys_.A, "f64", o, g.y, g.h, g.max_viol, g.r, label=str(shape))
            s.update_coeffs(translate=-v)


def test_full_size_fp32_sweep_c2(P):
    """n=8192, m=16384 FP32 (the benchmark's system): full element-wise parity
    of one sweep, with a translation pending, and the launch shape bench.py uses."""
    sys_ = W.c2(0)
    rng = np.random.default_rng(0)
    x = rng.normal(scale=0.05, size=sys_.n)
    v = rng.normal(scale=1e-2, size=sys_.n)
    say("c2 full-size sweep")
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype="f32")
        s.update_coeffs(translate=v)
        g = s.eval_sweep(x)
        tile = s.get_tile()
    b2 = oracle.translate(sys_.A, "f32", sys_.b, v)
    o = oracle.sweep(sys_.A, "f32", b2, x)
    err = check_sweep(sys_.A, "f32", o, g.y, g.h, g.max_viol, g.r, label="c2")
    say("  c2 errors", err, tile)
    assert fejer_gap(sys_.A, "f32", x, sys_.z + v, g.y, g.r) >= -1e-6 * np.abs(g.y).sum()


# The one-pass shapes that cover an 8192-element FP32 row (block, lanes per
# row, chunks, rows per step, depth): the shapes the autotuner chooses from
# for the benchmark's system.
C2_SHAPES = [(256, 256, 8, 1, 2), (512, 512, 4, 1, 2), (512, 512, 8, 1, 2), (512, 512, 4, 2, 2),
             (1024, 1024, 2, 1, 2), (512, 256, 8, 1, 2), (512, 512, 4, 1, 3), (512, 512, 4, 1, 4),
             (1024, 1024, 2, 1, 3)]


def test_full_size_c2_every_tunable_shape(P):
    """The benchmark's system under every launch shape the autotuner can pick
    for it (one workgroup per CU, both row orders; two per CU for the
    built-in shape), each sweep against the oracle element by element, with
    a translation pending as in the timed iterations."""
    sys_ = W.c2(0)
    rng = np.random.default_rng(4)
    x = rng.normal(scale=0.05, size=sys_.n)
    v = rng.normal(scale=1e-2, size=sys_.n)
    o = oracle.sweep(sys_.A, "f32", oracle.translate(sys_.A, "f32", sys_.b, v), x)
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype="f32")
        s.update_coeffs(translate=v)
        cases = [(shape, il, 0) for shape in C2_SHAPES for il in (0, 1)] + [(C2_SHAPES[0], 0, 512)]
        for (blk, lpr, ch, rs, pd), il, grid in cases:
            say(f"c2 shape {blk}/{lpr}/{ch}/{rs}/{pd} interleave={il} grid={grid}")
            s.set_tile(blk, lpr, ch, grid, rs, depth=pd, interleave=il)
            g = s.eval_sweep(x)
            check_sweep(sys_.A, "f32", o, g.y, g.h, g.max_viol, g.r, label=f"c2 {blk}/{lpr}/{ch}/{rs}/{pd}/{il}/{grid}")


@pytest.mark.timeout(900)
def test_full_size_bf16_sweep_c3(P):
    """n=16384, m=65536 BF16 storage (2 GiB): full parity of one sweep against
    the oracle on the same stored bytes, under the built-in launch shape and
    every shape the autotuner can pick for this system; then the same sweep
    against the FP64 system the BF16 rows were rounded from (quantisation,
    5e-3)."""
    sys_ = W.c3(0)
    x = np.random.default_rng(1).normal(scale=0.03, size=sys_.n)
    say("c3 full-size sweep")
    o = oracle.sweep(sys_.A, "bf16", sys_.b, x)
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype="bf16")
        g = s.eval_sweep(x)
        err = check_sweep(sys_.A, "bf16", o, g.y, g.h, g.max_viol, g.r, label="c3")
        say("  c3 errors", err, s.get_tile())
        for depth in (2, 3):
            for il in (0, 1):
                say(f"c3 shape 512/512/4/1/{depth} interleave={il}")
                s.set_tile(512, 512, 4, 0, 1, depth=depth, interleave=il)
                g2 = s.eval_sweep(x)
                check_sweep(sys_.A, "bf16", o, g2.y, g2.h, g2.max_viol, g2.r, label=f"c3 512/512/4/1/{depth}/{il}")
        del o
        # the FP64 rows of the same draw (the generator stream does not depend
        # on the storage type), with their own b on both sides
        s64 = W.gaussian(sys_.n, sys_.m, 0, "f64")
        assert np.array_equal(W.encode(s64.A[:64], "bf16"), sys_.A[:64])
        say("c3 against the FP64 original")
        s.set_system(sys_.A, s64.b, dtype="bf16")
        g3 = s.eval_sweep(x)
    o64 = oracle.sweep(s64.A, "f64", s64.b, x)
    err = check_sweep(s64.A, "f64", o64, g3.y, g3.h, g3.max_viol, g3.r, tol=TOL_BF16_VS_F64, label="c3 bf16-vs-f64")
    say("  c3 quantisation error", err)


def test_bf16_quantisation_against_fp64_original(P):
    """BF16-stored rows against the unrounded FP64 rows (same b, same x): the
    per-sweep error stays within 5e-3 on the condition scale."""
    n, m = 4096, 8192
    s64 = W.gaussian(n, m, seed=4, dtype="f64")
    A16 = W.encode(s64.A, "bf16")
    x = probe_point(s64, 0.05, seed=4)
    o = oracle.sweep(s64.A, "f64", s64.b, x)
    with P.Solver() as s:
        s.set_system(A16, s64.b, dtype="bf16")
        say("bf16 vs fp64 original")
        g = s.eval_sweep(x)
    err = check_sweep(s64.A, "f64", o, g.y, g.h, g.max_viol, g.r, tol=TOL_BF16_VS_F64, label="bf16-vs-f64")
    say("  quantisation error", err)


def test_deterministic_results(P):
    """Fixed-order reductions: repeated sweeps and repeated iterations are bitwise equal."""
    sys_ = W.gaussian(3000, 5000, seed=2, dtype="f32")
    x = probe_point(sys_, 0.05, seed=2)
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype="f32")
        say("determinism")
        g1 = s.eval_sweep(x)
        g2 = s.eval_sweep(x)
        assert np.array_equal(g1.y, g2.y) and np.array_equal(g1.r, g2.r)
        prm = P.params(lam=0.2, eps=1e-12)
        s.set_x(x)
        s.iterate(25, prm)
        xa, _, sa = s.query()
        s.set_x(x)
        s.iterate(25, prm)
        xb, _, sb = s.query()
    assert np.array_equal(xa, xb) and sa.iters == sb.iters > 0


def test_checkpoint_resume(P):
    """k iterations, read x, restart from it: the same as an uninterrupted run."""
    sys_ = W.gaussian(400, 900, seed=12, dtype="f64")
    prm = P.params(lam=0.3, eps=1e-12)
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype="f64")
        say("checkpoint")
        s.iterate(20, prm)
        xfull, _, _ = s.query()
        s.set_x(None)
        s.iterate(8, prm)
        xmid, _, _ = s.query()
        s.set_x(xmid)
        s.iterate(12, prm)
        xres, _, _ = s.query()
    assert np.array_equal(xfull, xres)


def test_feasible_start_is_a_fixed_point(P):
    sys_ = W.gaussian(128, 300, seed=1, dtype="f32")
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, x0=sys_.z, dtype="f32")
        say("fixed point")
        st, code = s.solve(P.params())
        x, _, _ = s.query()
    assert code == 0 and st.iters == 0 and st.h == 0
    assert np.array_equal(x, sys_.z)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_zero_iterations(P, dtype):
    """k = 0 queues nothing and leaves x alone; a solve with max_iters = 0
    still checks x0 (eq. 10) and stops there, with the oracle's violation."""
    sys_ = W.gaussian(300, 700, seed=9, dtype=dtype)
    o = oracle.sweep(sys_.A, dtype, sys_.b, sys_.x0)
    assert o.h > 0
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype=dtype)
        say("zero iterations", dtype)
        st = s.iterate(0, P.params())
        assert st.iters == 0 and st.sweeps == 0
        st, code = s.solve(P.params(max_iters=0), raise_on_stop=False)
        assert code == 6 and st.iters == 0 and st.sweeps == 1 and st.state == 4
        scale = float(np.max(o.t / np.sqrt(o.nu)))
        assert abs(st.max_viol - o.dmax) <= TOL[dtype] * scale and st.h == o.h
        x, _, _ = s.query()
        assert np.array_equal(x, sys_.x0)
        # from the hidden (feasible) point, the same call reports success
        s.set_x(sys_.z)
        st, code = s.solve(P.params(max_iters=0), raise_on_stop=False)
        assert code == 0 and st.iters == 0 and st.state == 1


def test_error_paths(P):
    with P.Solver() as s:
        say("errors")
        with pytest.raises(P.ModapError) as e:
            s.iterate(1, P.params())
        assert e.value.status == 5                      # before set_system
        for shape in ((0, 3), (3, 0)):                   # empty systems
            with pytest.raises(P.ModapError) as e:
                s.set_system(np.zeros(shape), np.zeros(shape[0]), dtype="f64")
            assert e.value.status == 1
        A = np.array([[1.0, 0.0], [0.0, 0.0]])
        with pytest.raises(P.ModapError) as e:
            s.set_system(A, np.zeros(2), dtype="f64")
        assert e.value.status == 2                      # zero row
        with pytest.raises(P.ModapError) as e:
            s.set_system(np.eye(2), np.array([0.0, np.nan]), dtype="f64")
        assert e.value.status == 1                      # non-finite b
        A = np.array([[np.inf, 1.0], [1.0, 1.0]])
        with pytest.raises(P.ModapError) as e:
            s.set_system(A, np.zeros(2), dtype="f64")
        assert e.value.status == 2                      # non-finite row
        # x <= -1 and -x <= -1: infeasible; at x = 0 both rows are violated and y = 0
        s.set_system(np.array([[1.0], [-1.0]]), np.array([-1.0, -1.0]), dtype="f64")
        st, code = s.solve(P.params(), raise_on_stop=False)
        assert code == 7 and st.state == 2
        # step limit
        sys_ = W.c1(0)
        s.set_system(sys_.A, sys_.b, x0=sys_.x0, dtype="f64")
        st, code = s.solve(P.params(max_iters=10), raise_on_stop=False)
        assert code == 6 and st.iters == 10
        # bad replacement rows
        with pytest.raises(P.ModapError) as e:
            s.update_coeffs(np.array([3]), np.zeros((1, sys_.n)), np.array([1.0]))
        assert e.value.status == 2
        with pytest.raises(P.ModapError) as e:
            s.update_coeffs(np.array([3, 3]), np.ones((2, sys_.n)), np.array([1.0, 1.0]))
        assert e.value.status == 1
        with pytest.raises(P.ModapError):
            s.iterate(1, P.params(lam=-1.0))
        with pytest.raises(P.ModapError):
            s.set_tile(256, 64, 3)                      # no such compiled shape


def test_numeric_stop(P):
    """E_NUMERIC: a non-finite value reaching the check (eq. 10) or the step
    length (eq. 12) stops the solve instead of stepping with it."""
    import torch
    with P.Solver() as s:
        say("numeric stop")
        # a device x is taken as is; a NaN in it reaches the residuals
        s.set_system(np.eye(2), np.zeros(2), dtype="f64")
        s.set_x(torch.tensor([np.nan, 0.0], dtype=torch.float64, device="cuda:0"))
        st, code = s.solve(P.params(), raise_on_stop=False)
        assert code == 8 and st.iters == 0 and st.state == 3
        # finite data whose y overflows: y = (1e300, 1e300), ||y|| = inf
        s.set_system(np.array([[1.0, 1.0]]), np.zeros(1), x0=np.array([1e300, 1e300]), dtype="f64")
        st, code = s.solve(P.params(), raise_on_stop=False)
        assert code == 8 and st.iters == 0 and st.state == 3
        # the context stays usable: a finite restart solves
        s.set_x(np.array([1.0, 1.0]))
        st, code = s.solve(P.params(), raise_on_stop=False)
        assert code == 0 and st.state == 1


def test_device_pointers_and_profile(P):
    """The same calls with torch device tensors (ptrs_on_device = 1), and the
    per-kernel HIP-event timing used by the benchmark."""
    import torch
    sys_ = W.gaussian(1024, 4096, seed=3, dtype="f32")
    dev = torch.device("cuda:0")
    A = torch.from_numpy(sys_.A).to(dev)
    b = torch.from_numpy(sys_.b).to(dev)
    x = torch.from_numpy(probe_point(sys_, 0.1, 3)).to(dev)
    with P.Solver() as s:
        say("device pointers")
        s.set_system(A, b, dtype="f32")
        g = s.eval_sweep(x)
        torch.cuda.synchronize()
        o = oracle.sweep(sys_.A, "f32", sys_.b, x.cpu().numpy())
        check_sweep(sys_.A, "f32", o, g.y.cpu().numpy(), g.h, g.max_viol, g.r.cpu().numpy())
        st = s.iterate(10, P.params(lam=0.1, eps=1e-12, profile=True))
        assert st.profiled == 10 and st.sweep_ms > 0 and st.reduce_ms > 0
        st = s.iterate(10, P.params(lam=0.1, eps=1e-12, profile=3))
        assert st.profiled == 4 and st.sweep_ms > 0


def test_autotune_keeps_parity_and_caches(P, tmp_path, monkeypatch):
    """The autotuner picks a compiled shape that covers the row, leaves the
    state untouched, records it in the cache file, and set_system reuses it."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("MODAP_TUNE_CACHE", str(cache))
    sys_ = W.gaussian(3000, 4000, seed=6, dtype="f32")
    x = probe_point(sys_, 0.1, seed=6)
    o = oracle.sweep(sys_.A, "f32", sys_.b, x)
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype="f32")
        say("autotune")
        best = s.autotune(3)
        assert best["lanes_per_row"] * 4 * best["chunks"] >= 3000 and best["grid"] > 0
        assert s.get_tile() == best
        g = s.eval_sweep(x)
        check_sweep(sys_.A, "f32", o, g.y, g.h, g.max_viol, g.r, label="autotuned")
        _, _, st = s.query()
        assert st.sweeps == 0 and st.iters == 0
    line = cache.read_text().split()
    assert [int(v) for v in line[:3]] == [1, 3000, 4000]
    with P.Solver() as s2:
        s2.set_system(sys_.A, sys_.b, dtype="f32")
        t2 = s2.get_tile()
        keys = ("block", "lanes_per_row", "chunks", "rows_per_step", "depth", "interleave", "grid")
    assert tuple(t2[k] for k in keys) == tuple(best[k] for k in keys)


SPLIT = {"f64": (256, 256, 8), "f32": (256, 256, 8), "bf16": (256, 256, 4)}


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n,m,bands", [(300, 700, 0), (5000, 3000, 0), (9000, 5000, 3), (20000, 9000, 0)])
def test_split_row_form_matches_oracle(P, dtype, n, m, bands):
    """The two-phase split-row sweep (column tiles, then an AXPY over the
    violated rows only), forced on any size, with a translation pending."""
    sys_ = W.gaussian(n, m, seed=n + m, dtype=dtype)
    v = np.random.default_rng(n).normal(scale=0.05, size=n)
    x = probe_point(sys_, 1.0 / np.sqrt(n) + 0.02, seed=m)
    o = oracle.sweep(sys_.A, dtype, oracle.translate(sys_.A, dtype, sys_.b, v), x)
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype=dtype)
        blk, lpr, ch = SPLIT[dtype]
        say(f"split dtype={dtype} n={n} m={m} bands={bands}")
        s.set_tile(blk, lpr, ch, bands, 1, kind=1)
        t = s.get_tile()
        assert t["kind"] == 1 and t["grid"] >= 1
        s.update_coeffs(translate=v)
        g = s.eval_sweep(x)
    check_sweep(sys_.A, dtype, o, g.y, g.h, g.max_viol, g.r, label=f"split {dtype} {n}x{m}")


def test_split_row_form_is_chosen_for_long_rows(P):
    """Rows longer than the one-pass shapes cover fall back to the split form."""
    sys_ = W.gaussian(20000, 200, seed=3, dtype="f64")
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype="f64")
        assert s.get_tile()["kind"] == 1


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_split_row_iteration_matches_oracle_steps(P, dtype):
    """Steps and the drift schedule through the split-row form."""
    n, m = 9000, 2000
    sys_ = W.gaussian(n, m, seed=77, dtype=dtype)
    V = W.drift(n, 10, sigma=1e-3, seed=77)
    lam, tol = 0.3, TOL[dtype]
    prm = P.params(lam=lam, eps=1e-9)
    b = sys_.b.copy()
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, x0=sys_.z + 0.05, dtype=dtype)
        blk, lpr, ch = SPLIT[dtype]
        s.set_tile(blk, lpr, ch, 0, 1, kind=1)
        s.set_drift(V)
        x = sys_.z + 0.05
        for k in range(5):
            say(f"split step k={k} dtype={dtype}")
            s.iterate(1, prm)
            x1, _, st = s.query()
            o = oracle.sweep(sys_.A, dtype, b, x)
            assert o.h > 0
            xo, status = oracle.step(o.y, o.h, 0, lam, x)
            near = o.r > -tol * o.t
            s_y = np.linalg.norm(weighted_abs_rows(sys_.A, dtype, np.where(near, o.t / o.nu, 0)))
            bound = tol * (np.linalg.norm(x) + lam * s_y / np.linalg.norm(o.y))
            assert np.linalg.norm(x1 - xo) <= bound, (k, np.linalg.norm(x1 - xo), bound)
            b = oracle.translate(sys_.A, dtype, b, V[k])
            x = x1


def _run_calls(P, sys_, dtype, V, prm, chunks, tile=None, x0=None):
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, x0=x0, dtype=dtype)
        if tile is not None:
            s.set_tile(*tile[:4], 1, kind=tile[4])
        s.set_drift(V)
        for k in chunks:
            st = s.iterate(k, prm)
        x, b, st = s.query(want_x=True, want_b=True)
    return x, b, st


@pytest.mark.parametrize("form", ["one-pass", "split"])
@pytest.mark.parametrize("track", [False, True])
def test_queued_iterations_equal_single_calls_f64(P, form, track):
    """Iterations queued in one call settle each check at the start of the
    next sweep; one iteration per call settles it at the end of the call.
    With FP64 storage the working vectors are exact, so both give the same
    bits: x, the translated b, and the counters, with the drift applied every
    iteration (and, in tracking mode, past the eps-feasible checks)."""
    n, m = 700, 1500
    sys_ = W.gaussian(n, m, seed=21, dtype="f64")
    V = W.drift(n, 40, sigma=2e-3, seed=21)
    prm = P.params(lam=0.2, eps=1e-6, track=track)
    tile = (256, 256, 8, 0, 1) if form == "split" else None
    x0 = sys_.z + 0.5   # about 13 from the feasible set: 30 steps of 0.2 do not reach it
    say(f"queued vs single form={form} track={track}")
    xa, ba, sa = _run_calls(P, sys_, "f64", V, prm, [30], tile, x0)
    xb, bb, sb = _run_calls(P, sys_, "f64", V, prm, [1] * 30, tile, x0)
    xc, bc, sc = _run_calls(P, sys_, "f64", V, prm, [7, 1, 15, 7], tile, x0)
    assert sa.sweeps == sb.sweeps == sc.sweeps == 30
    assert sa.iters == sb.iters == sc.iters > 0
    assert np.array_equal(xa, xb) and np.array_equal(xa, xc)
    assert np.array_equal(ba, bb) and np.array_equal(ba, bc)


def test_queued_iterations_follow_the_oracle_f32(P):
    """Three iterations queued in one call with the drift applied, against the
    oracle's three steps from the same start on the same moving data (rows far
    from the boundary, so the three masks are not in doubt)."""
    n, m = 512, 1200
    sys_ = W.gaussian(n, m, seed=8, dtype="f32")
    V = W.drift(n, 10, sigma=1e-3, seed=8)
    lam = 0.05
    x0 = sys_.z + 0.5
    say("queued f32 vs oracle")
    xg, bg, st = _run_calls(P, sys_, "f32", V, P.params(lam=lam, eps=1e-9), [3], None, x0)
    assert st.iters == 3
    x, b = x0.copy(), sys_.b.copy()
    for k in range(3):
        o = oracle.sweep(sys_.A, "f32", b, x)
        x, status = oracle.step(o.y, o.h, 0, lam, x)
        assert status == 0
        b = oracle.translate(sys_.A, "f32", b, V[k])
    assert np.linalg.norm(xg - x) <= 3 * TOL["f32"] * (np.linalg.norm(x) + lam), np.linalg.norm(xg - x)
    scale = np.abs(W.stored_to_f64(sys_.A, "f32")) @ np.abs(V[:3]).sum(axis=0) + np.abs(sys_.b)
    assert np.max(np.abs(bg - b) / scale) <= TOL["f32"]
