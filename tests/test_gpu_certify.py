"""The FP64 certificate of a stop, and the exact data the library keeps.

A stop decided from FP32 dot products (FP32 or BF16 storage) is confirmed by
a pass in FP64 over the same stored rows, on the exact right-hand side
bref + A w (w the FP64 sum of the translations applied); the final points are
then checked by the oracle against eq. 10 with no slack beyond FP64 rounding:
max violation <= eps_abs (1 + 1e-12).
"""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from parity import TOL, check_sweep

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


def exact_rhs(A, dtype, b0, V, steps):
    """b0 + A (V[0] + ... + V[steps-1]), the sum of the drift rows taken exactly
    rounded per coordinate (math.fsum), then one extended-precision translation."""
    if steps == 0:
        return np.asarray(b0, dtype=np.float64).copy()
    w = np.array([math.fsum(V[:steps, j]) for j in range(V.shape[1])])
    return oracle.translate(A, dtype, b0, w)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_certified_stop_is_eps_feasible_on_the_exact_data(P, dtype):
    """Eq. 10 on a moving system (section 5): the certified stop is
    eps-feasible on the data translated by every drift row applied, and the
    certificate's reported violation bounds the oracle's from above."""
    n, m = 400, 1000
    sys_ = W.gaussian(n, m, seed=81, dtype=dtype)
    V = W.drift(n, 600, sigma=1e-3, seed=81)
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype=dtype)
        s.set_drift(V)
        say(f"certified solve dtype={dtype}")
        st, code = s.solve(P.params(lam=0.05, eps=1e-6, max_iters=600))
        x, bq, _ = s.query(want_b=True)
    assert code == 0 and st.converged == 1 and st.certified == 1
    b = exact_rhs(sys_.A, dtype, sys_.b, V, st.iters)
    scale = np.abs(W.stored_to_f64(sys_.A, dtype)) @ np.abs(V[:st.iters]).sum(axis=0) + np.abs(sys_.b)
    assert np.max(np.abs(bq - b) / scale) <= 1e-12
    o = oracle.sweep(sys_.A, dtype, b, x)
    say(f"  steps {st.iters}, oracle dmax {o.dmax:.3e}, certificate {st.max_viol:.3e}, "
        f"eps_abs {1e-6 * o.binf:.3e}, working-b drift corrected {st.b_drift:.3e}")
    assert o.dmax <= 1e-6 * o.binf * (1 + 1e-12)
    assert o.dmax <= st.max_viol * (1 + 1e-12) + 1e-300
    assert st.max_viol <= st.eps_abs
    assert st.eps_abs == pytest.approx(1e-6 * o.binf, rel=1e-12)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_certified_stop_through_the_split_row_form(P, dtype):
    """The same moving system solved through the two-phase split-row sweep
    (forced): the stop it finds is certified and eps-feasible on the exact
    data, as through the one-pass sweep."""
    n, m = 400, 1000
    sys_ = W.gaussian(n, m, seed=81, dtype=dtype)
    V = W.drift(n, 600, sigma=1e-3, seed=81)
    blk, lpr, ch = {"f32": (256, 256, 8), "bf16": (256, 256, 4)}[dtype]
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype=dtype)
        s.set_tile(blk, lpr, ch, 0, 1, kind=1)
        assert s.get_tile()["kind"] == 1
        s.set_drift(V)
        say(f"certified split-row solve dtype={dtype}")
        st, code = s.solve(P.params(lam=0.05, eps=1e-6, max_iters=600))
        x, bq, _ = s.query(want_b=True)
    assert code == 0 and st.converged == 1 and st.certified == 1 and st.resident == 0
    b = exact_rhs(sys_.A, dtype, sys_.b, V, st.iters)
    o = oracle.sweep(sys_.A, dtype, b, x)
    say(f"  steps {st.iters}, oracle dmax {o.dmax:.3e}, certificate {st.max_viol:.3e}")
    assert o.dmax <= 1e-6 * o.binf * (1 + 1e-12)
    assert o.dmax <= st.max_viol * (1 + 1e-12) + 1e-300
    scale = np.abs(W.stored_to_f64(sys_.A, dtype)) @ np.abs(V[:st.iters]).sum(axis=0) + np.abs(sys_.b)
    assert np.max(np.abs(bq - b) / scale) <= 1e-12


def rounding_trap(dtype, n=64):
    """A box |x_j| <= 1000 and a point 3e-5 outside its face x_0 <= 1000.
    x is staged in FP32 by the FP32/BF16 sweep, and 1000 + 3e-5 rounds to 1000
    there (the FP32 spacing at 1000 is 2^-14 ~ 6.1e-5), so the working check
    sees the point on the face, not outside it.  With eps = 1e-8 relative
    (eps_abs = 1e-5) the point is not eps-feasible (eq. 10)."""
    I = np.eye(n)
    A64 = np.vstack([I, -I])
    b = np.full(2 * n, 1000.0)
    x = np.zeros(n)
    x[0] = 1000.0 + 3e-5
    return W.encode(A64, dtype), b, x


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f64"])
def test_certificate_overrules_a_working_precision_stop(P, dtype):
    A, b, x = rounding_trap(dtype)
    o = oracle.sweep(A, dtype, b, x)
    assert o.dmax == pytest.approx(3e-5, rel=1e-6) and o.h == 1
    lam = 1e-4
    with P.Solver() as s:
        s.set_system(A, b, x0=x, dtype=dtype)
        say(f"rounding trap dtype={dtype} uncertified")
        st0, code0 = s.solve(P.params(lam=lam, eps=1e-8, max_iters=50, certify=False))
        x0, _, _ = s.query()
        s.set_x(x)
        say(f"rounding trap dtype={dtype} certified")
        st1, code1 = s.solve(P.params(lam=lam, eps=1e-8, max_iters=50))
        x1, _, _ = s.query()
    assert code0 == 0 and code1 == 0 and st1.certified == 1
    if dtype == "f64":
        # the working precision is FP64 already: both take the step
        assert st0.iters == 1 and st1.iters == 1
    else:
        # the working check stops at x (wrongly); the certificate takes the step
        assert st0.iters == 0 and np.array_equal(x0, x)
        assert oracle.sweep(A, dtype, b, x0).dmax > 1e-8 * 1000.0
        assert st1.iters == 1
    o1 = oracle.sweep(A, dtype, b, x1)
    assert o1.dmax <= 1e-8 * o1.binf * (1 + 1e-12)
    # the certificate's step is the FP64 ModAP step of eq. 12 from x
    xo, status = oracle.step(o.y, o.h, 0, lam, x)
    assert status == 0 and np.allclose(x1, xo, rtol=0, atol=1e-12 * 1000)


def test_certificate_in_batch_and_server(P):
    """The same trap solved in a batch (beside an ordinary system) and served:
    both take the step the certificate asks for and end certified."""
    A, b, x = rounding_trap("f32")
    g = W.gaussian(300, 700, seed=5, dtype="f32")
    with P.Batch("f32") as B:
        i_trap = B.add(A, b, x0=x)
        i_g = B.add(g.A, g.b, x0=g.z)            # starts strictly feasible: certified at once
        say("batch trap")
        B.solve(P.params(lam=1e-4, eps=1e-8, max_iters=20000))
        xt, bt, qt = B.query(i_trap, want_b=True)
        xg, bg, qg = B.query(i_g, want_b=True)
    assert qt.state == 1 and qt.certified == 1 and qt.iters == 1
    assert oracle.sweep(A, "f32", b, xt).dmax <= 1e-8 * 1000.0 * (1 + 1e-12)
    og = oracle.sweep(g.A, "f32", g.b, xg)
    assert qg.certified == 1 and qg.iters == 0 and og.dmax <= 1e-8 * og.binf * (1 + 1e-12)
    with P.Server("f32", budget_bytes=1e9, prm=P.params(lam=1e-4, eps=1e-8, max_iters=100),
                  iters_per_round=4) as S:
        t = S.submit(A, b, x0=x)
        say("server trap")
        for _ in range(50):
            if S.round() == 0:
                break
        info = S.info(t)
        xs = S.result(t)
    assert info["state"] == 2 and info["status"] == 1 and info["iters"] == 1
    assert oracle.sweep(A, "f32", b, xs).dmax <= 1e-8 * 1000.0 * (1 + 1e-12)


def test_full_length_fp32_chase_is_certified_on_the_exact_data(P):
    """The FP32 n = 8192, m = 16384 system chased from x0 = 0 under a drift of
    N(0, 1e-2^2) per coordinate per iteration (lambda = 1, eps = 1e-6
    relative, at most 3000 steps).  The oracle checks the final x on
    b0 + A (V[0] + ... + V[k-1]); the drift of the working right-hand side,
    which the sweep translated with FP32 dot products, is reported."""
    n, m = 8192, 16384
    say("generating the n=8192 m=16384 FP32 system")
    sys_ = W.gaussian(n, m, 0, "f32")
    V = W.drift(n, 3000, sigma=1e-2, seed=1)
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype="f32")
        s.set_drift(V)
        say("chase")
        st, code = s.solve(P.params(lam=1.0, eps=1e-6, max_iters=3000), raise_on_stop=False)
        x, bq, _ = s.query(want_b=True)
    say(f"  code {code}, steps {st.iters}, certified {st.certified}, working-b drift {st.b_drift:.3e}, "
        f"eps_abs {st.eps_abs:.3e}")
    assert code == 0 and st.certified == 1
    b = exact_rhs(sys_.A, "f32", sys_.b, V, st.iters)
    scale = np.abs(W.stored_to_f64(sys_.A, "f32")) @ np.abs(V[:st.iters]).sum(axis=0) + np.abs(sys_.b)
    err_b = float(np.max(np.abs(bq - b) / scale))
    o = oracle.sweep(sys_.A, "f32", b, x)
    say(f"  oracle dmax {o.dmax:.3e} (eps_abs {1e-6 * o.binf:.3e}), |b - exact| / scale {err_b:.2e}")
    assert err_b <= 1e-12
    assert o.dmax <= 1e-6 * o.binf * (1 + 1e-12)
    # the working b drifted by far less than eps_abs before the certificate rebased it
    assert st.b_drift < 0.5 * st.eps_abs


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_query_of_b_does_not_change_the_iteration(P, dtype):
    """Reading b commits nothing: a run with queries of b between its calls
    (with a one-shot translation and a drift row pending) takes the same
    steps, bit for bit, as the same run without them."""
    sys_ = W.gaussian(300, 800, seed=17, dtype=dtype)
    V = W.drift(300, 40, sigma=1e-3, seed=17)
    v = np.random.default_rng(17).normal(scale=1e-2, size=300)
    prm = P.params(lam=0.05, eps=1e-12)
    out = []
    for read in (False, True):
        with P.Solver() as s:
            s.set_system(sys_.A, sys_.b, dtype=dtype)
            s.set_drift(V)
            s.update_coeffs(translate=v)
            if read:
                s.query(want_b=True)
            s.iterate(7, prm)
            if read:
                s.query(want_b=True)
            s.update_coeffs(translate=-v)
            if read:
                s.query(want_b=True)
            s.iterate(5, prm)
            x, b, st = s.query(want_b=True)
            out.append((x, b, st.iters))
    assert out[0][2] == out[1][2] == 12
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_row_replacement_after_drift_steps(P, dtype):
    """Rows replaced after k drift steps (the translation V[k-1] still due at
    the next sweep) keep the right-hand side the caller gave: the data are
    the translated system with the rows replaced (section 1: coefficients and
    right-hand side change during the computation)."""
    n, m, k = 256, 700, 6
    sys_ = W.gaussian(n, m, seed=23, dtype=dtype)
    V = W.drift(n, 40, sigma=1e-2, seed=23)
    idx, rows, nb = W.replacement_rows(sys_, 25, seed=23)
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype=dtype)
        s.set_drift(V)
        s.iterate(k, P.params(lam=0.05, eps=1e-12))
        x, _, st = s.query()
        assert st.iters == k
        say(f"replacement after drift dtype={dtype}")
        s.update_coeffs(rows=idx, new_rows=rows, new_b=nb)
        g = s.eval_sweep(x)
        _, bq, _ = s.query(want_x=False, want_b=True)
    b = exact_rhs(sys_.A, dtype, sys_.b, V, k)
    A2, b2 = oracle.replace_rows(sys_.A, dtype, b, idx, rows, nb)
    np.testing.assert_allclose(bq[idx], nb, rtol=1e-12, atol=1e-12)
    assert np.max(np.abs(bq - b2) / (np.abs(b2) + 1.0)) <= 1e-12
    o = oracle.sweep(A2, dtype, b2, x)
    check_sweep(A2, dtype, o, g.y, g.h, g.max_viol, g.r, label=f"replace-after-drift {dtype}")


def test_repeated_device_row_index_is_rejected(P):
    """A replacement with a repeated device-side row index is refused on the
    device before any row is written: the next synchronising call reports
    E_ZERO_ROW, and the stored system is unchanged."""
    import torch
    dev = torch.device("cuda:0")
    sys_ = W.gaussian(200, 500, seed=29, dtype="f32")
    idx = np.array([3, 7, 3], dtype=np.int64)
    rng = np.random.default_rng(29)
    rows = W.encode(rng.normal(size=(3, 200)), "f32")
    nb = np.ones(3)
    x = sys_.z + rng.normal(scale=0.2, size=200)
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype="f32")
        say("repeated device row index")
        s.update_coeffs(rows=torch.from_numpy(idx).to(dev), new_rows=torch.from_numpy(rows).to(dev),
                        new_b=torch.from_numpy(nb).to(dev))
        with pytest.raises(P.ModapError, match="E_ZERO_ROW"):
            s.iterate(1, P.params())
        g = s.eval_sweep(x)
    o = oracle.sweep(sys_.A, "f32", sys_.b, x)
    check_sweep(sys_.A, "f32", o, g.y, g.h, g.max_viol, g.r, label="unchanged after a refused replacement")


def test_server_inputs_may_be_released_right_after_submit(P):
    """modap_server_submit copies its inputs: overwriting host arrays and
    device tensors right after the call (NaN and zeros) changes nothing; the
    requests finish certified and eps-feasible on the data submitted."""
    import torch
    dev = torch.device("cuda:0")
    systems = [W.gaussian(n, 4 * n, seed=90 + n, dtype="bf16") for n in (300, 4500)]
    keep = [(s.A.copy(), s.b.copy()) for s in systems]
    prm = P.params(lam=0.1, eps=1e-6, max_iters=5000)
    with P.Server("bf16", budget_bytes=40e9, prm=prm, iters_per_round=8) as S:
        A0, b0 = systems[0].A.copy(), systems[0].b.copy()
        t0 = S.submit(A0, b0)
        A0[:] = 0
        b0[:] = np.nan
        dA = torch.from_numpy(systems[1].A.view(np.int16)).to(dev)
        db = torch.from_numpy(systems[1].b).to(dev)
        torch.cuda.synchronize()
        t1 = S.submit(dA, db)
        dA.zero_()
        db.fill_(float("nan"))
        torch.cuda.synchronize()
        say("server submit copies")
        for _ in range(5000):
            if S.round() == 0:
                break
        infos = [S.info(t) for t in (t0, t1)]
        xs = [S.result(t) for t in (t0, t1)]
    assert all(i["state"] == 2 and i["status"] == 1 for i in infos), infos
    for (A, b), x in zip(keep, xs):
        o = oracle.sweep(A, "bf16", b, x)
        assert o.dmax <= 1e-6 * o.binf * (1 + 1e-12)
