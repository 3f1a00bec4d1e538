"""Seeded random shapes and batches, against the oracle.

The shapes are drawn log-uniformly (n from 1 to 20000, m from 1 to 6000) with
every storage type, so that row lengths fall anywhere relative to the tile
widths of the one-pass, short-row, split-row and resident forms.  Each case
compares a stateless sweep at a point with violated rows element by element
(r, y, h, dmax), then one iteration against the oracle's step from the same
point.  Random batches (3 to 9 systems of any row length the batch covers,
with random tiles) take two steps of every system against the oracle;
random data-update sequences (drift, row replacement, translation) take a
step on the data the update rules define; random served request streams end
eps-feasible, each request the same bits alone as in the stream; randomly
forced one-pass tiles sweep as the oracle does; random certified solves end
eps-feasible on the exact data; a context reloaded with random systems and a
batch whose systems come and go at random keep stepping as the oracle does;
served requests receiving random updates end eps-feasible on their final data;
the relaxed step of Algorithm 1 matches the oracle's on random shapes;
contexts driven concurrently from threads give the bits of sequential runs.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from parity import TOL, check_sweep, weighted_abs_rows

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


def draw(k):
    rng = np.random.default_rng(np.random.SeedSequence([2003, 9956, k]))
    n = int(np.exp(rng.uniform(0.0, np.log(20000.0))))
    m = int(np.exp(rng.uniform(0.0, np.log(6000.0))))
    dtype = ("f64", "f32", "bf16")[int(rng.integers(3))]
    return max(n, 1), max(m, 1), dtype


CASES = [draw(k) for k in range(96)]


@pytest.mark.parametrize("n,m,dtype", CASES)
def test_random_shape_sweep_and_step_match_oracle(P, n, m, dtype):
    sys_ = W.gaussian(n, m, seed=n * 31 + m, dtype=dtype)
    rng = np.random.default_rng(n + 7 * m)
    x = sys_.z + rng.normal(scale=1.5 / np.sqrt(n) + 0.1, size=n)
    lam, tol = 0.5, TOL[dtype]
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, x0=x, dtype=dtype)
        say(f"random shape n={n} m={m} dtype={dtype} tile={s.get_tile()}")
        g = s.eval_sweep(x)
        o = oracle.sweep(sys_.A, dtype, sys_.b, x)
        check_sweep(sys_.A, dtype, o, g.y, g.h, g.max_viol, g.r, label=f"random {dtype} {n}x{m}")
        st = s.iterate(1, P.params(lam=lam, eps=1e-12))
        x1 = s.query()[0]
    xo, status = oracle.step(o.y, o.h, 0, lam, x)
    if status != 0:                     # nothing violated: the point stays
        assert st.converged == 1 and np.array_equal(x1, x)
        return
    near = o.r > -tol * o.t
    s_y = np.linalg.norm(weighted_abs_rows(sys_.A, dtype, np.where(near, o.t / o.nu, 0)))
    bound = tol * (np.linalg.norm(x) + lam * s_y / np.linalg.norm(o.y))
    assert np.linalg.norm(x1 - xo) <= bound, (np.linalg.norm(x1 - xo), bound)


ROW_LIMIT = {"f32": 2048, "bf16": 4096, "f64": 1024}


def draw_batch(k):
    rng = np.random.default_rng(np.random.SeedSequence([2003, 9956, 1000 + k]))
    dtype = ("f64", "f32", "bf16")[k % 3]
    count = int(rng.integers(3, 10))
    shapes = []
    for _ in range(count):
        n = int(np.exp(rng.uniform(0.0, np.log(ROW_LIMIT[dtype]))))
        m = int(np.exp(rng.uniform(0.0, np.log(3000.0))))
        shapes.append((max(n, 1), max(m, 1)))
    kib = [int(2 ** rng.integers(5, 15)) for _ in range(4)]
    min_items = int((0, 1, 2, 4, 16)[int(rng.integers(5))])
    return dtype, shapes, kib, min_items


@pytest.mark.parametrize("k", range(24))
def test_random_batch_mix_follows_oracle(P, k):
    """A seeded random batch (3 to 9 systems of any row length the batch
    covers, a random tile): two steps of every system against the oracle,
    and one system alone against the mix at the same tile and call
    boundaries."""
    dtype, shapes, kib, min_items = draw_batch(k)
    systems = [W.gaussian(n, m, seed=k * 101 + i, dtype=dtype) for i, (n, m) in enumerate(shapes)]
    lam, tol = 0.4, TOL[dtype]
    prm = P.params(lam=lam, eps=1e-12)
    xs = [s_.z + np.random.default_rng(i).normal(scale=1.5 / np.sqrt(s_.n) + 0.1, size=s_.n)
          for i, s_ in enumerate(systems)]
    x_first = xs[-1].copy()
    stopped = [False] * len(systems)
    with P.Batch(dtype) as B:
        B.set_tile(item_kib=kib, min_items=min_items)
        ids = [B.add(s_.A, s_.b, x0=x) for s_, x in zip(systems, xs)]
        for step in range(2):
            say(f"random batch k={k} {dtype} shapes={shapes} tile={B.get_tile()} step={step}")
            B.iterate(1, prm)
            for i, (s_, sid) in enumerate(zip(systems, ids)):
                x1, _, q = B.query(sid)
                if stopped[i]:
                    assert np.array_equal(x1, xs[i])
                    continue
                o = oracle.sweep(s_.A, dtype, s_.b, xs[i])
                xo, status = oracle.step(o.y, o.h, 0, lam, xs[i])
                if status != 0:
                    assert q.converged == 1 and np.array_equal(x1, xs[i]), (i, step)
                    stopped[i] = True
                    continue
                near = o.r > -tol * o.t
                s_y = np.linalg.norm(weighted_abs_rows(s_.A, dtype, np.where(near, o.t / o.nu, 0)))
                bound = tol * (np.linalg.norm(xs[i]) + lam * s_y / np.linalg.norm(o.y))
                assert q.iters == step + 1 and np.linalg.norm(x1 - xo) <= bound, (i, step)
                xs[i] = x1
    with P.Batch(dtype) as B:
        B.set_tile(item_kib=kib, min_items=min_items)
        sid = B.add(systems[-1].A, systems[-1].b, x0=x_first)
        B.iterate(1, prm)
        B.iterate(1, prm)
        assert np.array_equal(B.query(sid)[0], xs[-1])


@pytest.mark.parametrize("k", range(24))
def test_random_shape_data_updates_follow_oracle(P, k):
    """One step under the drift schedule, then rows replaced and a one-shot
    translation, then a second step: the second step against the oracle's on
    the data as the update rules define them (the replaced rows exactly as
    given on the data after the drift row already due; the translation on
    every row), and the right-hand side read back against the exact data."""
    rng = np.random.default_rng(np.random.SeedSequence([2003, 9956, 2000 + k]))
    n = max(1, int(np.exp(rng.uniform(0.0, np.log(20000.0)))))
    m = max(2, int(np.exp(rng.uniform(np.log(2.0), np.log(4000.0)))))
    dtype = ("f64", "f32", "bf16")[k % 3]
    sys_ = W.gaussian(n, m, seed=7 * n + m, dtype=dtype)
    V = W.drift(n, 3, sigma=1e-3, seed=k)
    v = rng.normal(scale=1e-2, size=n)
    idx, rows, nb = W.replacement_rows(sys_, max(1, m // 10), seed=k)
    x0 = sys_.z + rng.normal(scale=1.5 / np.sqrt(n) + 0.1, size=n)
    lam, tol = 0.3, TOL[dtype]
    prm = P.params(lam=lam, eps=1e-12)
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, x0=x0, dtype=dtype)
        s.set_drift(V)
        say(f"random updates k={k} n={n} m={m} dtype={dtype} tile={s.get_tile()}")
        s.iterate(1, prm)
        x1, _, st1 = s.query()
        if st1.converged:          # the start is feasible: no step, so no drift row was applied
            return
        s.update_coeffs(rows=idx, new_rows=rows, new_b=nb, translate=v)
        st2 = s.iterate(1, prm)
        x2, bq, st = s.query(want_b=True)
    b1 = oracle.translate(sys_.A, dtype, sys_.b, V[0])
    A2, b2 = oracle.replace_rows(sys_.A, dtype, b1, idx, rows, nb)
    b3 = oracle.translate(A2, dtype, b2, v)
    o = oracle.sweep(A2, dtype, b3, x1)
    xo, status = oracle.step(o.y, o.h, 0, lam, x1)
    if status != 0 or st.converged:
        # a feasible point stays where it is (and the last translation waits)
        assert np.array_equal(x2, x1)
        return
    assert st1.iters == 1 and st.iters == 2
    near = o.r > -tol * o.t
    s_y = np.linalg.norm(weighted_abs_rows(A2, dtype, np.where(near, o.t / o.nu, 0)))
    bound = tol * (np.linalg.norm(x1) + lam * s_y / np.linalg.norm(o.y))
    assert np.linalg.norm(x2 - xo) <= bound, (np.linalg.norm(x2 - xo), bound)
    b4 = oracle.translate(A2, dtype, b3, V[1])
    scale = (np.abs(W.stored_to_f64(A2, dtype)) @ (np.abs(V[0]) + np.abs(V[1]) + np.abs(v))
             + np.abs(sys_.b) + np.abs(b2))
    assert np.max(np.abs(bq - b4) / scale) <= 1e-12


@pytest.mark.parametrize("k", range(6))
def test_random_server_mix_results_equal_alone(P, k):
    """A seeded random stream of requests (short and long rows, with or
    without drift schedules, rounds between some submissions, a random limit
    on long requests): every request ends eps-feasible on its final data,
    and a chosen one takes the same bits and steps as served alone."""
    rng = np.random.default_rng(np.random.SeedSequence([2003, 9956, 3000 + k]))
    dtype = ("bf16", "f32", "f64")[k % 3]
    count = int(rng.integers(3, 7))
    reqs = []
    for i in range(count):
        n = int(np.exp(rng.uniform(np.log(16.0), np.log(3000.0))))
        m = int(n * rng.uniform(2.0, 4.0))
        sys_ = W.gaussian(n, m, seed=k * 97 + i, dtype=dtype)
        V = W.drift(n, 400, sigma=1e-5, seed=k * 97 + i) if rng.random() < 0.5 else None
        reqs.append((sys_, V, bool(rng.random() < 0.5)))
    max_long = int(rng.integers(0, 2))
    target = int(rng.integers(count))
    prm = P.params(lam=0.1, eps=1e-6, max_iters=5000)

    def serve(items):
        with P.Server(dtype, budget_bytes=20e9, prm=prm, iters_per_round=8) as S:
            S.set_max_long(max_long)
            tickets = []
            for sys_, V, round_after in items:
                tickets.append(S.submit(sys_.A, sys_.b, V=V))
                if round_after:
                    S.round()
            for _ in range(20000):
                if S.round() == 0:
                    break
            infos = [S.info(t) for t in tickets]
            return infos, [S.result(t) for t in tickets]

    say(f"random server k={k} {dtype} shapes={[r[0].A.shape for r in reqs]} max_long={max_long}")
    infos, xs = serve(reqs)
    for (sys_, V, _), info, x in zip(reqs, infos, xs):
        assert info["state"] == 2 and info["status"] == 1, info
        b = sys_.b.copy()
        if V is not None:
            for q in range(min(info["iters"], V.shape[0])):
                b = oracle.translate(sys_.A, dtype, b, V[q])
        o = oracle.sweep(sys_.A, dtype, b, x)
        assert o.dmax <= 1e-6 * o.binf * (1 + 1e-12), (sys_.A.shape, o.dmax, o.binf)
    alone_infos, alone_xs = serve([reqs[target][:2] + (False,)])
    assert alone_infos[0]["iters"] == infos[target]["iters"]
    assert np.array_equal(alone_xs[0], xs[target])


@pytest.mark.parametrize("k", range(48))
def test_random_forced_tile_sweep_matches_oracle(P, k):
    """A compiled one-pass sweep shape drawn at random, forced on a row it
    covers with a ragged tail, at a random grid and row order, with or
    without a pending translation: the sweep against the oracle's."""
    from test_gpu_parity import ALL_SHAPES, VEC
    from parity import check_sweep
    rng = np.random.default_rng(np.random.SeedSequence([2003, 9956, 5000 + k]))
    dtype = ("f64", "f32", "bf16")[k % 3]
    shapes = ALL_SHAPES[dtype]
    blk, lpr, ch, rs, pd = shapes[int(rng.integers(len(shapes)))]
    cover = lpr * VEC[dtype] * ch
    n = int(rng.integers(max(1, cover // 4), cover + 1))
    m = max(1, int(np.exp(rng.uniform(0.0, np.log(5000.0)))))
    grid = int((0, 1, 2, 3, 7, 64, 256)[int(rng.integers(7))])
    il = int(rng.integers(2))
    translate = bool(rng.random() < 0.5)
    sys_ = W.gaussian(n, m, seed=k, dtype=dtype)
    x = sys_.z + rng.normal(scale=1.5 / np.sqrt(n) + 0.1, size=n)
    v = rng.normal(scale=1e-2, size=n)
    label = f"{dtype} n={n} m={m} tile={blk}/{lpr}/{ch}/{rs}/{pd} grid={grid} il={il} v={translate}"
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype=dtype)
        s.set_tile(blk, lpr, ch, grid, rs, depth=pd, interleave=il)
        say(f"random tile {label}")
        if translate:
            s.update_coeffs(translate=v)
        g = s.eval_sweep(x)
    b = oracle.translate(sys_.A, dtype, sys_.b, v) if translate else sys_.b
    o = oracle.sweep(sys_.A, dtype, b, x)
    check_sweep(sys_.A, dtype, o, g.y, g.h, g.max_viol, g.r, label=label)


@pytest.mark.parametrize("k", range(12))
def test_random_certified_solve_is_feasible_on_the_exact_data(P, k):
    """A random system solved under a random drift: the certified stop is
    eps-feasible on the exact data (the system translated by the exact sum of
    the drift rows applied), bounded by the certificate's reported violation,
    and the right-hand side read back is that of the exact data."""
    import math
    rng = np.random.default_rng(np.random.SeedSequence([2003, 9956, 7000 + k]))
    dtype = ("f32", "bf16", "f64")[k % 3]
    n = int(np.exp(rng.uniform(np.log(8.0), np.log(3000.0))))
    m = int(n * rng.uniform(1.5, 4.0))
    sys_ = W.gaussian(n, m, seed=k + 91, dtype=dtype)
    V = W.drift(n, 3000, sigma=float(10 ** rng.uniform(-6, -3.5)), seed=k)
    lam = float(rng.choice([0.05, 0.1, 0.2]))
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, dtype=dtype)
        s.set_drift(V)
        say(f"random certified solve k={k} {dtype} n={n} m={m} lam={lam}")
        st, code = s.solve(P.params(lam=lam, eps=1e-6, max_iters=3000))
        x, bq, _ = s.query(want_b=True)
    assert code == 0 and st.converged == 1 and st.certified == 1
    w = np.array([math.fsum(V[:st.iters, j]) for j in range(n)])
    b = oracle.translate(sys_.A, dtype, sys_.b, w)
    o = oracle.sweep(sys_.A, dtype, b, x)
    assert o.dmax <= 1e-6 * o.binf * (1 + 1e-12)
    assert o.dmax <= st.max_viol * (1 + 1e-12) + 1e-300
    scale = np.abs(W.stored_to_f64(sys_.A, dtype)) @ np.abs(V[:st.iters]).sum(axis=0) + np.abs(sys_.b)
    assert np.max(np.abs(bq - b) / scale) <= 1e-12


def _step_matches(A, dtype, b, x, x1, lam):
    o = oracle.sweep(A, dtype, b, x)
    xo, status = oracle.step(o.y, o.h, 0, lam, x)
    if status != 0:
        return np.array_equal(x1, x)
    tol = TOL[dtype]
    near = o.r > -tol * o.t
    s_y = np.linalg.norm(weighted_abs_rows(A, dtype, np.where(near, o.t / o.nu, 0)))
    return np.linalg.norm(x1 - xo) <= tol * (np.linalg.norm(x) + lam * s_y / np.linalg.norm(o.y))


def test_one_context_reloaded_with_random_systems(P):
    """One context loaded 30 times with systems of random size and storage
    (its buffers grow and shrink, the resident plan and the sweep shape are
    chosen again): each load sweeps and steps as the oracle does."""
    rng = np.random.default_rng(np.random.SeedSequence([2003, 9956, 8000]))
    with P.Solver() as s:
        for k in range(30):
            dtype = ("f64", "f32", "bf16")[int(rng.integers(3))]
            n = max(1, int(np.exp(rng.uniform(0.0, np.log(20000.0)))))
            m = max(1, int(np.exp(rng.uniform(0.0, np.log(5000.0)))))
            label = f"reload k={k} {dtype} n={n} m={m}"
            say(label)
            sys_ = W.gaussian(n, m, seed=k, dtype=dtype)
            x = sys_.z + rng.normal(scale=1.5 / np.sqrt(n) + 0.1, size=n)
            s.set_system(sys_.A, sys_.b, x0=x, dtype=dtype)
            g = s.eval_sweep(x)
            o = oracle.sweep(sys_.A, dtype, sys_.b, x)
            check_sweep(sys_.A, dtype, o, g.y, g.h, g.max_viol, g.r, label=label)
            s.iterate(1, P.params(lam=0.5, eps=1e-12))
            assert _step_matches(sys_.A, dtype, sys_.b, x, s.query()[0], 0.5), label


@pytest.mark.parametrize("trial", range(6))
def test_random_batch_membership_churn(P, trial):
    """Systems of random size join and leave a batch at random between
    iterations: every live system steps as the oracle does from its own
    point, and a system that stopped stays where it is."""
    rng = np.random.default_rng(np.random.SeedSequence([2003, 9956, 9000 + trial]))
    dtype = ("f64", "f32", "bf16")[trial % 3]
    limit = ROW_LIMIT[dtype]
    live = {}
    with P.Batch(dtype) as B:
        for it in range(12):
            for sid in list(live):
                if rng.random() < 0.3:
                    B.remove(sid)
                    del live[sid]
            for _ in range(int(rng.integers(0, 4))):
                n = max(1, int(np.exp(rng.uniform(0.0, np.log(limit)))))
                m = max(1, int(np.exp(rng.uniform(0.0, np.log(3000.0)))))
                sys_ = W.gaussian(n, m, seed=trial * 100 + it * 7 + len(live), dtype=dtype)
                x = sys_.z + rng.normal(scale=1.5 / np.sqrt(n) + 0.1, size=n)
                live[B.add(sys_.A, sys_.b, x0=x)] = [sys_, x, False]
            if not live:
                continue
            say(f"churn trial={trial} it={it} {dtype} live={len(live)}")
            B.iterate(1, P.params(lam=0.4, eps=1e-12))
            for sid, rec in live.items():
                sys_, x, stopped = rec
                x1, _, q = B.query(sid)
                if stopped:
                    assert np.array_equal(x1, x), (it, sid)
                    continue
                o = oracle.sweep(sys_.A, dtype, sys_.b, x)
                _, status = oracle.step(o.y, o.h, 0, 0.4, x)
                if status != 0:
                    assert q.converged == 1 and np.array_equal(x1, x), (it, sid)
                    rec[2] = True
                    continue
                assert _step_matches(sys_.A, dtype, sys_.b, x, x1, 0.4), (it, sid, sys_.A.shape)
                rec[1] = x1


@pytest.mark.parametrize("trial", range(6))
def test_random_server_updates_end_feasible(P, trial):
    """A random stream of requests that receive random row replacements and
    translations between rounds, from host or device memory at random: each
    request ends eps-feasible on its final data (the updates applied in
    order by the oracle)."""
    import torch
    dev = torch.device("cuda:0")

    def to_dev(a):
        if a is None:
            return None
        if a.dtype == np.uint16:
            return torch.from_numpy(a.view(np.int16).copy()).to(dev)
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    rng = np.random.default_rng(np.random.SeedSequence([2003, 9956, 11000 + trial]))
    dtype = ("bf16", "f32", "f64")[trial % 3]
    systems = []
    for i in range(int(rng.integers(3, 6))):
        n = int(np.exp(rng.uniform(np.log(16.0), np.log(5000.0))))
        systems.append(W.gaussian(n, int(n * rng.uniform(2.0, 4.0)), seed=trial * 31 + i, dtype=dtype))
    prm = P.params(lam=0.1, eps=1e-6, max_iters=6000)
    with P.Server(dtype, budget_bytes=40e9, prm=prm, iters_per_round=8) as S:
        S.set_max_long(int(rng.integers(0, 2)))
        tickets = [S.submit(s_.A, s_.b) for s_ in systems]
        data = {t: (s_.A.copy(), s_.b.copy(), s_) for t, s_ in zip(tickets, systems)}
        say(f"random server updates trial={trial} {dtype} shapes={[s_.A.shape for s_ in systems]}")
        for r in range(3000):
            if S.round() == 0:
                break
            for t in tickets:
                if S.info(t)["state"] != 1 or rng.random() > 0.2:
                    continue
                A, b, s_ = data[t]
                v = rng.normal(scale=1e-5, size=s_.n) if rng.random() < 0.7 else None
                k = int(rng.integers(0, max(1, s_.m // 20) + 1))
                idx = rows = nb = None
                if k:
                    idx, rows, nb = W.replacement_rows(W.System(A, b, s_.x0, dtype, s_.z, {}), k,
                                                       seed=trial * 10007 + r)
                if rng.random() < 0.5:
                    S.update(t, rows=to_dev(idx), new_rows=to_dev(rows), new_b=to_dev(nb), translate=to_dev(v))
                else:
                    S.update(t, rows=idx, new_rows=rows, new_b=nb, translate=v)
                if k:
                    A, b = oracle.replace_rows(A, dtype, b, idx, rows, nb)
                if v is not None:
                    b = oracle.translate(A, dtype, b, v)
                data[t] = (A, b, s_)
        infos = [S.info(t) for t in tickets]
        xs = [S.result(t) for t in tickets]
    for t, x, info in zip(tickets, xs, infos):
        assert info["state"] == 2 and info["status"] == 1, info
        A, b, _ = data[t]
        o = oracle.sweep(A, dtype, b, x)
        assert o.dmax <= 1e-6 * o.binf * (1 + 1e-12)


@pytest.mark.parametrize("k", range(48))
def test_random_shape_relaxed_step_matches_oracle(P, k):
    """Algorithm 1 with relaxation (x <- x - (lambda/h) y) on a random shape:
    one step against the oracle's.  h is the step's divisor, so the points
    are compared where no row is in the ambiguous band (h then agrees
    exactly); otherwise h must agree up to the band's rows."""
    rng = np.random.default_rng(np.random.SeedSequence([2003, 9956, 13000 + k]))
    n = max(1, int(np.exp(rng.uniform(0.0, np.log(20000.0)))))
    m = max(1, int(np.exp(rng.uniform(0.0, np.log(6000.0)))))
    dtype = ("f64", "f32", "bf16")[k % 3]
    lam = float(rng.uniform(0.2, 1.9))
    sys_ = W.gaussian(n, m, seed=n * 13 + m, dtype=dtype)
    x = sys_.z + rng.normal(scale=1.5 / np.sqrt(n) + 0.1, size=n)
    tol = TOL[dtype]
    with P.Solver() as s:
        s.set_system(sys_.A, sys_.b, x0=x, dtype=dtype)
        say(f"relaxed step k={k} n={n} m={m} dtype={dtype} lam={lam:.3f}")
        st = s.iterate(1, P.params(lam=lam, eps=1e-12, step=P.STEP_AVG))
        x1, _, st = s.query()
    o = oracle.sweep(sys_.A, dtype, sys_.b, x)
    xo, status = oracle.step(o.y, o.h, 1, lam, x)
    if status != 0:
        assert st.converged == 1 and np.array_equal(x1, x)
        return
    band = int((np.abs(o.r) <= tol * o.t).sum())
    assert abs(int(st.h) - o.h) <= band
    if band:
        return
    near = o.r > -tol * o.t
    s_y = np.linalg.norm(weighted_abs_rows(sys_.A, dtype, np.where(near, o.t / o.nu, 0)))
    bound = tol * (np.linalg.norm(x) + lam * s_y / o.h)
    assert np.linalg.norm(x1 - xo) <= bound, (np.linalg.norm(x1 - xo), bound)


def test_contexts_driven_from_threads_equal_sequential_runs(P):
    """Eight contexts, each driven by its own host thread on its own stream
    (their kernels overlap on the device; small systems take the resident
    form, larger ones two kernels per iteration): sweeps, queued iterations
    under drift and solves give the same bits as the same work run one
    context after another."""
    import threading
    import torch

    def job(k, stream, out):
        rng = np.random.default_rng(np.random.SeedSequence([2003, 9956, 14000 + k]))
        dtype = ("f64", "f32", "bf16")[k % 3]
        n = int(np.exp(rng.uniform(np.log(16.0), np.log(6000.0))))
        m = int(n * rng.uniform(1.5, 3.0))
        sys_ = W.gaussian(n, m, seed=k, dtype=dtype)
        V = W.drift(n, 400, sigma=1e-5, seed=k)
        x0 = sys_.z + rng.normal(scale=1.5 / np.sqrt(n) + 0.1, size=n)
        with P.Solver(0, stream=stream.cuda_stream if stream is not None else None) as s:
            s.set_system(sys_.A, sys_.b, x0=x0, dtype=dtype)
            g = s.eval_sweep(x0)
            s.set_drift(V)
            s.iterate(20, P.params(lam=0.2, eps=1e-9))
            x20 = s.query()[0]
            st, code = s.solve(P.params(lam=0.2, eps=1e-6, max_iters=3000), raise_on_stop=False)
            out[k] = (g.y.copy(), g.h, x20, int(code), int(st.iters), s.query()[0], int(st.resident))

    seq, par = {}, {}
    for k in range(8):
        job(k, None, seq)
    streams = [torch.cuda.Stream() for _ in range(8)]
    threads = [threading.Thread(target=job, args=(k, streams[k], par)) for k in range(8)]
    say("eight contexts from eight threads")
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=300)
    assert sorted(par) == list(range(8))
    assert {par[k][6] for k in range(8)} == {0, 1}      # both iteration forms ran
    for k in range(8):
        a, b = seq[k], par[k]
        assert np.array_equal(a[0], b[0]) and a[1] == b[1] and np.array_equal(a[2], b[2]), k
        assert a[3] == b[3] and a[4] == b[4] and np.array_equal(a[5], b[5]), k
