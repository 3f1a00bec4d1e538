"""GPU parity of the batched sweep (many systems, one persistent launch).

Each system of a batch is checked against the CPU oracle step by step from
the GPU's own x (the tolerances of tests/parity.py), and a system's results
must be the same bits whether it is alone in a batch or mixed with others."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))

import oracle
import workloads as W
from parity import TOL, weighted_abs_rows

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "these tests need the GPU"
    import paper_2003_09956_amd as P
    P.lib()
    return P


# row lengths covering every chunk bucket (1, 2, 4, 8 chunks per lane) with ragged ends
SHAPES = {"f32": [(64, 150), (255, 700), (300, 1201), (513, 1100), (1000, 2500), (2048, 4100)],
          "bf16": [(100, 300), (511, 1500), (1024, 2100), (2000, 4000), (4096, 5000)],
          "f64": [(60, 200), (129, 500), (500, 1500), (1024, 2048)]}


def step_bound(sys_, dtype, o, x, lam):
    tol = TOL[dtype]
    near = o.r > -tol * o.t
    s_y = np.linalg.norm(weighted_abs_rows(sys_.A, dtype, np.where(near, o.t / o.nu, 0)))
    return tol * (np.linalg.norm(x) + lam * s_y / np.linalg.norm(o.y))


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f64"])
def test_batch_steps_match_oracle(P, dtype):
    """Every system of a mixed batch, three single iterations, each compared
    with the oracle's step from the GPU's previous x."""
    systems = [W.gaussian(n, m, seed=n + m, dtype=dtype) for (n, m) in SHAPES[dtype]]
    lam = 0.3
    prm = P.params(lam=lam, eps=1e-9)
    with P.Batch(dtype) as B:
        ids = [B.add(s.A, s.b, x0=s.z + 0.3) for s in systems]
        xs = [s.z + 0.3 for s in systems]
        for k in range(3):
            say(f"batch step k={k} dtype={dtype}")
            st = B.iterate(1, prm)
            assert st.running == len(systems)
            for sid, sys_ in zip(ids, systems):
                x1, _, q = B.query(sid)
                o = oracle.sweep(sys_.A, dtype, sys_.b, xs[sid])
                xo, status = oracle.step(o.y, o.h, 0, lam, xs[sid])
                assert status == 0 and q.iters == k + 1
                err = np.linalg.norm(x1 - xo)
                assert err <= step_bound(sys_, dtype, o, xs[sid], lam), (sid, k, err)
                xs[sid] = x1


def test_batch_alone_equals_in_mix(P):
    """Per-item partials make a system's result independent of the batch it
    shares: the same bits alone and among other systems (FP32 storage, with a
    drift schedule and a translation update)."""
    target = W.gaussian(777, 2000, seed=5, dtype="f32")
    others = [W.gaussian(n, m, seed=n, dtype="f32") for (n, m) in [(100, 400), (2048, 3000), (400, 900)]]
    V = W.drift(777, 30, sigma=1e-3, seed=5)
    v1 = np.random.default_rng(1).normal(scale=1e-2, size=777)
    prm = P.params(lam=0.5, eps=1e-7)
    out = []
    for mix in (False, True):
        with P.Batch("f32") as B:
            if mix:
                B.add(others[0].A, others[0].b)
                B.add(others[1].A, others[1].b, x0=others[1].z + 1)
            sid = B.add(target.A, target.b, x0=target.z + 0.2)
            if mix:
                B.add(others[2].A, others[2].b)
            B.set_drift(sid, V)
            say(f"alone/mix mix={mix}")
            B.iterate(7, prm)
            B.update(sid, translate=v1)
            B.iterate(9, prm)
            x, b, q = B.query(sid, want_b=True)
            out.append((x, b, q.iters, q.sweeps))
    assert out[0][2] == out[1][2] and out[0][3] == out[1][3]
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_batch_membership_changes_between_iterations(P):
    """Systems leave and join a batch between iterations (as the server
    does): the systems that stay, and the one that joins, take the same bits
    as in batches that never held the others."""
    keep = [W.gaussian(n, m, seed=n + 1, dtype="f32") for (n, m) in [(300, 800), (1500, 3100)]]
    gone = W.gaussian(2048, 6000, seed=8, dtype="f32")
    late = W.gaussian(640, 1700, seed=6, dtype="f32")
    prm = P.params(lam=0.4, eps=1e-9)
    with P.Batch("f32") as B:
        say("membership: mixed batch")
        ids = [B.add(s.A, s.b, x0=s.z + 0.4) for s in keep]
        gid = B.add(gone.A, gone.b, x0=gone.z + 0.4)
        B.iterate(6, prm)
        B.remove(gid)
        lid = B.add(late.A, late.b, x0=late.z + 0.4)
        B.iterate(5, prm)
        mixed = [B.query(i)[0] for i in ids] + [B.query(lid)[0]]
        assert [B.query(i)[2].iters for i in ids] == [11, 11] and B.query(lid)[2].iters == 5
    with P.Batch("f32") as B:
        say("membership: reference batches")
        ids = [B.add(s.A, s.b, x0=s.z + 0.4) for s in keep]
        B.iterate(6, prm)                   # the same call boundaries as above
        B.iterate(5, prm)
        ref = [B.query(i)[0] for i in ids]
    with P.Batch("f32") as B:
        lid = B.add(late.A, late.b, x0=late.z + 0.4)
        B.iterate(5, prm)
        ref.append(B.query(lid)[0])
    for a, b in zip(mixed, ref):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_queued_equals_single_calls(P, dtype):
    """The in-sweep decision of queued iterations against one iteration per
    call: same bits for FP64 storage, within the step tolerance for FP32."""
    systems = [W.gaussian(n, m, seed=3 * n, dtype=dtype) for (n, m) in [(200, 600), (700, 1600), (1000, 2200)]]
    drifts = [W.drift(s.n, 20, sigma=2e-3, seed=i) for i, s in enumerate(systems)]
    prm = P.params(lam=0.2, eps=1e-9)
    res = []
    for chunks in ([12], [1] * 12, [5, 7]):
        with P.Batch(dtype) as B:
            ids = [B.add(s.A, s.b, x0=s.z + 0.5) for s in systems]
            for sid, V in zip(ids, drifts):
                B.set_drift(sid, V)
            for k in chunks:
                B.iterate(k, prm)
            res.append([B.query(sid, want_b=True) for sid in ids])
    for r in res[1:]:
        for (xa, ba, qa), (xb, bb, qb) in zip(res[0], r):
            assert qa.iters == qb.iters == 12
            if dtype == "f64":
                assert np.array_equal(xa, xb) and np.array_equal(ba, bb)
            else:
                assert np.linalg.norm(xa - xb) <= 1e-4 * np.linalg.norm(xa)


def test_batch_update_rows_and_translation(P):
    """Row replacement and a translation in one update, then a sweep: the
    step equals the oracle's on the updated data."""
    sys_ = W.gaussian(300, 900, seed=9, dtype="f32")
    rows, new_rows, new_b = W.replacement_rows(sys_, 30, seed=9)
    v = np.random.default_rng(2).normal(scale=0.05, size=300)
    lam = 0.3
    x0 = sys_.z + 0.3
    with P.Batch("f32") as B:
        sid = B.add(sys_.A, sys_.b, x0=x0)
        B.update(sid, rows=rows, new_rows=new_rows, new_b=new_b, translate=v)
        say("batch update")
        B.iterate(1, P.params(lam=lam, eps=1e-9))
        x1, b1, _ = B.query(sid, want_b=True)
    A2, b2 = oracle.replace_rows(sys_.A, "f32", sys_.b, rows, new_rows, new_b)
    b2 = oracle.translate(A2, "f32", b2, v)
    o = oracle.sweep(A2, "f32", b2, x0)
    xo, status = oracle.step(o.y, o.h, 0, lam, x0)
    assert status == 0
    tol = TOL["f32"]
    assert np.linalg.norm(x1 - xo) <= step_bound(W.System(A2, b2, x0, "f32", sys_.z, {}), "f32", o, x0, lam)
    scale = np.abs(W.stored_to_f64(A2, "f32")) @ np.abs(v) + np.abs(b2)
    assert np.max(np.abs(b1 - b2) / scale) <= tol


def test_batch_long_items_write_b_in_the_row_loop(P):
    """A system cut into items of about 500 rows (125 per wavefront): the
    translated b the wavefronts keep is written out inside the row loop as
    well as after it.  Each step and the translated b follow the oracle."""
    sys_ = W.gaussian(100, 8000, seed=13, dtype="f32")
    V = W.drift(100, 10, sigma=1e-3, seed=13)
    lam = 0.3
    prm = P.params(lam=lam, eps=1e-9)
    x = sys_.z + 0.3
    b = sys_.b.copy()
    with P.Batch("f32") as B:
        sid = B.add(sys_.A, sys_.b, x0=x)
        B.set_drift(sid, V)
        for k in range(3):
            say(f"batch long items k={k}")
            B.iterate(1, prm)
            x1, b1, q = B.query(sid, want_b=True)
            o = oracle.sweep(sys_.A, "f32", b, x)
            xo, status = oracle.step(o.y, o.h, 0, lam, x)
            assert status == 0 and q.iters == k + 1
            assert np.linalg.norm(x1 - xo) <= step_bound(sys_, "f32", o, x, lam), k
            b = oracle.translate(sys_.A, "f32", b, V[k])
            scale = np.abs(W.stored_to_f64(sys_.A, "f32")) @ np.abs(V[:k + 1]).sum(axis=0) + np.abs(sys_.b)
            assert np.max(np.abs(b1 - b) / scale) <= TOL["f32"], k
            x = x1


# short rows (at most 64 VEC elements): 1, 2 and 4 chunks per lane of the
# 16-lanes-per-row form, ragged row counts, items long enough that the
# translated b is written inside the row loop
SHORT = [("f32", 20, 777), ("f32", 200, 3001), ("bf16", 500, 2501), ("bf16", 130, 901), ("f64", 50, 1999),
         ("f64", 100, 2999)]


@pytest.mark.parametrize("form", ["short", "wavefront"])
@pytest.mark.parametrize("dtype,n,m", SHORT)
def test_batch_short_rows_follow_oracle(P, monkeypatch, dtype, n, m, form):
    """Short rows swept four to a wavefront (16 lanes each) and, for
    comparison, one to a wavefront: three steps with a drift schedule, each
    step and the translated b against the oracle."""
    monkeypatch.setenv("MODAP_BATCH_SHORT", "1" if form == "short" else "0")
    sys_ = W.gaussian(n, m, seed=n * 7 + m, dtype=dtype)
    V = W.drift(n, 10, sigma=1e-3, seed=n)
    lam = 0.3
    prm = P.params(lam=lam, eps=1e-9)
    x = sys_.z + 0.3
    b = sys_.b.copy()
    with P.Batch(dtype) as B:
        B.set_tile(item_kib=[256, 2048, 4096, 8192])   # items of 260-3300 rows
        sid = B.add(sys_.A, sys_.b, x0=x)
        B.set_drift(sid, V)
        for k in range(3):
            say(f"batch short rows {dtype} n={n} m={m} form={form} k={k}")
            B.iterate(1, prm)
            x1, b1, q = B.query(sid, want_b=True)
            o = oracle.sweep(sys_.A, dtype, b, x)
            xo, status = oracle.step(o.y, o.h, 0, lam, x)
            assert status == 0 and q.iters == k + 1
            assert np.linalg.norm(x1 - xo) <= step_bound(sys_, dtype, o, x, lam), k
            b = oracle.translate(sys_.A, dtype, b, V[k])
            scale = np.abs(W.stored_to_f64(sys_.A, dtype)) @ np.abs(V[:k + 1]).sum(axis=0) + np.abs(sys_.b)
            assert np.max(np.abs(b1 - b) / scale) <= TOL[dtype], k
            x = x1


# the degenerate sizes: one column, one row, one of each, beside a system
# that spans several items
TINY = [(1, 1), (1, 6), (3, 1), (7, 2), (40, 900)]


@pytest.mark.parametrize("form", ["short", "wavefront"])
@pytest.mark.parametrize("dtype", ["f32", "bf16", "f64"])
def test_batch_tiny_systems_follow_oracle(P, monkeypatch, dtype, form):
    """Systems of one row and of one column in one batch: three steps each
    against the oracle, a system that the oracle finds feasible stopping in
    place."""
    monkeypatch.setenv("MODAP_BATCH_SHORT", "1" if form == "short" else "0")
    systems = [W.gaussian(n, m, seed=n * 11 + m, dtype=dtype) for (n, m) in TINY]
    lam = 0.4
    prm = P.params(lam=lam, eps=1e-12)
    xs = [s_.z + np.random.default_rng(i).normal(scale=1.0, size=s_.n) for i, s_ in enumerate(systems)]
    stopped = [False] * len(systems)
    with P.Batch(dtype) as B:
        ids = [B.add(s_.A, s_.b, x0=x) for s_, x in zip(systems, xs)]
        for k in range(3):
            say(f"batch tiny {dtype} form={form} k={k}")
            B.iterate(1, prm)
            for i, (s_, sid) in enumerate(zip(systems, ids)):
                x1, _, q = B.query(sid)
                if stopped[i]:
                    assert np.array_equal(x1, xs[i])
                    continue
                o = oracle.sweep(s_.A, dtype, s_.b, xs[i])
                xo, status = oracle.step(o.y, o.h, 0, lam, xs[i])
                if status != 0:
                    assert q.converged == 1 and np.array_equal(x1, xs[i]), (i, k)
                    stopped[i] = True
                    continue
                assert q.iters == k + 1, (i, k)
                assert np.linalg.norm(x1 - xo) <= step_bound(s_, dtype, o, xs[i], lam), (i, k)
                xs[i] = x1


def test_batch_solve_reaches_feasibility(P):
    """Systems of several sizes solved together, each stopping on its own:
    box-plus-sum systems (a ball of radius 100 inside, so ModAP with lambda = 1
    terminates) and a Gaussian system that starts feasible (no step).  Each
    final x is eps-feasible for its own data, checked by the oracle, and the
    step counts equal those of the same systems solved one at a time."""
    systems = [W.box_sum(n, seed=n, dtype="f32") for n in (64, 100, 256, 300, 512)]
    g = W.gaussian(700, 1500, seed=3, dtype="f32")
    systems.append(W.System(g.A, g.b, g.z.copy(), "f32", g.z, {}))
    eps = 1e-6
    prm = P.params(lam=1.0, eps=eps, max_iters=40000)
    with P.Batch("f32") as B:
        ids = [B.add(s.A, s.b, x0=s.x0) for s in systems]
        say("batch solve")
        st = B.solve(prm)
        assert st.running == 0
        steps = []
        for sid, sys_ in zip(ids, systems):
            x, b, q = B.query(sid, want_b=True)
            assert q.state == 1, (sid, q.as_dict())
            steps.append(q.iters)
            o = oracle.sweep(sys_.A, "f32", b, x)
            assert q.certified == 1
            assert o.dmax <= eps * o.binf * (1 + 1e-12)
    assert steps[-1] == 0 and len(set(steps[:-1])) > 1
    for sys_, k in zip(systems[:2], steps[:2]):
        with P.Batch("f32") as B1:
            sid = B1.add(sys_.A, sys_.b, x0=sys_.x0)
            B1.solve(prm)
            assert B1.query(sid)[2].iters == k


def test_batch_autotune_keeps_results(P):
    """The autotuner only changes speed: a tuned batch gives the oracle's step."""
    systems = [W.gaussian(n, m, seed=n, dtype="f32") for (n, m) in [(128, 800), (900, 3000), (2000, 2500)]]
    lam = 0.4
    with P.Batch("f32") as B:
        ids = [B.add(s.A, s.b, x0=s.z + 0.3) for s in systems]
        say("batch autotune")
        best = B.autotune(2)
        assert best["grid"] >= 0 and all(k >= 32 for k in best["item_kib"]) and 0 <= best["min_items"] <= 16
        assert B.get_tile() == best
        B.iterate(1, P.params(lam=lam, eps=1e-9))
        for sid, sys_ in zip(ids, systems):
            x1, _, _ = B.query(sid)
            o = oracle.sweep(sys_.A, "f32", sys_.b, sys_.z + 0.3)
            xo, _ = oracle.step(o.y, o.h, 0, lam, sys_.z + 0.3)
            assert np.linalg.norm(x1 - xo) <= step_bound(sys_, "f32", o, sys_.z + 0.3, lam)


@pytest.mark.timeout(900)
def test_full_size_batch_c4(P):
    """The benchmark's 512-system FP32 family (15.8 GB; n ~ U{64..2048},
    m ~ U{2n..8n}, generated on the device as the benchmark does), one
    iteration in one launch with the autotuned tile.  The largest and the
    smallest system and two others are checked against the oracle's step
    from x0 = 0; every system has taken its step."""
    import torch
    shapes = W.batch_shapes(512, seed=0)
    sizes = [n * m for n, m in shapes]
    pick = sorted({int(np.argmax(sizes)), int(np.argmin(sizes)), 7, 300})
    lam = 0.3
    prm = P.params(lam=lam, eps=1e-9)
    keep = {}
    with P.Batch("f32") as B:
        ids = []
        for i, (n, m) in enumerate(shapes):
            A, b, z = W.gaussian_device(n, m, seed=i, dtype="f32")
            ids.append(B.add(A, b))
            if i in pick:
                keep[i] = (A.cpu().numpy(), b.cpu().numpy(), z.cpu().numpy())
            del A, b, z
        torch.cuda.synchronize()
        say("c4 full-size batch: autotune and one iteration")
        B.autotune(1)
        st = B.iterate(1, prm)
        assert st.running == 512
        for i in pick:
            A, b, z = keep[i]
            n = A.shape[1]
            x1, _, q = B.query(ids[i])
            assert q.iters == 1
            x0 = np.zeros(n)
            o = oracle.sweep(A, "f32", b, x0)
            xo, status = oracle.step(o.y, o.h, 0, lam, x0)
            assert status == 0 and o.h > 0
            sys_ = W.System(A, b, x0, "f32", z, {})
            assert np.linalg.norm(x1 - xo) <= step_bound(sys_, "f32", o, x0, lam), (i, shapes[i])
        for sid in ids:
            assert B.query(sid, want_x=False)[2].iters == 1


@pytest.mark.parametrize("min_items", [1, 2, 16])
def test_batch_items_per_system_follow_oracle(P, min_items):
    """The cut of each system into work items (whole systems as one item, two,
    or sixteen of at least 32 KiB) changes only the order in which item
    partials are added: two steps of every system against the oracle, and a
    system's bits the same alone and in the mix at each cut."""
    shapes = [(256, 2048), (100, 301), (1000, 2500), (40, 64)]
    systems = [W.gaussian(n, m, seed=n + 3 * m, dtype="f32") for (n, m) in shapes]
    lam = 0.3
    prm = P.params(lam=lam, eps=1e-9)
    xs = [s_.z + 0.3 for s_ in systems]
    with P.Batch("f32") as B:
        B.set_tile(item_kib=[16384] * 4, min_items=min_items)
        assert B.get_tile()["min_items"] == min_items
        ids = [B.add(s_.A, s_.b, x0=x) for s_, x in zip(systems, xs)]
        for k in range(2):
            say(f"batch min_items={min_items} k={k}")
            B.iterate(1, prm)
            for i, (s_, sid) in enumerate(zip(systems, ids)):
                x1, _, q = B.query(sid)
                o = oracle.sweep(s_.A, "f32", s_.b, xs[i])
                xo, status = oracle.step(o.y, o.h, 0, lam, xs[i])
                assert status == 0 and q.iters == k + 1
                assert np.linalg.norm(x1 - xo) <= step_bound(s_, "f32", o, xs[i], lam), (i, k)
                xs[i] = x1
    with P.Batch("f32") as B:
        B.set_tile(item_kib=[16384] * 4, min_items=min_items)
        sid = B.add(systems[2].A, systems[2].b, x0=systems[2].z + 0.3)
        B.iterate(1, prm)                   # the same call boundaries as above
        B.iterate(1, prm)
        alone = B.query(sid)[0]
    assert np.array_equal(alone, xs[2])


def test_batch_errors(P):
    with P.Batch("f32") as B:
        with pytest.raises(P.ModapError, match="E_STATE"):
            B.iterate(1)
        B.set_tile(item_kib=[256, 1024, 2048, 4096], grid=0, min_items=4)
        with pytest.raises(P.ModapError, match="E_STATE"):  # nothing to tune on; the tile stays
            B.autotune(1)
        assert B.get_tile() == {"item_kib": [256, 1024, 2048, 4096], "grid": 0, "min_items": 4}
        sys_ = W.gaussian(3000, 10, seed=1, dtype="f32")
        with pytest.raises(P.ModapError, match="E_INVAL"):
            B.add(sys_.A, sys_.b)                       # rows longer than the batched sweep covers
        for shape in ((0, 4), (4, 0)):                     # empty systems
            with pytest.raises(P.ModapError, match="E_INVAL"):
                B.add(np.zeros(shape, dtype=np.float32), np.zeros(shape[0]))
        small = W.gaussian(50, 80, seed=2, dtype="f32")
        sid = B.add(small.A, small.b)
        with pytest.raises(P.ModapError, match="E_INVAL"):
            B.query(sid + 5)
        B.remove(sid)
        with pytest.raises(P.ModapError, match="E_INVAL"):
            B.remove(sid)
        for bad in (-1, 65):                               # items per system out of range
            with pytest.raises(P.ModapError, match="E_INVAL"):
                B.set_tile(item_kib=[512, 2048, 4096, 8192], min_items=bad)
