"""GPU tests of the continuous-batching solve server.

A request's result must not depend on the requests served with it: the same
bits alone and in a mix, on both the batched path (short rows) and the path
with a context of its own (long rows); admission must keep the device
footprint within the budget; every finished request is eps-feasible for its
own final data, checked by the CPU oracle."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))

import oracle
import workloads as W
from parity import TOL

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


def run_until_done(S, tickets, max_rounds=20000):
    for _ in range(max_rounds):
        if S.round() == 0:
            break
    return [S.info(t) for t in tickets]


def final_b(sys_, V, steps):
    b = sys_.b.copy()
    for k in range(steps):
        b = oracle.translate(sys_.A, sys_.dtype, b, V[k])
    return b


@pytest.mark.parametrize("dtype", ["bf16", "f64"])
def test_server_result_same_alone_and_in_mix(P, dtype):
    """Two requests (one batched, one with a context of its own because its
    rows exceed the batched sweep) with drift schedules, served alone and
    then among other requests arriving in between: identical x and step
    counts."""
    short = W.gaussian(600, 2400, seed=11, dtype=dtype)
    long = W.gaussian(5000, 6000, seed=12, dtype=dtype)
    fillers = [W.gaussian(n, 4 * n, seed=n, dtype=dtype) for n in (128, 300, 4200, 900)]
    Vs = W.drift(600, 400, sigma=1e-5, seed=11)
    Vl = W.drift(5000, 400, sigma=1e-5, seed=12)
    prm = P.params(lam=0.1, eps=1e-6, max_iters=5000)
    out = {}
    for mix in (False, True):
        with P.Server(dtype, budget_bytes=40e9, prm=prm, iters_per_round=8) as S:
            tickets = []
            if mix:
                tickets.append(S.submit(fillers[0].A, fillers[0].b))
                tickets.append(S.submit(fillers[2].A, fillers[2].b))
            ts = S.submit(short.A, short.b, V=Vs)
            if mix:
                S.round()
                tickets.append(S.submit(fillers[1].A, fillers[1].b))
            tl = S.submit(long.A, long.b, V=Vl)
            if mix:
                tickets.append(S.submit(fillers[3].A, fillers[3].b))
            say(f"server dtype={dtype} mix={mix}")
            infos = run_until_done(S, tickets + [ts, tl])
            assert all(i["state"] == 2 and i["status"] == 1 for i in infos), infos
            i_s, i_l = S.info(ts), S.info(tl)
            assert i_s["batched"] == 1 and i_l["batched"] == 0
            out[mix] = (S.result(ts), S.result(tl), i_s["iters"], i_l["iters"])
    assert out[False][2] == out[True][2] and out[False][3] == out[True][3]
    assert np.array_equal(out[False][0], out[True][0]) and np.array_equal(out[False][1], out[True][1])
    # and each result is eps-feasible for its own final (translated) data
    for sys_, V, x, it in ((short, Vs, out[True][0], out[True][2]), (long, Vl, out[True][1], out[True][3])):
        o = oracle.sweep(sys_.A, dtype, final_b(sys_, V, it), x)
        assert o.dmax <= 1e-6 * o.binf * (1 + 1e-12)


def test_server_long_requests_one_at_a_time(P):
    """max_long = 1: a second request with long rows waits in the queue while
    the first is live, a short one submitted after it is admitted past it,
    and the waiting request's result is the same bits as served alone."""
    dtype = "f32"
    long1 = W.gaussian(2500, 5000, seed=21, dtype=dtype)
    long2 = W.gaussian(2600, 5200, seed=22, dtype=dtype)
    short = W.gaussian(300, 1200, seed=23, dtype=dtype)
    prm = P.params(lam=0.1, eps=1e-6, max_iters=5000)
    with P.Server(dtype, budget_bytes=40e9, prm=prm, iters_per_round=8) as S:
        S.set_max_long(1)
        t1 = S.submit(long1.A, long1.b)
        t2 = S.submit(long2.A, long2.b)
        ts = S.submit(short.A, short.b)
        say("server max_long=1")
        S.round(now=1.0)
        assert S.info(t1)["state"] == 1 and S.info(ts)["state"] == 1
        assert S.info(t2)["state"] == 0, "the second long request waits"
        for k in range(2, 20000):   # the round index is the clock
            left = S.round(now=float(k))
            if S.info(t1)["state"] != 2:
                assert S.info(t2)["state"] == 0
            if left == 0:
                break
        infos = [S.info(t) for t in (t1, t2, ts)]
        assert all(i["state"] == 2 and i["status"] == 1 for i in infos), infos
        assert infos[1]["t_admit"] >= infos[0]["t_done"]
        x2, it2 = S.result(t2), infos[1]["iters"]
    with P.Server(dtype, budget_bytes=40e9, prm=prm, iters_per_round=8) as S:
        t2 = S.submit(long2.A, long2.b)
        run_until_done(S, [t2])
        assert S.info(t2)["iters"] == it2 and np.array_equal(S.result(t2), x2)


def test_server_admission_respects_budget(P):
    """A budget that holds about one request: the requests are served one
    after the other, memory in use never exceeds the budget, and all finish."""
    systems = [W.gaussian(n, 4 * n, seed=n, dtype="bf16") for n in (1500, 1600, 1700)]
    prm = P.params(lam=0.1, eps=1e-6, max_iters=5000)
    budget = 1.5 * 1700 * 4 * 1700 * 2     # a little more than the largest A
    with P.Server("bf16", budget_bytes=budget, prm=prm, iters_per_round=16) as S:
        tickets = [S.submit(s.A, s.b, now=0.0) for s in systems]
        say("server budget")
        now = 0.0
        for _ in range(20000):
            now += 1.0
            left = S.round(now)
            assert S.totals()["memory_in_use"] <= budget
            live = [t for t in tickets if S.info(t)["state"] == 1]
            assert len(live) <= 1
            if left == 0:
                break
        infos = [S.info(t) for t in tickets]
    assert all(i["state"] == 2 and i["status"] == 1 for i in infos)
    for a, b in zip(infos, infos[1:]):
        assert b["t_admit"] >= a["t_done"]


def test_server_updates_and_feasibility(P):
    """Requests that receive a translation and row replacements between
    rounds: each finishes eps-feasible for its final data."""
    systems = [W.gaussian(n, 4 * n, seed=50 + n, dtype="bf16") for n in (200, 700, 4500)]
    prm = P.params(lam=0.1, eps=1e-6, max_iters=5000)
    rng = np.random.default_rng(5)
    with P.Server("bf16", budget_bytes=40e9, prm=prm, iters_per_round=8) as S:
        tickets = [S.submit(s.A, s.b) for s in systems]
        data = {t: (s.A.copy(), s.b.copy(), s) for t, s in zip(tickets, systems)}
        say("server updates")
        for r in range(2000):
            left = S.round()
            if left == 0:
                break
            if r % 3 == 0:
                for t in tickets:
                    if S.info(t)["state"] != 1:
                        continue
                    A, b, s = data[t]
                    v = rng.normal(scale=1e-5, size=s.n)
                    sub = W.System(A, b, s.x0, "bf16", s.z, {})
                    idx, rows, nb = W.replacement_rows(sub, max(1, s.m // 100), seed=r)
                    S.update(t, rows=idx, new_rows=rows, new_b=nb, translate=v)
                    A2, b2 = oracle.replace_rows(A, "bf16", b, idx, rows, nb)
                    data[t] = (A2, oracle.translate(A2, "bf16", b2, v), s)
        infos = [S.info(t) for t in tickets]
        xs = [S.result(t) for t in tickets]
    assert all(i["state"] == 2 and i["status"] == 1 for i in infos), infos
    for t, x in zip(tickets, xs):
        A, b, _ = data[t]
        o = oracle.sweep(A, "bf16", b, x)
        assert o.dmax <= 1e-6 * o.binf * (1 + 1e-12)


def test_server_update_inputs_may_be_reused_at_once(P):
    """Device-side update inputs are copied before modap_server_update
    returns: overwriting them right after the call (with NaN and zeros) does
    not reach the requests, which finish eps-feasible for the data the update
    described, on both the batched path and a context of its own."""
    import torch
    dev = torch.device("cuda:0")
    systems = [W.gaussian(n, 4 * n, seed=70 + n, dtype="bf16") for n in (400, 4500)]
    prm = P.params(lam=0.1, eps=1e-6, max_iters=5000)
    with P.Server("bf16", budget_bytes=40e9, prm=prm, iters_per_round=8) as S:
        tickets = [S.submit(s.A, s.b) for s in systems]
        S.round()
        say("server update inputs")
        data = {}
        for t, s in zip(tickets, systems):
            assert S.info(t)["state"] == 1
            idx, rows, nb = W.replacement_rows(s, max(1, s.m // 100), seed=t)
            v = np.random.default_rng(t).normal(scale=1e-5, size=s.n)
            d = [torch.from_numpy(a).to(dev) for a in (idx, rows.view(np.int16), nb, v)]
            S.update(t, rows=d[0], new_rows=d[1], new_b=d[2], translate=d[3])
            d[1].zero_()
            d[2].fill_(float("nan"))
            d[3].fill_(float("nan"))
            torch.cuda.synchronize()
            A2, b2 = oracle.replace_rows(s.A, "bf16", s.b, idx, rows, nb)
            data[t] = (A2, oracle.translate(A2, "bf16", b2, v))
        infos = run_until_done(S, tickets)
        xs = [S.result(t) for t in tickets]
    assert all(i["state"] == 2 and i["status"] == 1 for i in infos), infos
    for t, x in zip(tickets, xs):
        A, b = data[t]
        o = oracle.sweep(A, "bf16", b, x)
        assert o.dmax <= 1e-6 * o.binf * (1 + 1e-12)


def test_server_errors(P):
    prm = P.params(lam=0.1, eps=1e-6, max_iters=100)
    with P.Server("bf16", budget_bytes=1e6, prm=prm) as S:
        big = W.gaussian(600, 2000, seed=1, dtype="bf16")
        with pytest.raises(P.ModapError, match="E_NOMEM"):
            S.submit(big.A, big.b)              # alone exceeds the budget
        with pytest.raises(P.ModapError, match="E_INVAL"):
            S.info(3)
        small = W.gaussian(30, 60, seed=2, dtype="bf16")
        t = S.submit(small.A, small.b)
        with pytest.raises(P.ModapError, match="E_STATE"):
            S.update(t, translate=np.zeros(30))   # not admitted yet
        with pytest.raises(P.ModapError, match="E_STATE"):
            S.result(t)
        with pytest.raises(P.ModapError, match="E_STATE"):
            S.release(t)                          # queued: nothing to release
        with pytest.raises(P.ModapError, match="E_INVAL"):
            S.release(t + 7)


def test_server_release_frees_a_result_and_keeps_its_info(P):
    """A finished request's result is read, then released: reading it again
    is refused, its statistics stay, releasing twice is a no-op, and the
    requests after it are served as before."""
    prm = P.params(lam=0.2, eps=1e-6, max_iters=5000)
    systems = [W.gaussian(n, 3 * n, seed=n, dtype="bf16") for n in (40, 90, 150)]
    with P.Server("bf16", budget_bytes=1e9, prm=prm, iters_per_round=32) as S:
        tickets = [S.submit(s_.A, s_.b, x0=s_.z + 0.5) for s_ in systems]
        for k in range(400):
            say(f"server release round {k}")
            if S.round(float(k)) == 0:
                break
        infos = [S.info(t) for t in tickets]
        assert all(i["state_name"] == "done" for i in infos)
        x0 = S.result(tickets[0])
        S.release(tickets[0])
        S.release(tickets[0])
        with pytest.raises(P.ModapError, match="E_STATE"):
            S.result(tickets[0])
        assert S.info(tickets[0]) == infos[0]
        for t, s_ in zip(tickets[1:], systems[1:]):
            x = S.result(t)
            assert x.shape == (s_.n,) and np.all(np.isfinite(x))
        assert x0.shape == (systems[0].n,)
