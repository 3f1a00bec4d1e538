#!/usr/bin/env python3
"""Benchmark of the pseudo-projection sweep on one MI355X.

Workload (one "step" = one full iteration of the method on one GPU: the fused
sweep over A -- residuals, violated-row mask, positive-slice sum y, eps test,
and the translation of the system by that iteration's drift vector, b <- b + A v
-- then the fixed-order reduction of y and the ModAP step x <- x - lambda
y/||y||):

  default: the BF16-stored Gaussian system n = 16384, m = 65536 (2 GiB of A):
  rows a_i ~ N(0,1) normalised in FP64 and rounded to BF16, hidden point
  z ~ U(-1,1)^n, b = A z + U(0,1) from the stored rows in FP64, generated on the
  device with a seeded generator; drift |v| = 1e-4 per iteration; lambda = 1;
  eps = 1e-6 * ||b||_inf.  FP32 accumulation, FP64 norms, stop test and step.
  The same line carries the FP32 system n = 8192, m = 16384 (drift N(0,1e-2^2)
  per coordinate per iteration) as a second object, `fp32_n8192_m16384`.
  --workload f32-8192x16384 / f64-4096x32768: one of those systems alone.

The timed loop runs in tracking mode (an eps-feasible check takes no step but
the system keeps moving), so every timed step reads all of A.  The sweep runs
in the library's built-in launch shape unless --autotune or --tile is given.

Printed JSON line: `value` is the whole-job algorithmic HBM throughput of the
timed steps, m*n*sizeof(A) + 24*m bytes per step (A, b read and written,
||a_i||^2), divided by wall time, inputs resident in HBM; `roofline` is the
same byte count over the sweep kernel's average duration (HIP events recorded
by the dispatches of every timed iteration when --steps <= 50, else of every
tenth, on the library's stream).  Time-to-feasible p50/p99 (every stop
certified by the library's FP64 certificate) comes from solves of the FP64
box-plus-sum system (n=256, m=513, 20 seeds), of the FP32 system from x0 = 0
under 10 drift sequences (at most 3000 iterations each; a chase not ended by
then counts as slower than every ended one), and of the BF16 system and of
the FP64 system its rows were rounded from, side by side, under the same 3
drift sequences of norm 1e-4 per iteration.  `cpu_baseline` times the CPU
oracle on a bounded number of iterations of the same system on one core, and
`cpu_baseline_all_cores` the same oracle run by one thread per available core
(at most 16) at once.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DRIFT_SEEDS = 10        # drift sequences of the time-to-feasible chase on the default system
DRIFT_STEPS = 3000      # iterations allowed per chase
DRIFT_SPEEDS = (1e-5, 1e-4, 1e-3)   # drift norms |v| per iteration swept on the BF16 system
SPEED_STEPS = 8000      # iterations allowed per chase of the BF16 system and of its FP64 original
SPEED_SEEDS = 3         # drift sequences per speed
SPEED_LAMBDA = 0.1      # ModAP step length of those chases
BATCH_TTF_STEPS = 4000  # iterations allowed per system in the chase of the batched family
METRIC = "pseudo-projection sweep HBM GB/s (% of peak); p50/p99 time-to-feasible"
KERNEL_SOURCES = ["paper_2003_09956_amd/csrc/sweep_wide.hpp", "paper_2003_09956_amd/csrc/modap_device.hpp",
                  "paper_2003_09956_amd/csrc/sweep_inst.inc"]
# The systems a step can run on: storage, n, m, drift sigma, description.
WORKLOADS = {
    "f32-8192x16384": ("f32", 8192, 16384, 1e-2,
                       "FP32 non-stationary Gaussian system n=8192 m=16384, drift N(0,1e-2^2) per coordinate "
                       "per iteration, lambda=1, eps=1e-6*||b||inf, ModAP fixed-length step"),
    "bf16-16384x65536": ("bf16", 16384, 65536, 1e-4 / 128,
                         "BF16-stored Gaussian system n=16384 m=65536 (FP32 accumulation, FP64 scalars), "
                         "drift |v|=1e-4 per iteration, lambda=1, eps=1e-6*||b||inf, ModAP fixed-length step"),
    "f64-4096x32768": ("f64", 4096, 32768, 1e-4 / 64,
                       "FP64-stored Gaussian system n=4096 m=32768 (1 GiB, FP64 throughout), drift |v|=1e-4 per "
                       "iteration, lambda=1, eps=1e-6*||b||inf, ModAP fixed-length step"),
}
ELEM_BYTES = {"f64": 8, "f32": 4, "bf16": 2}
# Workloads of many systems: the batched family (512 FP32 systems, n ~ U{64..2048},
# m ~ U{2n..8n}) and the served family (Poisson arrivals, n log-uniform in
# [128, 16384], m = 4n, BF16).
MULTI = {
    "batch-f32-512": "512 FP32 Gaussian systems (n ~ U{64..2048}, m ~ U{2n..8n}), each with its own drift "
                     "N(0,1e-3^2) per coordinate per iteration, advanced together (one persistent sweep launch "
                     "per iteration), lambda=1, eps=1e-6*||b||inf, autotuned tiles",
    "batch-f32-512-n256": "512 FP32 Gaussian systems of n=256, m=2048 (1 KiB rows), each with its own drift "
                          "N(0,1e-3^2) per coordinate per iteration, advanced together (one persistent sweep "
                          "launch per iteration), lambda=1, eps=1e-6*||b||inf, autotuned tiles",
    "catchup-box": "box-plus-sum system (FP64, dense, m=2n+1) translated along (1,...,1) at r units per "
                   "coordinate per wall-clock second; the highest r at which ModAP (lambda=1) still reaches "
                   "eps-feasibility (distance 1e-6) from x0=0 one unit outside (the translation experiment of "
                   "section 5)",
    "serve-bf16-poisson": "Poisson arrivals of BF16 Gaussian systems (n log-uniform in [128,16384], m=4n), every "
                          "10 ms of wall clock each live system translated (random walk, |v|=1e-4 per tick) and 1% "
                          "of its rows replaced (ticks elapsed during a round applied together after it), "
                          "admission by HBM footprint, ModAP lambda=0.1, eps=1e-6*||b||inf; the same arrivals and "
                          "updates also served one request at a time, in BF16 and in FP64, for comparison",
}
DT_CODE = {"f64": 0, "f32": 1, "bf16": 2}


def _code_only(path: str) -> bytes:
    """A C++ source without its comments and with whitespace collapsed, so that
    the hash below changes with the code and not with its commentary."""
    import re
    with open(os.path.join(ROOT, path)) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split()).encode()


def kernel_source_hash(dt: str = "f32") -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES + [f"paper_2003_09956_amd/csrc/sweep_{dt}.hip"]:
        h.update(_code_only(p))
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=float), q)) if xs else None


def tile_str(tile) -> str:
    return (f"{tile['block']},{tile['lanes_per_row']},{tile['chunks']},{tile['rows_per_step']},"
            f"{tile['depth']},{tile['interleave']},{tile['grid']}")


def counters_path(dt: str, n: int, m: int, tile: str) -> str:
    """Committed rocprofv3 counter summary of the sweep at one tile
    (block,lanes_per_row,chunks,rows_per_step,depth,interleave,grid)."""
    return os.path.join(ROOT, "profiles", f"sweep_wide_{dt}_n{n}_m{m}_tile{tile.replace(',', '-')}_counters.txt")


# what fixes the batched sweep's traffic: its kernel sources and the host rules that cut systems into items
BATCH_SOURCES = ["paper_2003_09956_amd/csrc/batch_kernels.hpp", "paper_2003_09956_amd/csrc/batch_plan.hpp",
                 "paper_2003_09956_amd/csrc/modap_device.hpp", "paper_2003_09956_amd/csrc/sweep_wide.hpp"]


def batch_source_hash() -> str:
    h = hashlib.sha256()
    for p in BATCH_SOURCES:
        h.update(_code_only(p))
    return h.hexdigest()[:16]


def batch_tile_str(tile) -> str:
    """k1,k2,k3,k4,grid, then ,min_items when it is not the library's choice (0)."""
    s = ",".join(str(k) for k in tile["item_kib"]) + f",{tile['grid']}"
    return s + (f",{tile['min_items']}" if tile.get("min_items", 0) else "")


BATCH_FAMILY_FILES = {"batch-f32-512": "sweep_batch_f32_512sys", "batch-f32-512-n256": "sweep_batch_f32_512x256"}


def batch_counters_path(tile: str, workload: str = "batch-f32-512") -> str:
    """Committed rocprofv3 counter summary of the batched sweep of one
    512-system FP32 family at one tile (item_kib for the four buckets, grid)."""
    return os.path.join(ROOT, "profiles", f"{BATCH_FAMILY_FILES[workload]}_tile{tile.replace(',', '-')}_counters.txt")


def measured_batch_traffic(tile, workload="batch-f32-512"):
    """HBM bytes per batched sweep launch from the committed counter summary
    taken on the current batch kernel source at this tile; else None."""
    want = batch_tile_str(tile)
    try:
        with open(batch_counters_path(want, workload)) as f:
            kv = dict(l.split(" = ", 1) for l in f.read().splitlines() if " = " in l and not l.startswith("#"))
    except OSError:
        return None
    if kv.get("source_hash") != batch_source_hash() or kv.get("tile") != want:
        return None
    return int(float(kv["bytes_per_launch"]))


def measured_traffic(dt, n, m, tile):
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by a plain copy of known size), if
    one was taken on the current kernel source at this shape; else None."""
    want = tile_str(tile)
    try:
        with open(counters_path(dt, n, m, want)) as f:
            kv = dict(l.split(" = ", 1) for l in f.read().splitlines() if " = " in l and not l.startswith("#"))
    except OSError:
        return None
    if kv.get("source_hash") != kernel_source_hash(dt) or kv.get("tile") != want:
        return None
    return int(float(kv["bytes_per_launch"]))


def time_to_feasible(P, W, seeds):
    """FP64 stationary box-plus-sum system: solve from x0 = 400 + U(0,100)."""
    out, iters, forms = [], [], set()
    prm = P.params(lam=1.0, eps=1e-6, max_iters=100000)
    with P.Solver(0) as s:
        for seed in seeds:
            sys_ = W.c1(seed)
            s.set_system(sys_.A, sys_.b, x0=sys_.x0, dtype="f64")
            st, code = s.solve(prm)
            if code != 0:
                raise RuntimeError(f"box-sum seed {seed}: solve status {code}")
            out.append(st.seconds * 1e3)
            iters.append(st.iters)
            forms.add("resident" if st.resident else "two-kernel")
    return out, iters, ",".join(sorted(forms))


def cpu_baseline(sys_, V, seconds_budget):
    """The CPU oracle, as it is, on the same system: iterations of translate +
    sweep + step, single thread, bounded to about `seconds_budget` seconds."""
    import oracle
    oracle.build(force=False)

    def run(k):
        t0 = time.perf_counter()
        res = oracle.solve(sys_.A, sys_.dtype, sys_.b, sys_.x0, lam=1.0, eps=1e-300, eps_relative=False,
                           rule=0, max_steps=k, V=V[:k])
        return time.perf_counter() - t0, res

    # size the sample: a call costs a fixed part (the row norms) plus one
    # part per iteration; the first call also touches A for the first time
    run(1)
    t1, _ = run(1)
    t3, _ = run(3)
    per = max((t3 - t1) / 2, 1e-4)
    fixed = max(t1 - per, 0.0)
    steps = max(1, min(len(V), round((seconds_budget - fixed) / per)))
    dt, res = run(steps)
    assert res.iters == steps
    return steps, dt


def cpu_baseline_all_cores(sys_, V, steps, threads):
    """The same oracle iterations run by `threads` threads at once, each on
    its own copy of the iterate (A shared, read only).  The oracle is one C
    call per solve, which releases the interpreter lock, so the threads run
    in parallel: the host's aggregate sweep throughput with every core busy."""
    import threading
    import oracle
    done = []

    def work():
        res = oracle.solve(sys_.A, sys_.dtype, sys_.b, sys_.x0, lam=1.0, eps=1e-300, eps_relative=False,
                           rule=0, max_steps=steps, V=V[:steps])
        done.append(res.iters)

    ts = [threading.Thread(target=work) for _ in range(threads)]
    t0 = time.perf_counter()
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    dt = time.perf_counter() - t0
    assert done == [steps] * threads
    return dt


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--device-warmup", type=float, default=0.3, metavar="SECONDS",
                    help="single systems: seconds of stateless sweeps before the warm-up iterations")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ttf", action="store_true",
                    help="skip the time-to-feasible solves (catch-up workload: the bisection over rates)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workload", choices=sorted(WORKLOADS) + sorted(MULTI), default="bf16-16384x65536",
                    help="system the timed steps run on (default: the BF16 n=16384 m=65536 system, 2 GiB)")
    ap.add_argument("--no-extra", action="store_true",
                    help="single-system workloads: skip the second line of the FP32 n=8192 m=16384 system (and, "
                         "on the default BF16 workload, the batched and served families measured after it)")
    ap.add_argument("--drift-speeds", action="store_true",
                    help="BF16 workload: chase at drift norms 1e-5, 1e-4 and 1e-3 (default: 1e-4 only)")
    ap.add_argument("--rate", type=float, default=5.0, help="serving: Poisson arrival rate per second")
    ap.add_argument("--horizon", type=float, default=10.0, help="serving: seconds of arrivals")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="serving: HBM budget of the server")
    ap.add_argument("--iters-per-round", type=int, default=64,
                    help="serving: iterations every live request takes per round of the server")
    ap.add_argument("--max-long", type=int, default=1,
                    help="serving: live requests with rows too long for the batch at most (0: no limit)")
    ap.add_argument("--n", type=int, default=32000, help="translation experiment: number of variables")
    ap.add_argument("--lam", type=float, default=1.0, help="translation experiment: ModAP step length")
    ap.add_argument("--tile", type=str, default=None,
                    help="force the sweep shape block,lanes_per_row,chunks,rows_per_step,depth,interleave,grid")
    ap.add_argument("--autotune", action="store_true",
                    help="single-system workloads: run the sweep autotuner before timing (default: the library's "
                         "built-in shape, so that a kernel trace of the same command names the same kernel)")
    ap.add_argument("--batch-tile", type=str, default=None,
                    help="batched workload: force item_kib for the four row-length buckets, the grid and "
                         "optionally the least items per system, k1,k2,k3,k4,grid[,min_items] (skips the "
                         "batch autotuner)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes five times (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              f"(the sweep runs on a single MI355X; row sharding across GPUs is not built)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2003_09956_amd as P
    import workloads as W

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.copy_calibration:
        nbytes = args.copy_calibration // 16 * 16
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "launches": 5}), flush=True)
        return
    P.lib()
    if args.workload in ("batch-f32-512", "batch-f32-512-n256"):
        return bench_batch(args, P, W, torch)
    if args.workload == "serve-bf16-poisson":
        return bench_serve(args, P, W, torch)
    if args.workload == "catchup-box":
        return bench_catchup(args, P, W, torch)

    K, WU = args.steps, args.warmup
    dt, n, m, sigma, desc = WORKLOADS[args.workload]
    lam, eps = 1.0, 1e-6
    log(f"generating the {args.workload} system ...")
    sys_ = None
    if dt == "bf16":
        # built on the device (seeded; the host copy is made only for the CPU baseline)
        A_d, b_d, _ = W.gaussian_device(n, m, seed=args.seed, dtype=dt)
        A_in, b_in = A_d, b_d
    else:
        sys_ = W.gaussian(n, m, args.seed, dt)
        A_in, b_in = sys_.A, sys_.b
    V = W.drift(n, 2 * (K + WU), sigma=sigma, seed=args.seed)
    res = timed_steps(P, torch, A_in, b_in, dt, V, K, WU, lam, eps, args)
    line = step_line(args, dt, n, m, desc, res)
    extra_fp32 = None
    if dt != "f32" and not args.no_extra:
        # the FP32 n = 8192, m = 16384 system of round numbers as a second line
        log("generating the FP32 n=8192 m=16384 system ...")
        s2 = W.gaussian(8192, 16384, args.seed, "f32")
        V2 = W.drift(8192, 2 * (K + WU), sigma=1e-2, seed=args.seed)
        res2 = timed_steps(P, torch, s2.A, s2.b, "f32", V2, K, WU, lam, eps, args)
        extra_fp32 = step_line(args, "f32", 8192, 16384, WORKLOADS["f32-8192x16384"][4], res2)
        for key in ("metric", "unit", "n_gpus", "steps", "warmup", "higher_is_better", "scaling", "vs_baseline",
                    "data"):
            extra_fp32.pop(key, None)
        line["fp32_n8192_m16384"] = extra_fp32
    if not args.no_ttf:
        ms, its, form = time_to_feasible(P, W, range(20))
        line["time_to_feasible"] = {
            "box_sum_f64_n256_m513": {"p50_ms": round(percentile(ms, 50), 3), "p99_ms": round(percentile(ms, 99), 3),
                                      "seeds": 20, "steps_p50": percentile(its, 50), "iteration_form": form},
        }
        if dt == "f32" or extra_fp32 is not None:
            s2 = sys_ if dt == "f32" else s2
            line["time_to_feasible"]["gaussian_f32_n8192_m16384_drift"] = fp32_chase(P, W, s2, args.seed)
        if dt == "bf16":
            line["time_to_feasible"]["bf16_vs_f64_n16384_m65536"] = bf16_vs_f64_chase(
                P, W, torch, n, m, args.seed, DRIFT_SPEEDS if args.drift_speeds else (1e-4,))
    if not args.no_cpu_baseline:
        if sys_ is None:
            import numpy as np
            Ah = A_d.view(torch.int16).cpu().numpy().view(np.uint16) if dt == "bf16" else A_d.cpu().numpy()
            sys_ = W.System(Ah, b_d.cpu().numpy(), np.zeros(n), dt)
        line.update(cpu_lines(args, sys_, V, res["bytes_per_step"], n, m, dt))
    if dt == "bf16" and not args.no_extra and not args.no_ttf:
        # the batched and served families, measured in the same run: their
        # lines (without the keys this line already carries) as objects of it
        import copy
        A_d = b_d = A_in = b_in = sys_ = None   # the BF16 system's device memory goes back
        torch.cuda.empty_cache()
        for wl, key, fn in (("batch-f32-512", "batch_f32_512", bench_batch),
                            ("serve-bf16-poisson", "serve_bf16_poisson", bench_serve)):
            a2 = copy.copy(args)
            a2.workload, a2.batch_tile = wl, None
            log(f"--- {wl} ---")
            try:
                sub = fn(a2, P, W, torch, emit=False)
            except Exception as e:     # the headline stands on its own: record the failure, go on
                log(f"{wl} failed: {e!r}")
                line[key] = {"error": repr(e)}
                torch.cuda.empty_cache()
                continue
            for k in ("metric", "unit", "n_gpus", "higher_is_better", "scaling", "vs_baseline"):
                sub.pop(k, None)
            line[key] = sub
            torch.cuda.empty_cache()
    print(json.dumps(line), flush=True)


def warm_device(s, torch, n, seconds):
    """Stateless sweeps of the loaded system (eval_sweep, which leaves the
    solver's state alone) until `seconds` of wall clock have passed; returns
    their number.  In a fresh process the first 15-40 ms of sustained sweeps
    run up to 15% slower than later ones, whatever the iterate's phase (the
    same trajectory restarted from x0 later in the process runs at the steady
    rate from its first step), so the device is brought to that rate before
    the warm-up iterations."""
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    k, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        s.eval_sweep(x, want_r=False, y_out=y)
        k += 1
    torch.cuda.synchronize()
    return k


def timed_steps(P, torch, A, b, dt, V, K, WU, lam, eps, args):
    """K timed steps (after WU untimed ones) of one system in tracking mode,
    then the same K steps again with HIP events on every iteration's kernel
    dispatches (the roofline's kernel durations).  The events cost 8-10 us per
    step on this stack, so the throughput is taken from the first pass, which
    carries none.  V needs 2 (K + WU) rows."""
    m, n = int(A.shape[0]), int(A.shape[1])
    with P.Solver(0) as s:
        s.set_system(A, b, dtype=dt)      # first call: allocation and warm-up
        torch.cuda.synchronize()
        u0 = time.perf_counter()
        s.set_system(A, b, dtype=dt)      # the upload (PCIe when A is a host array), then the row norms
        torch.cuda.synchronize()
        upload_s = time.perf_counter() - u0
        s.set_drift(V)
        if args.tile:
            blk, lpr, ch, rs, depth, il, grid = (int(v) for v in args.tile.split(","))
            s.set_tile(blk, lpr, ch, grid, rs, depth=depth, interleave=il)
            tile = s.get_tile()
            log("tile (forced)", tile)
        elif args.autotune:
            tile = s.autotune(5)
            log("tile (autotuned)", tile)
        else:
            tile = s.get_tile()
            log("tile (built-in)", tile)
        warm = warm_device(s, torch, n, args.device_warmup) if args.device_warmup > 0 else 0
        s.iterate(WU, P.params(lam=lam, eps=eps, track=True))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = s.iterate(K, P.params(lam=lam, eps=eps, track=True))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if st.sweeps != K + WU:
            raise RuntimeError(f"timed region ran {st.sweeps - WU} sweeps, expected {K}")
        # the profiled pass: WU untimed iterations that also create the events
        # (none is created while the device runs ahead), then K with events
        s.iterate(WU, P.params(lam=lam, eps=eps, track=True, profile=1))
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        sp = s.iterate(K, P.params(lam=lam, eps=eps, track=True, profile=1))
        torch.cuda.synchronize()
        p1 = time.perf_counter()
        if sp.profiled != K:
            raise RuntimeError(f"profiled pass timed {sp.profiled} sweeps, expected {K}")
    wall = t1 - t0
    sweep_us = sp.sweep_ms * 1e3 / sp.profiled
    reduce_us = sp.reduce_ms * 1e3 / sp.profiled
    log(f"{dt} n={n} m={m}: timed {K} steps in {wall * 1e3:.2f} ms ({(p1 - p0) * 1e3:.2f} ms with events); "
        f"sweep {sweep_us:.1f} us, reduce {reduce_us:.1f} us ({sp.profiled} profiled)")
    return {"wall": wall, "wall_profiled": p1 - p0, "sweep_us": sweep_us, "reduce_us": reduce_us,
            "profiled": int(sp.profiled), "tile": tile, "upload_s": upload_s, "warm_sweeps": warm,
            "host_bytes": int(A.nbytes if hasattr(A, "nbytes") else 0),
            "feasible_steps": int(st.sweeps - st.iters), "bytes_per_step": m * n * ELEM_BYTES[dt] + 24 * m,
            "on_host": not hasattr(A, "is_cuda")}


def step_line(args, dt, n, m, desc, res):
    K, WU = args.steps, args.warmup
    tile, wall = res["tile"], res["wall"]
    bps = res["bytes_per_step"]
    value = bps * K / wall / 1e9
    achieved = bps / (res["sweep_us"] * 1e-6) / 1e9
    kind = "sweep_split" if tile["kind"] == 1 else "sweep_wide"
    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": WU,
        "ms_per_step": round(wall * 1e3 / K, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dt,
        "data": "synthetic (seeded" + (", generated on the device)" if not res["on_host"] else ")"),
        "config": {"workload": desc, "n": n, "m": m, "storage": dt,
                   "accumulate": "f64" if dt == "f64" else "f32 dot, f64 scalars",
                   "bytes_per_step": bps, "tile": tile},
        "pct_of_peak": round(100 * value / HBM_PEAK_GBS, 2),
        "iterations_per_s": round(K / wall, 1),
        "feasible_checks_in_timed_steps": res["feasible_steps"],
        "device_warmup": {"seconds": args.device_warmup, "stateless_sweeps": res["warm_sweeps"],
                          "note": "before the warm-up iterations; the solver's state is untouched"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dt, n, m, tile) if tile["kind"] == 0 else None,
                     "kernel": f"{kind}<{DT_CODE[dt]},{tile['block']},{tile['lanes_per_row']},{tile['chunks']},"
                               f"{tile['rows_per_step']},{tile['depth']},true>",
                     "avg_us": round(res["sweep_us"], 3), "reduce_avg_us": round(res["reduce_us"], 3),
                     "profiled_sweeps": res["profiled"],
                     "profiled_pass": "the same K steps again, every kernel dispatch carrying HIP events "
                                      f"({res['wall_profiled'] * 1e3 / K:.4f} ms per step with them)"},
    }
    if res["on_host"]:
        line["host_upload"] = {"ms": round(res["upload_s"] * 1e3, 3), "bytes": res["host_bytes"],
                               "pcie_inclusive_GBs": round(bps * K / (wall + res["upload_s"]) / 1e9, 2)}
    return line


def fp32_chase(P, W, sys_, seed):
    """Time-to-feasible of the FP32 system chased from x0 = 0 under DRIFT_SEEDS
    drift sequences (whether and when a chase ends is decided by the random
    walk of the drift, so one sequence says little); every stop certified in
    FP64.  A sequence not caught within DRIFT_STEPS counts as slower than any
    caught one."""
    import numpy as np
    n = sys_.n
    runs = []
    with P.Solver(0) as s:
        for sd in range(DRIFT_SEEDS):
            s.set_system(sys_.A, sys_.b, dtype="f32")
            s.set_drift(W.drift(n, DRIFT_STEPS, sigma=1e-2, seed=seed + 1 + sd))
            st2, code = s.solve(P.params(lam=1.0, eps=1e-6, max_iters=DRIFT_STEPS), raise_on_stop=False)
            runs.append((code == 0 and st2.certified == 1, st2.seconds * 1e3, int(st2.iters), st2.b_drift,
                         st2.eps_abs))
            log("fp32 chase", sd, runs[-1])
    ms = [r[1] if r[0] else math.inf for r in runs]
    its = [r[2] if r[0] else math.inf for r in runs]
    pct = lambda v, q: float(np.percentile(np.asarray(v), q, method="higher"))
    fin = lambda v: round(v, 3) if math.isfinite(v) else None
    return {"seeds": DRIFT_SEEDS, "caught": int(sum(r[0] for r in runs)), "max_steps": DRIFT_STEPS,
            "certified": True, "p50_ms": fin(pct(ms, 50)), "p99_ms": fin(pct(ms, 99)),
            "steps_p50": fin(pct(its, 50)),
            "max_b_drift_over_eps_abs": round(max(r[3] / r[4] for r in runs if r[4] > 0), 4)}


def bf16_vs_f64_chase(P, W, torch, n, m, seed, speeds):
    """The BF16-stored system chased from x0 = 0 under drifts of norm |v| per
    iteration, and the FP64 system its rows were rounded from (same random
    numbers before rounding) chased under the same drift sequences on the
    same GPU: p50/p99 time-to-feasible of both forms, every stop certified in
    FP64; and the violation each BF16 result leaves on the FP64 system (the
    error of the storage precision in the final point).  ModAP with
    lambda = SPEED_LAMBDA, the step length that reaches eps on these systems
    in the fewest iterations."""
    import numpy as np
    dev = torch.device("cuda")
    log("generating the BF16 system and the FP64 system its rows were rounded from ...")
    A16, b16, _ = W.gaussian_device(n, m, seed=seed, dtype="bf16")
    A64, b64, _ = W.gaussian_device(n, m, seed=seed, dtype="f64")
    prm = P.params(lam=SPEED_LAMBDA, eps=1e-6, max_iters=SPEED_STEPS)
    fin = lambda v: round(v, 3) if math.isfinite(v) else None
    pct = lambda v, q: float(np.percentile(np.asarray(v), q, method="higher"))
    out = []
    with P.Solver(0) as q16, P.Solver(0) as q64:
        for k, speed in enumerate(speeds):
            runs = {"bf16": [], "f64": []}
            viol, vrows, eps_abs = 0.0, 0, 0.0
            for sd in range(SPEED_SEEDS):
                g = torch.Generator(device="cuda")
                g.manual_seed(seed * 1000 + k * 10 + sd)
                V = torch.randn((SPEED_STEPS, n), generator=g, device=dev, dtype=torch.float64)
                V *= speed / math.sqrt(n)
                for name, q, A, b in (("bf16", q16, A16, b16), ("f64", q64, A64, b64)):
                    q.set_system(A, b, dtype=name)
                    q.set_drift(V)
                    st, code = q.solve(prm, raise_on_stop=False)
                    runs[name].append((code == 0 and st.certified == 1, st.seconds * 1e3, int(st.iters),
                                       st.seconds * 1e3 / max(st.sweeps, 1)))
                    log("drift", speed, sd, name, code, runs[name][-1])
                    if name == "bf16":
                        eps_abs = max(eps_abs, st.eps_abs)
                # the BF16 result on the FP64 data as they stand at its final
                # check (the translations of the steps it took)
                x16, _, _ = q16.query()
                steps = runs["bf16"][-1][2]
                q64.set_system(A64, b64, dtype="f64")
                if steps:
                    q64.update_coeffs(translate=V[:steps].sum(dim=0).contiguous())
                ev = q64.eval_sweep(torch.from_numpy(x16).to(dev), want_r=False)
                viol, vrows = max(viol, float(ev.max_viol)), max(vrows, int(ev.h))
                del V
            row = {"v_norm": speed, "seeds": SPEED_SEEDS, "max_steps": SPEED_STEPS, "lambda": SPEED_LAMBDA,
                   "certified": True}
            for name, rr in runs.items():
                ms = [r[1] if r[0] else math.inf for r in rr]
                row[name] = {"caught": sum(r[0] for r in rr), "p50_ms": fin(pct(ms, 50)), "p99_ms": fin(pct(ms, 99)),
                             "steps": [r[2] for r in rr],
                             "ms_per_step": round(float(np.mean([r[3] for r in rr])), 4)}
            row["bf16_result_on_fp64_system"] = {"max_viol": viol, "violated_rows": vrows, "eps_abs": eps_abs}
            p16, p64 = row["bf16"]["p50_ms"], row["f64"]["p50_ms"]
            row["p50_speedup_bf16_over_f64"] = round(p64 / p16, 2) if p16 and p64 else None
            out.append(row)
    del A16, b16, A64, b64
    return out if len(out) > 1 else out[0]


def cpu_lines(args, sys_, V, bytes_per_step, n, m, dt):
    steps, secs = cpu_baseline(sys_, V, args.cpu_seconds)
    out = {"cpu_baseline": {"value": round(bytes_per_step * steps / secs / 1e9, 4), "unit": "GB/s", "cores": 1,
                            "kind": "oracle",
                            "sample": f"{steps} iterations (translate, sweep, step) of the full n={n} m={m} "
                                      f"{dt} system, {secs:.1f} s, single-threaded extended-precision oracle"}}
    # every core the process may use (at most 16, the host share of one GPU)
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    per = max(1, steps // 2)
    secs_all = cpu_baseline_all_cores(sys_, V, per, threads)
    out["cpu_baseline_all_cores"] = {
        "value": round(bytes_per_step * per * threads / secs_all / 1e9, 4), "unit": "GB/s", "cores": threads,
        "kind": "oracle",
        "sample": f"{threads} threads, each {per} iterations of the same system from its own copy of the "
                  f"iterate, {secs_all:.1f} s wall"}
    return out


def bench_batch(args, P, W, torch, emit=True):
    """One step = one iteration of all 512 systems (one sweep launch, one
    reduction launch); data generated on the device with a seeded generator."""
    K, WU = args.steps, args.warmup
    shapes = W.batch_shapes(512, seed=args.seed) if args.workload == "batch-f32-512" else [(256, 2048)] * 512
    B = P.Batch("f32")
    bytes_per_step = 0
    for i, (n, m) in enumerate(shapes):
        A, b, _ = W.gaussian_device(n, m, seed=args.seed * 100003 + i, dtype="f32")
        sid = B.add(A, b)
        g = torch.Generator(device="cuda")
        g.manual_seed(args.seed * 7 + i)
        B.set_drift(sid, torch.randn((2 * (K + WU), n), generator=g, device="cuda", dtype=torch.float64) * 1e-3)
        bytes_per_step += m * n * 4 + 24 * m
        del A, b
    torch.cuda.synchronize()
    if args.batch_tile:
        v = [int(x) for x in args.batch_tile.split(",")]
        if len(v) not in (5, 6):
            raise SystemExit("--batch-tile takes k1,k2,k3,k4,grid[,min_items]")
        B.set_tile(item_kib=v[:4], grid=v[4], min_items=v[5] if len(v) == 6 else 0)
        tile = B.get_tile()
        log("batch tile (forced)", tile)
    else:
        tile = B.autotune(5)
        log("batch tile (autotuned)", tile)
    lam, eps = 1.0, 1e-6
    # the timed pass carries no events; the same K steps again with events on
    # every iteration give the kernel durations (as in timed_steps)
    B.iterate(WU, P.params(lam=lam, eps=eps, track=True))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.iterate(K, P.params(lam=lam, eps=eps, track=True))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    B.iterate(WU, P.params(lam=lam, eps=eps, track=True, profile=1))
    torch.cuda.synchronize()
    st = B.iterate(K, P.params(lam=lam, eps=eps, track=True, profile=1))
    torch.cuda.synchronize()
    if st.profiled != K:
        raise RuntimeError(f"profiled pass timed {st.profiled} sweeps, expected {K}")
    sweep_us = st.sweep_ms * 1e3 / st.profiled
    reduce_us = st.reduce_ms * 1e3 / st.profiled
    B.close()
    del B
    value = bytes_per_step * K / wall / 1e9
    achieved = bytes_per_step / (sweep_us * 1e-6) / 1e9
    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": K, "warmup": WU,
        "ms_per_step": round(wall * 1e3 / K, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (generated on the device, seeded)",
        "config": {"workload": MULTI[args.workload], "systems": 512, "elements": int(sum(n * m for n, m in shapes)),
                   "bytes_per_step": bytes_per_step, "tile": tile},
        "pct_of_peak": round(100 * value / HBM_PEAK_GBS, 2),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_batch_traffic(tile, args.workload),
                     "kernel": "sweep_batch<1>",
                     "avg_us": round(sweep_us, 3), "reduce_avg_us": round(reduce_us, 3)},
    }
    if not args.no_ttf:
        line["time_to_feasible"] = batch_time_to_feasible(args, P, W, torch, shapes, tile)
    if emit:
        print(json.dumps(line), flush=True)
    return line


def batch_time_to_feasible(args, P, W, torch, shapes, tile):
    """All systems of the batched family chased from x0 = 0 to eps-feasibility
    under drifts of their own (N(0, 1e-3^2) per coordinate per iteration),
    ModAP with lambda = 0.1: advanced together by the batch, and -- the plain
    single-system form -- the FP64 rows they were rounded from solved one
    system at a time under the same drifts."""
    import numpy as np
    prm = P.params(lam=SPEED_LAMBDA, eps=1e-6, max_iters=BATCH_TTF_STEPS)

    def drift_of(i, n):
        g = torch.Generator(device="cuda")
        g.manual_seed(args.seed * 7919 + i)
        return torch.randn((BATCH_TTF_STEPS, n), generator=g, device="cuda", dtype=torch.float64) * 1e-3

    seed_of = lambda i: args.seed * 100003 + i
    B = P.Batch("f32")
    ids = []
    for i, (n, m) in enumerate(shapes):
        A, b, _ = W.gaussian_device(n, m, seed=seed_of(i), dtype="f32")
        ids.append(B.add(A, b))
        B.set_drift(ids[-1], drift_of(i, n))
        del A, b
    B.set_tile(item_kib=tile["item_kib"], grid=tile["grid"], min_items=tile.get("min_items", 0))
    torch.cuda.synchronize()
    bst = B.solve(prm)
    steps = [int(B.query(sid, want_x=False)[2].iters) for sid in ids]
    caught = sum(int(B.query(sid, want_x=False)[2].state == 1) for sid in ids)
    B.close()
    del B
    log(f"batch chase: {caught} of {len(ids)} caught in {bst.seconds:.2f} s")
    # the FP64 single-system form, one system after another
    done, secs, steps64 = 0, [], []
    with P.Solver(0) as s:
        for i, (n, m) in enumerate(shapes):
            A, b, _ = W.gaussian_device(n, m, seed=seed_of(i), dtype="f64")
            s.set_system(A, b, dtype="f64")
            s.set_drift(drift_of(i, n))
            st, code = s.solve(prm, raise_on_stop=False)
            done += code == 0
            secs.append(st.seconds)
            steps64.append(int(st.iters))
            del A, b
    finish = np.cumsum(secs)
    log(f"FP64 one at a time: {done} of {len(shapes)} caught in {finish[-1]:.2f} s")
    pct = lambda v, q: float(np.percentile(np.asarray(v, dtype=float), q))
    return {"systems": len(shapes), "lambda": SPEED_LAMBDA, "max_steps": BATCH_TTF_STEPS,
            "batched_f32": {"caught": caught, "all_done_s": round(bst.seconds, 3),
                            "steps_p50": pct(steps, 50), "steps_p99": pct(steps, 99)},
            "f64_one_at_a_time": {"caught": done, "all_done_s": round(float(finish[-1]), 3),
                                  "p50_done_s": round(pct(finish, 50), 3),
                                  "steps_p50": pct(steps64, 50), "steps_p99": pct(steps64, 99)},
            "speedup_all_done": round(float(finish[-1]) / bst.seconds, 2)}


def _replace_rows_device(torch, n, m, k, z, gen, dtype):
    """k fresh normalised Gaussian rows with b = a.z + U(0,1) (device tensors)."""
    idx = torch.randperm(m, generator=gen, device="cuda")[:k].sort().values
    rows = torch.randn((k, n), generator=gen, device="cuda", dtype=torch.float64)
    rows /= torch.linalg.vector_norm(rows, dim=1, keepdim=True)
    rows = rows.to({"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dtype])
    nb = rows.to(torch.float64) @ z + torch.rand(k, generator=gen, device="cuda", dtype=torch.float64)
    return idx.contiguous(), rows.contiguous(), nb.contiguous()


def catchup_trial(P, s, A, b, n, rate, lam, limit_s, chunk=4):
    """One run: the polytope starts one unit per coordinate above x0 = 0 and
    moves at `rate` per coordinate per second of wall clock (translations
    applied between chunks of iterations, each by rate * elapsed time).
    Returns (caught, seconds, iterations)."""
    import numpy as np
    import torch
    s.set_system(A, b, dtype="f64")
    # eps is an absolute distance here: ||b||_inf is dominated by the sum row
    prm = P.params(lam=lam, eps=1e-6, eps_relative=False, max_iters=10 ** 9)
    ones = torch.ones(n, device="cuda", dtype=torch.float64)
    t0 = time.perf_counter()
    last = t0
    iters = 0
    while True:
        st = s.iterate(chunk, prm)
        iters += chunk
        if st.converged:
            return True, time.perf_counter() - t0, int(st.sweeps)
        now = time.perf_counter()
        if now - t0 > limit_s:
            return False, now - t0, int(st.sweeps)
        s.update_coeffs(translate=ones * (rate * (now - last)))
        last = now


def paper_catchup_context(n):
    """The paper's highest caught translation rates at this n (section 5),
    with the hardware they were measured on: context, not a target."""
    runs = []
    with open(os.path.join(ROOT, "tests", "golden", "paper_catchup_rates.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            nn, nodes, r, total, _ = line.split()
            if int(nn) == n:
                runs.append({"nodes": int(nodes), "per_coord": int(r), "total": int(total)})
    if not runs:
        return None
    return {"hardware": "cluster nodes of 2x Intel Xeon X5680 (6 cores, 3.33 GHz), 24 GB DDR3, "
                        "InfiniBand QDR (section 5, Table 1)",
            "lambda": "not stated", "eps": 1e-7, "runs": runs}


def bench_catchup(args, P, W, torch):
    """Highest translation rate at which the iteration catches the moving
    polytope, found by bisection on measured runs."""
    import math
    n = args.n
    A, b = W.box_sum_device(n, "f64", offset=1.0)
    torch.cuda.synchronize()
    lam = args.lam
    limit = 30.0
    trials = []
    with P.Solver(0) as s:
        # iteration time with the polytope at rest, from the same start
        s.set_system(A, b, dtype="f64")
        st = s.iterate(20, P.params(lam=lam, eps=1e-6, eps_relative=False, max_iters=10 ** 9, profile=1,
                                    track=True))
        t_iter = (st.sweep_ms + st.reduce_ms) / st.profiled / 1e3
        t_sweep = st.sweep_ms / st.profiled / 1e3
        h_rest = int(st.h)
        r_est = lam / (math.sqrt(n) * t_iter)
        lo, hi = 0.0, None
        r = 0.5 * r_est
        for _ in range(0 if args.no_ttf else 7):     # --no-ttf: the iteration time only
            caught, secs, sweeps = catchup_trial(P, s, A, b, n, r, lam, limit)
            trials.append({"rate_per_coord": round(r, 4), "caught": caught, "seconds": round(secs, 3),
                           "sweeps": sweeps})
            log("catch-up trial", trials[-1])
            if caught:
                lo = r
                r = r * 1.5 if hi is None else 0.5 * (r + hi)
            else:
                hi = r
                r = 0.5 * (lo + r)
        tile = s.get_tile()
    bytes_per_iter = (2 * n + 1) * n * 8 + 24 * (2 * n + 1)
    line = {
        "metric": METRIC, "value": round(bytes_per_iter / t_iter / 1e9, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": 20, "warmup": 0, "ms_per_step": round(t_iter * 1e3, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic (generated on the device)",
        "config": {"workload": MULTI["catchup-box"], "n": n, "m": 2 * n + 1, "lambda": lam, "tile": tile,
                   "A_bytes": (2 * n + 1) * n * 8},
        "max_caught_rate": None if args.no_ttf else {
            "per_coord": round(lo, 4), "total": round(lo * math.sqrt(n), 2),
            "first_missed_per_coord": round(hi, 4) if hi is not None else None,
            "model_lambda_over_sqrt_n_t_iter": round(r_est, 4), "trials": trials},
        "paper_context": paper_catchup_context(n),
    }
    # The sweep of these long rows is the split-row form (all its kernels
    # between the same two events): algorithmic bytes are one pass over A; it
    # moves (1 + h/m) A, re-reading the violated rows.
    m = 2 * n + 1
    alg = bytes_per_iter / t_sweep / 1e9
    line["roofline"] = {"bound": "hbm", "achieved": round(alg, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(alg / HBM_PEAK_GBS, 4), "traffic": None,
                        "kernel": f"sweep_split (tile {tile['block']},{tile['lanes_per_row']},{tile['chunks']})"
                        if tile["kind"] == 1 else "sweep_wide",
                        "avg_us": round(t_sweep * 1e6, 3),
                        "moved_bytes_model": int(m * n * 8 * (1 + h_rest / m)) if tile["kind"] == 1 else None,
                        "moved_GBs": round(m * n * 8 * (1 + h_rest / m) / t_sweep / 1e9, 2)
                        if tile["kind"] == 1 else None}
    print(json.dumps(line), flush=True)


def serve_pass(args, P, W, torch, arrivals, storage, max_live, wall_cap, ipr=8, max_long=0):
    """Drive one server over the arrivals: requests generated on the device at
    their arrival time, every 10 ms each live request translated (|v| = 1e-4)
    and 1% of its rows replaced by fresh rows that keep its moving hidden point
    feasible.  Time-to-feasible runs from arrival to the end of the round that
    saw the request eps-feasible; requests not finished within wall_cap
    seconds are reported as censored."""
    import math
    lam, eps, tick, vnorm, frac = 0.1, 1e-6, 0.010, 1e-4, 0.01
    prm = P.params(lam=lam, eps=eps, max_iters=200000)
    S = P.Server(storage, budget_bytes=args.budget_gb * 1e9, prm=prm, iters_per_round=ipr)
    if max_live:
        S.set_max_live(max_live)
    if max_long:
        S.set_max_long(max_long)
    # the generators run on torch's stream; waiting for that stream alone
    # leaves the server's iterations in flight
    gen = torch.Generator(device="cuda")
    gen.manual_seed(args.seed + 17)
    reqs = {}
    active = set()      # tickets not yet finished: the only ones an update tick looks at
    i = 0
    t0 = time.perf_counter()
    next_tick = tick
    rounds = 0
    last_log = 0.0
    while True:
        now = time.perf_counter() - t0
        while i < len(arrivals) and arrivals[i][0] <= now:
            t_arr, n, m, sd = arrivals[i]
            A, b, z = W.gaussian_device(n, m, seed=sd, dtype=storage)
            torch.cuda.current_stream().synchronize()
            tk = S.submit(A, b, now=t_arr)
            reqs[tk] = {"n": n, "m": m, "z": z}
            active.add(tk)
            i += 1
        if now >= next_tick:
            # every tick that has elapsed since the last update counts: k ticks
            # are one translation by the sum of k steps (a random walk) and the
            # replacement of k times 1% of the rows, so the systems move at the
            # same rate per second however long a round takes
            k = 1 + int((now - next_tick) / tick)
            live = []
            for tk in sorted(active):
                state = S.info(tk)["state"]
                if state == 1:
                    live.append(tk)
                elif state >= 2:          # finished: its result is not needed here
                    active.discard(tk)
                    reqs[tk].pop("z", None)
                    S.release(tk)
            for tk in live:
                r = reqs[tk]
                v = torch.randn(r["n"], generator=gen, device="cuda", dtype=torch.float64) * (
                    vnorm * math.sqrt(k / r["n"]))
                r["z"] = r["z"] + v
                nrep = min(r["m"], k * max(1, math.ceil(frac * r["m"])))
                idx, rows, nb = _replace_rows_device(torch, r["n"], r["m"], nrep, r["z"], gen, storage)
                r["upd"] = (idx, rows, nb, v)
            torch.cuda.current_stream().synchronize()
            for tk in live:
                idx, rows, nb, v = reqs[tk].pop("upd")
                S.update(tk, rows=idx, new_rows=rows, new_b=nb, translate=v)
            next_tick += k * tick
        left = S.round(now)
        rounds += 1
        if now - last_log > 5.0:
            log(f"{storage} max_live={max_live}: t={now:.1f}s arrivals {i}/{len(arrivals)} outstanding {left}")
            last_log = now
        if (i == len(arrivals) and left == 0) or now > wall_cap:
            break
        if left == 0:
            # nothing queued or live: wait for the next arrival instead of
            # calling empty rounds
            time.sleep(max(0.0, arrivals[i][0] - (time.perf_counter() - t0)))
    wall = time.perf_counter() - t0
    infos = [S.info(tk) for tk in reqs]
    tot = S.totals()
    S.close()
    ttf = [inf["t_done"] - inf["t_submit"] for inf in infos if inf["state"] == 2 and inf["status"] == 1]
    done = sorted(((inf["t_done"] - inf["t_submit"], tk) for tk, inf in zip(reqs, infos)
                   if inf["state"] == 2 and inf["status"] == 1), reverse=True)
    slowest = [{"n": reqs[tk]["n"], "t_submit_s": round(infos[list(reqs).index(tk)]["t_submit"], 3),
                "ttf_ms": round(1e3 * t, 1)} for t, tk in done[:3]]
    out = {"p50_ms": round(1e3 * percentile(ttf, 50), 3) if ttf else None,
           "p99_ms": round(1e3 * percentile(ttf, 99), 3) if ttf else None,
           "feasible": len(ttf), "requests": len(reqs), "censored": sum(1 for inf in infos if inf["state"] < 2),
           "GBs": round(tot["hbm_bytes"] / wall / 1e9, 2), "rounds": rounds, "wall_s": round(wall, 3),
           "storage": storage, "max_live": max_live or None, "max_long": max_long or None,
           "slowest": slowest}
    return out, tot["hbm_bytes"], wall, rounds


def bench_serve(args, P, W, torch, emit=True):
    """Served BF16 (continuous batching) against the same BF16 requests served
    one at a time (a queue alone) and the plain FP64 form served one at a
    time, on the same arrival process and update schedule."""
    arrivals = W.serving_arrivals(args.rate, args.horizon, seed=args.seed)
    log(f"{len(arrivals)} arrivals over {args.horizon} s at {args.rate}/s")
    cap = max(60.0, 6.0 * args.horizon)
    ipr = args.iters_per_round
    served, bytes_, wall, rounds = serve_pass(args, P, W, torch, arrivals, "bf16", 0, cap, ipr=ipr,
                                              max_long=args.max_long)
    log("served", served)
    queue, _, _, _ = serve_pass(args, P, W, torch, arrivals, "bf16", 1, cap, ipr=ipr)
    log("bf16 one at a time", queue)
    plain, _, _, _ = serve_pass(args, P, W, torch, arrivals, "f64", 1, cap, ipr=ipr)
    log("fp64 one at a time", plain)
    value = bytes_ / wall / 1e9
    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": rounds, "warmup": 0,
        "ms_per_step": round(wall * 1e3 / max(rounds, 1), 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic (generated on the device, seeded)",
        "config": {"workload": MULTI["serve-bf16-poisson"], "rate_per_s": args.rate, "horizon_s": args.horizon,
                   "budget_gb": args.budget_gb, "iters_per_round": ipr, "max_long": args.max_long,
                   "requests": len(arrivals)},
        "pct_of_peak": round(100 * value / HBM_PEAK_GBS, 2),
        # no single kernel dominates a served pass: the aggregate algorithmic
        # bytes of every sweep of every live request over the pass's wall time
        "roofline": {"bound": "hbm", "achieved": round(value, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(value / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "sweep_batch and sweep_wide of all live requests (aggregate over the pass)"},
        "time_to_feasible": {"served_bf16_continuous_batching": served, "bf16_queue_one_at_a_time": queue,
                             "fp64_single_system_one_at_a_time": plain},
    }
    if emit:
        print(json.dumps(line), flush=True)
    return line


if __name__ == "__main__":
    main()
