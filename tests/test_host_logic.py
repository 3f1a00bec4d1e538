"""CPU tests of host-side logic: the benchmark's counter lookup and
percentiles, and the seeded input generators (same seed, same inputs; the
shapes and value distributions the workloads state)."""
import math
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import workloads as W  # noqa: E402

TILE = {"block": 256, "lanes_per_row": 256, "chunks": 8, "rows_per_step": 1, "depth": 2, "interleave": 0,
        "grid": 256}


def write_counters(root, dt, n, m, tile, source_hash, bytes_per_launch):
    os.makedirs(os.path.join(root, "profiles"), exist_ok=True)
    path = os.path.join(root, "profiles", f"sweep_wide_{dt}_n{n}_m{m}_tile{tile.replace(',', '-')}_counters.txt")
    with open(path, "w") as f:
        f.write("# a comment line = ignored\n")
        f.write(f"tile = {tile}\nsource_hash = {source_hash}\nbytes_per_launch = {bytes_per_launch}\n")
    return path


def test_tile_string_names_every_field_in_order():
    assert bench.tile_str(TILE) == "256,256,8,1,2,0,256"
    assert bench.counters_path("f32", 8192, 16384, "256,256,8,1,2,0,256").endswith(
        os.path.join("profiles", "sweep_wide_f32_n8192_m16384_tile256-256-8-1-2-0-256_counters.txt"))


def test_traffic_is_reported_only_for_the_current_kernel_source(tmp_path, monkeypatch):
    # the hash is taken over the real sources; the counter file lives in a scratch root
    h = bench.kernel_source_hash("f32")
    monkeypatch.setattr(bench, "counters_path",
                        lambda dt, n, m, tile: os.path.join(tmp_path, "profiles",
                                                            f"sweep_wide_{dt}_n{n}_m{m}_tile"
                                                            f"{tile.replace(',', '-')}_counters.txt"))
    assert bench.measured_traffic("f32", 8192, 16384, TILE) is None          # no file
    write_counters(tmp_path, "f32", 8192, 16384, "256,256,8,1,2,0,256", h, 547205521)
    assert bench.measured_traffic("f32", 8192, 16384, TILE) == 547205521
    write_counters(tmp_path, "f32", 8192, 16384, "256,256,8,1,2,0,256", "0" * 16, 547205521)
    assert bench.measured_traffic("f32", 8192, 16384, TILE) is None          # kernel changed since
    other = dict(TILE, grid=512)
    assert bench.measured_traffic("f32", 8192, 16384, other) is None         # another launch shape


def test_batch_tile_string_and_counter_lookup(tmp_path, monkeypatch):
    """The batch tile names its item sizes and grid, then the least items per
    system when it is not the library's choice; a batch counter file counts
    only for its family, its tile and the current batch kernel and plan."""
    t0 = {"item_kib": [512, 2048, 4096, 8192], "grid": 0, "min_items": 0}
    t2 = dict(t0, item_kib=[16384, 2048, 4096, 8192], min_items=2)
    assert bench.batch_tile_str(t0) == "512,2048,4096,8192,0"
    assert bench.batch_tile_str(t2) == "16384,2048,4096,8192,0,2"
    assert bench.batch_counters_path("16384,2048,4096,8192,0,2", "batch-f32-512-n256").endswith(
        os.path.join("profiles", "sweep_batch_f32_512x256_tile16384-2048-4096-8192-0-2_counters.txt"))
    real = bench.batch_counters_path
    monkeypatch.setattr(bench, "batch_counters_path",
                        lambda tile, wl="batch-f32-512": os.path.join(tmp_path, os.path.basename(real(tile, wl))))
    path = bench.batch_counters_path("16384,2048,4096,8192,0,2", "batch-f32-512-n256")

    def put(tile, h):
        open(path, "w").write(f"tile = {tile}\nsource_hash = {h}\nbytes_per_launch = 1103400000\n")
    assert bench.measured_batch_traffic(t2, "batch-f32-512-n256") is None            # no file
    put("16384,2048,4096,8192,0,2", bench.batch_source_hash())
    assert bench.measured_batch_traffic(t2, "batch-f32-512-n256") == 1103400000
    assert bench.measured_batch_traffic(t0, "batch-f32-512-n256") is None            # another tile
    assert bench.measured_batch_traffic(t2, "batch-f32-512") is None                 # another family
    put("16384,2048,4096,8192,0,2", "0" * 16)
    assert bench.measured_batch_traffic(t2, "batch-f32-512-n256") is None            # sources changed
    # the hash covers the batch kernel and the rules that cut systems into items
    assert any(p.endswith("batch_plan.hpp") for p in bench.BATCH_SOURCES)
    assert not any(p.endswith("batch.hip") for p in bench.BATCH_SOURCES)


def test_kernel_source_hash_depends_on_the_storage_table():
    assert bench.kernel_source_hash("f32") != bench.kernel_source_hash("bf16")
    assert len(bench.kernel_source_hash("f64")) == 16


def test_percentile_of_samples():
    assert bench.percentile([1.0, 2.0, 3.0, 4.0], 50) == pytest.approx(2.5)
    assert bench.percentile([], 50) is None
    # the drift chase counts an unfinished run as slower than every finished one
    v = np.asarray([3.0, 1.0, math.inf, 2.0])
    assert float(np.percentile(v, 50, method="higher")) == 3.0
    assert math.isinf(float(np.percentile(v, 99, method="higher")))


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_gaussian_generator_is_seeded_and_feasible(dtype):
    a = W.gaussian(40, 90, seed=3, dtype=dtype)
    b = W.gaussian(40, 90, seed=3, dtype=dtype)
    c = W.gaussian(40, 90, seed=4, dtype=dtype)
    assert np.array_equal(a.A, b.A) and np.array_equal(a.b, b.b)
    assert not np.array_equal(a.A, c.A)
    A64 = W.stored_to_f64(a.A, dtype)
    # rows normalised before rounding to the storage type; the hidden point is strictly feasible
    assert np.allclose(np.linalg.norm(A64, axis=1), 1.0, atol={"f64": 1e-12, "f32": 1e-6, "bf16": 1e-2}[dtype])
    assert np.all(A64 @ a.z < a.b)


def test_box_sum_generator_shape_and_rows():
    s = W.box_sum(8, seed=1, dtype="f64")
    assert s.A.shape == (17, 8)
    A = s.A
    assert np.array_equal(A[:8], np.eye(8)) and np.array_equal(A[8:16], -np.eye(8))
    assert np.array_equal(A[16], np.ones(8))


def test_batch_shapes_follow_the_stated_ranges():
    shapes = W.batch_shapes(512, seed=0)
    assert len(shapes) == 512 and shapes == W.batch_shapes(512, seed=0)
    assert all(64 <= n <= 2048 and 2 * n <= m <= 8 * n for n, m in shapes)


def test_serving_arrivals_are_poisson_and_log_uniform():
    arr = W.serving_arrivals(5.0, 200.0, seed=1)
    t = np.array([a[0] for a in arr])
    n = np.array([a[1] for a in arr])
    assert np.all(np.diff(t) > 0) and t[-1] < 200.0
    assert abs(len(arr) / 200.0 - 5.0) < 1.0                       # rate within a few sigma
    assert np.all((n >= 128) & (n <= 16384)) and all(a[2] == 4 * a[1] for a in arr)
    # log-uniform: about half the sizes below the geometric mean of the range
    assert 0.4 < np.mean(n < math.sqrt(128 * 16384)) < 0.6


def test_drift_is_seeded_gaussian():
    V = W.drift(1000, 50, sigma=1e-2, seed=7)
    assert V.shape == (50, 1000) and np.array_equal(V, W.drift(1000, 50, sigma=1e-2, seed=7))
    assert abs(V.std() / 1e-2 - 1.0) < 0.02 and abs(V.mean()) < 1e-3


def test_counter_hash_follows_code_not_comments(tmp_path, monkeypatch):
    a = "// first\nint f(int x) { return x + 1; }  /* block\n comment */\n"
    b = "// another comment\nint f(int x)   {\n  return x + 1;   // the same code\n}\n"
    c = "int f(int x) { return x + 2; }\n"
    for name, text in (("a.hpp", a), ("b.hpp", b), ("c.hpp", c)):
        (tmp_path / name).write_text(text)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench._code_only("a.hpp") == bench._code_only("b.hpp")
    assert bench._code_only("a.hpp") != bench._code_only("c.hpp")


def test_catchup_line_quotes_the_papers_rates_as_context():
    ctx = bench.paper_catchup_context(32000)
    assert [(r["nodes"], r["per_coord"], r["total"]) for r in ctx["runs"]] == [(50, 10, 1789), (75, 15, 2683),
                                                                               (100, 18, 3220)]
    assert [r["nodes"] for r in bench.paper_catchup_context(54000)["runs"]] == [75, 100, 150]
    assert bench.paper_catchup_context(1000) is None          # no printed run at this size


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_step_line_keeps_the_benchmark_contract():
    """The line of a single-system workload carries every field the driver
    reads, value is whole-step bytes over wall time, and the roofline object
    is the sweep kernel's achieved rate over the HBM peak."""
    import argparse
    args = argparse.Namespace(steps=200, warmup=20, device_warmup=0.3)
    bps = 16384 * 65536 * 2 + 24 * 65536
    res = {"tile": dict(TILE, kind=0), "wall": 200 * 322e-6, "wall_profiled": 200 * 337e-6,
           "sweep_us": 315.0, "reduce_us": 5.5, "profiled": 200, "upload_s": 0.0, "host_bytes": 0,
           "feasible_steps": 0, "bytes_per_step": bps, "on_host": False, "warm_sweeps": 800}
    line = bench.step_line(args, "bf16", 16384, 65536, "BF16 test system", res)
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert key in line, key
    assert line["metric"] == bench.METRIC and line["unit"] == "GB/s" and line["n_gpus"] == 1
    assert line["steps"] == 200 and line["warmup"] == 20 and line["higher_is_better"] is True
    assert line["vs_baseline"] is None and line["dtype"] == "bf16" and "workload" in line["config"]
    assert line["value"] == pytest.approx(bps * 200 / (200 * 322e-6) / 1e9, rel=1e-4)
    assert line["ms_per_step"] == pytest.approx(0.322, rel=1e-4)
    r = line["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == bench.HBM_PEAK_GBS == 8000.0
    assert r["achieved"] == pytest.approx(bps / 315e-6 / 1e9, rel=1e-4)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], abs=1e-4)
    assert "traffic" in r and line["device_warmup"]["stateless_sweeps"] == 800
