"""The C-ABI library loads and exports every entry point its header declares.

CPU-only: no compute call is made here (there is no GPU in this environment);
only calls that return before touching a device are exercised.
"""
import ctypes as C
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "modap.h")


@pytest.fixture(scope="module")
def L():
    import paper_2003_09956_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_2003_09956_amd import _build
        _build.build()
    return P.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(modap_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for verb in ("create", "destroy", "set_system", "update_coeffs", "iterate", "solve",
                 "eval_sweep", "query", "strerror"):
        assert f"modap_{verb}" in names


def test_every_declared_symbol_is_exported(L):
    import paper_2003_09956_amd as P
    names = declared_functions()
    assert sorted(P.EXPORTS) == names
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for name in names:
        assert name in exported, name
        assert getattr(L, name) is not None


def test_no_torch_in_the_abi():
    """Declarations use plain C types only (comments may mention callers)."""
    text = open(HEADER).read()
    code = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    assert "torch" not in code.lower() and "::" not in code and "std::" not in code
    assert "extern \"C\"" in text


def test_strerror_covers_every_status(L):
    msgs = [L.modap_strerror(s).decode() for s in range(9)]
    assert msgs[0] == "ok"
    assert len(set(msgs)) == 9
    assert L.modap_strerror(99).decode() == "unknown status"


def test_null_context_is_rejected_without_a_device(L):
    assert L.modap_set_system(None, 1, 1, 0, None, 1, None, None, 0) == 1
    assert L.modap_iterate(None, None, 1, None) == 1
    assert L.modap_solve(None, None, None) == 1
    assert L.modap_query(None, None, None, None, 0) == 1
    assert L.modap_eval_sweep(None, None, None, None, None, None, 0) == 1
    assert L.modap_update_coeffs(None, 0, None, None, None, None, 0) == 1
    assert L.modap_set_drift(None, 0, None, 0, 0) == 1
    assert L.modap_set_x(None, None, 0) == 1
    assert L.modap_get_tile(None, None) == 1
    assert L.modap_last_error(None).decode() == "null context"
    L.modap_destroy(None)


def test_create_fails_cleanly_without_gpu(L):
    from conftest import gpu_available
    if gpu_available():
        pytest.skip("a GPU is present")
    ctx = C.c_void_p()
    assert L.modap_create(0, None, C.byref(ctx)) in (4, 1)
    assert not ctx.value
    assert L.modap_create(0, None, None) == 1


def test_binding_has_no_cpu_fallback(tmp_path, monkeypatch):
    """The Python binding raises when the library is missing; it never computes on the CPU."""
    import paper_2003_09956_amd as P
    monkeypatch.setattr(P, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(P, "_lib", None)
    with pytest.raises(ImportError):
        P.lib()


def test_product_never_imports_the_oracle():
    """Only tests, the smoke check and the benchmark's CPU leg may use oracle/."""
    pkg = os.path.join(ROOT, "paper_2003_09956_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".inc", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), f


C_TYPES = {"int32_t": C.c_int32, "int64_t": C.c_int64, "double": C.c_double}


@pytest.mark.parametrize("cls,name", [("Params", "modap_params"), ("Stats", "modap_stats"), ("Tile", "modap_tile"),
                                      ("BatchStats", "modap_batch_stats"), ("BatchTile", "modap_batch_tile"),
                                      ("RequestInfo", "modap_request_info")])
def test_binding_structs_follow_the_header(cls, name):
    """Every struct the binding passes across the boundary has the header's
    fields, in the header's order, with the header's types."""
    import paper_2003_09956_amd as P
    code = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + r";", code).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        ctype, names = decl.split(None, 1)
        for nm in names.split(","):
            arr = re.fullmatch(r"\s*(\w+)\s*\[(\d+)\]\s*", nm)
            fields.append((arr.group(1), C_TYPES[ctype] * int(arr.group(2))) if arr else (nm.strip(), C_TYPES[ctype]))
    # (a field named by a Python keyword carries a trailing underscore)
    got = [(f.rstrip("_"), t) for f, t in getattr(P, cls)._fields_]
    assert [f for f, _ in got] == [f for f, _ in fields]
    for (f, t), (_, u) in zip(got, fields):
        assert C.sizeof(t) == C.sizeof(u) and getattr(t, "_type_", t) == getattr(u, "_type_", u), f


def test_library_records_its_tracing_ranges():
    """The library links the ROCm tracing-range API (one range per call, per
    queued chunk of a solve, per served request)."""
    import paper_2003_09956_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("library not built")
    out = subprocess.run(["readelf", "-d", P.LIB_PATH], capture_output=True, text=True).stdout
    assert "librocprofiler-sdk-roctx" in out
    und = subprocess.run(["nm", "-D", "--undefined-only", P.LIB_PATH], capture_output=True, text=True).stdout
    for sym in ("roctxRangePushA", "roctxRangePop", "roctxRangeStartA", "roctxRangeStop"):
        assert sym in und, sym


def test_loading_the_library_first_maps_one_hip_runtime():
    """Loading the library before anything imports torch leaves a single HIP
    runtime mapped in the process (torch brings its own copy; two runtimes in
    one process share no device state)."""
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_2003_09956_amd as P; P.lib(); import torch\n"
            "maps = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
            "print(len(maps))" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().splitlines()[-1] == "1", r.stdout
