"""CPU safety nets: the oracle and the library's host-side checks built with
AddressSanitizer and UndefinedBehaviorSanitizer.

* The oracle's C is compiled with -fsanitize=address,undefined and every pin
  of tests/test_oracle_pins.py is run against that build, in a child process
  that preloads the sanitizer runtimes (any report fails the run: UBSan does
  not recover, ASan aborts).
* The host-side validation and admission logic of the library
  (paper_2003_09956_amd/csrc/validate.cpp, which needs no device) is linked
  with a test driver under the same sanitizers and run.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.fixture(scope="module")
def runtimes():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    return asan, ubsan


def test_oracle_pins_under_address_and_undefined_behaviour_sanitizers(tmp_path, runtimes):
    lib = tmp_path / "liboracle_san.so"
    subprocess.check_call(["gcc", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", *SAN,
                           os.path.join(ROOT, "oracle", "modap_oracle.c"), "-o", str(lib), "-lm"])
    env = dict(os.environ)
    # the sanitizer runtimes first, before anything the environment already preloads
    env["LD_PRELOAD"] = " ".join([*runtimes, env.get("LD_PRELOAD", "")]).strip()
    env["ASAN_OPTIONS"] = "detect_leaks=0:verify_asan_link_order=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["MODAP_ORACLE_LIB"] = str(lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert " passed" in out


def test_host_validation_under_sanitizers(tmp_path, runtimes):
    exe = tmp_path / "validate_test"
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2003_09956_amd", "csrc"),
                           os.path.join(ROOT, "paper_2003_09956_amd", "csrc", "validate.cpp"),
                           os.path.join(ROOT, "tests", "native", "validate_test.cpp"), "-o", str(exe)])
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([str(exe)], env=env, capture_output=True, text=True, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "all host checks passed" in out, out[-4000:]
