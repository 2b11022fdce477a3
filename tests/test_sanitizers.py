"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The sampler's planning code (csrc/plan.hpp: structure checks of the rating
  matrix, the host Cholesky of W0, the launch table and record offsets) is
  compiled with g++ -fsanitize=address,undefined into a driver that checks
  its invariants on random count patterns under every launch-shape choice.
* The FP64 oracle is compiled with gcc and the same sanitizers, and the
  oracle's pin tests run against it in a child process with libasan
  preloaded.
Any sanitizer report aborts the program and fails the test.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV_ASAN = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1", "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _libasan():
    out = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not out or not os.path.exists(out):
        pytest.skip("libasan is not available")
    return out


def test_planning_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_check")
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "paper_1705_10633_amd", "csrc"),
                           "-o", exe, os.path.join(ROOT, "tests", "sanitize", "plan_check.cpp")])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env={**os.environ, **ENV_ASAN})
    print(r.stdout, r.stderr[-2000:])
    assert r.returncode == 0 and "plan checks passed" in r.stdout


def test_oracle_pins_under_sanitizers(tmp_path):
    from oracle import oracle
    lib = oracle.build_sanitized(str(tmp_path / "liboracle_asan.so"))
    env = {**os.environ, **ENV_ASAN, "LD_PRELOAD": _libasan(), "BPMF_ORACLE_LIB": lib}
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu and not slow",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_rank_one_algebra.py")],
                       capture_output=True, text=True, timeout=600, env=env, cwd=ROOT)
    print(r.stdout[-1500:], r.stderr[-2000:])
    assert r.returncode == 0
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
