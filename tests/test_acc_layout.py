"""CPU check of the Gram accumulator layouts (csrc/common.hpp).

The Normal-Wishart step writes Lambda / alpha into the K <= 64 row kernel's
accumulator layout with lambda_acc_index, and the row kernel starts its Gram
accumulators from it. The check compiles the header as plain C++ (a host
stand-in for the HIP runtime header) and verifies, for the 32 x 32 and the
16 x 16 tile layouts, that every accumulator slot is written exactly once and
that slot i * 64 + l holds the entry the matrix cores leave in element i of
lane l. The hardware's own lane layout is pinned by the GPU parity tests.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _clang():
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if c and os.path.exists(c):
            return c
    pytest.skip("clang++ is not available")


def test_accumulator_layouts_agree(tmp_path):
    exe = str(tmp_path / "acc_layout_check")
    subprocess.check_call([_clang(), "-std=c++17", "-O1",
                           "-I", os.path.join(ROOT, "tests", "layout"),
                           "-I", os.path.join(ROOT, "paper_1705_10633_amd", "csrc"),
                           "-o", exe, os.path.join(ROOT, "tests", "layout", "acc_layout_check.cpp")])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    print(r.stdout)
    assert r.returncode == 0 and "layout checks passed" in r.stdout
