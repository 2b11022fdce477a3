"""Host-side parts of bench.py that need no GPU: the refusal of more than one
GPU, the counter-summary lookup, and the oracle baseline's sampling."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1705_10633_amd import synth  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_traffic_is_reported_only_for_the_profiled_sources():
    traffic, note = bench.measured_traffic()
    with open(bench.TRAFFIC_PROFILE) as f:
        text = f.read()
    recorded = [l.split(":", 1)[1].strip() for l in text.splitlines() if l.startswith("kernel_sources_sha256:")]
    assert len(recorded) == 1
    if recorded[0] == bench.row_kernel_digest():
        assert traffic is not None and traffic > 0 and "FETCH_SIZE" in note
    else:
        assert traffic is None and "changed" in note


def test_cpu_baseline_whole_sweeps_and_row_sample():
    prob = synth.uniform_planted(M=600, N=300, K=8, nnz=6000, seed=3, n_sweeps=1, burnin=0)
    whole = bench.cpu_baseline(prob, n_sweeps=1)
    assert whole["kind"] == "oracle" and whole["unit"] == "rows/s" and whole["value"] > 0
    assert whole["cores"] >= 1 and "whole FP64 oracle sweeps" in whole["sample"]
    R = prob.R
    flops = 2.0 * R.nnz * prob.K ** 2 + (R.M + R.N) * prob.K ** 3 / 3.0
    part = bench.row_sample(prob, 1, 0.5, 7, flops)
    assert part["cores"] == 1 and part["value"] > 0 and "sample of the rows" in part["sample"]
    assert isinstance(bench.host_cpu_model(), str)

