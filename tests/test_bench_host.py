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



def test_users_by_count_relabelling_is_a_permutation():
    """The reordering option renumbers users in descending rating count and
    carries U0 and the held-out pairs along: the same ratings, the same
    predictions from the same factors."""
    import numpy as np
    from oracle import oracle as O
    from paper_1705_10633_amd import synth
    p = synth.uniform_planted(M=300, N=120, K=4, nnz=4000, seed=9, n_sweeps=1)
    q = synth.relabel_users_by_count(p)
    c = q.R.row_counts()
    assert np.all(c[:-1] >= c[1:]) and q.R.nnz == p.R.nnz
    assert sorted(c.tolist()) == sorted(p.R.row_counts().tolist())
    np.testing.assert_array_equal(O.predict(p.U0, p.V0, p.test_rows, p.test_cols, 3.0),
                                  O.predict(q.U0, q.V0, q.test_rows, q.test_cols, 3.0))
    # each user's set of (movie, rating) pairs is kept
    new_of_old = np.empty(300, np.int64)
    new_of_old[np.argsort(-p.R.row_counts(), kind="stable")] = np.arange(300)
    for u in (0, 17, 299):
        a = p.R.col_idx[p.R.row_ptr[u]:p.R.row_ptr[u + 1]]
        v = new_of_old[u]
        b = q.R.col_idx[q.R.row_ptr[v]:q.R.row_ptr[v + 1]]
        np.testing.assert_array_equal(a, b)
