"""Launch shapes (bpmf_launch_shape) and the autotuner that picks one.

Every shape cuts the same rows into different launches, so every shape must
meet the mixed-precision bounds against the FP64 oracle on the same state and
draws; the tuner must return one of the shapes it timed."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1705_10633_amd import synth

from .gpu_common import MIXED_FLOOR, MIXED_TOL, check_arith, make_sampler, row_rel_err, tape_for, within
from .test_gpu_parity import _dev, _f32_start

pytestmark = pytest.mark.gpu


def _skewed(K, seed):
    """Six users rate 1100..3000 of 3000 movies, 300 rate 0..4, 200 rate 10..29."""
    rng = np.random.default_rng(seed)
    M, N = 506, 3000
    counts = np.concatenate([rng.integers(1100, N + 1, 6), rng.integers(0, 5, 300), rng.integers(10, 30, 200)])
    rows = np.repeat(np.arange(M), counts)
    cols = np.concatenate([rng.choice(N, c, replace=False) for c in counts]).astype(np.int64)
    vals = 3.0 + rng.standard_normal(rows.size)
    R = synth.from_coo(M, N, rows, cols, vals)
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    return synth.Problem("skewed", R, K, 2.0, np.zeros(K), 2.0, float(K), np.eye(K), 1, 0,
                         f32(0.3 * rng.standard_normal((M, K))), f32(0.3 * rng.standard_normal((N, K))),
                         np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0), 0, float(vals.mean()))


SHAPES = [
    {},
    {"heavy_split": 1, "heavy_min_ratings": 1024, "piece_min_ratings": 64},
    {"heavy_split": -1, "rank1_max_ratings": -1},
    {"rank1_max_ratings": 4, "rank1_split": 1},
    {"heavy_split": 1, "heavy_min_ratings": 2048, "piece_min_ratings": 1024, "rank1_max_ratings": 1,
     "rank1_split": 1},
]


@pytest.mark.parametrize("precision,K", [("fp32", 32), ("fp32", 64), ("bf16", 64)])
def test_every_launch_shape_meets_the_oracle(precision, K):
    prob = _f32_start(_skewed(K, seed=K + 11))
    tape = tape_for(prob, 1, seed=K + 13)
    ref = O.gibbs(prob, tape, n_sweeps=1, nthreads=8)
    import torch
    for shape in SHAPES:
        s = make_sampler(prob, precision=precision, with_test=False, shape=shape)
        s.sweep(1, tape=_dev(tape))
        torch.cuda.synchronize()
        eu = row_rel_err(s.U.cpu().numpy(), ref["U"], MIXED_FLOOR)
        ev = row_rel_err(s.V.cpu().numpy(), ref["V"], MIXED_FLOOR)
        print(f"{precision} K={K} {shape}: U median {np.median(eu):.2e} max {eu.max():.2e}; "
              f"V median {np.median(ev):.2e} max {ev.max():.2e}", flush=True)
        assert within(eu, prob.R.row_counts(), MIXED_TOL[precision]), shape
        assert within(ev, prob.R.col_counts(), MIXED_TOL[precision], factor=3.0), shape
        assert s.info()["fallback_rows"] == 0
        check_arith(prob, s, tape, precision, str(shape))
        del s


def test_autotune_returns_a_timed_candidate():
    from paper_1705_10633_amd import autotune
    from paper_1705_10633_amd.sampler import DeviceRatings
    prob = _skewed(32, seed=5)
    cands = autotune.candidate_shapes([prob.R.row_counts(), prob.R.col_counts()], prob.K)
    assert len(cands) > 4
    R = DeviceRatings(prob.R, val_dtype="float32")
    best, table = autotune.tune(R, prob.K, prob.U0.astype(np.float32), prob.V0.astype(np.float32),
                                [prob.R.row_counts(), prob.R.col_counts()], precision="bf16",
                                sweeps=3, warmup=1, mean_rating=prob.mean_rating)
    assert [c for c, _ in table] == cands
    assert all(ms > 0 for _, ms in table)
    assert best in cands
    assert min(ms for _, ms in table) == next(ms for c, ms in table if c == best)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_side_entirely_in_the_rank_one_launch(precision):
    """Every user has at most two ratings and the shape forces the rank-one
    launch, so the users' one-wavefront launch is empty; with the rank-one
    kernels switched off the same rows, those without ratings included, run
    in the full kernel.  Both meet the oracle."""
    K = 32
    rng = np.random.default_rng(3)
    M, N = 700, 400
    counts = rng.integers(0, 3, M)
    rows = np.repeat(np.arange(M), counts)
    cols = np.concatenate([rng.choice(N, c, replace=False) for c in counts]).astype(np.int64)
    vals = 3.0 + rng.standard_normal(rows.size)
    R = synth.from_coo(M, N, rows, cols, vals)
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    prob = synth.Problem("all-small", R, K, 2.0, np.zeros(K), 2.0, float(K), np.eye(K), 1, 0,
                         f32(0.3 * rng.standard_normal((M, K))), f32(0.3 * rng.standard_normal((N, K))),
                         np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0), 0, float(vals.mean()))
    tape = tape_for(prob, 1, seed=9)
    ref = O.gibbs(prob, tape, n_sweeps=1, nthreads=8)
    import torch
    for shape in ({"rank1_max_ratings": 2, "rank1_split": 1}, {"rank1_max_ratings": -1}):
        s = make_sampler(prob, precision=precision, with_test=False, shape=shape)
        s.sweep(1, tape=_dev(tape))
        torch.cuda.synchronize()
        eu = row_rel_err(s.U.cpu().numpy(), ref["U"], MIXED_FLOOR)
        ev = row_rel_err(s.V.cpu().numpy(), ref["V"], MIXED_FLOOR)
        print(f"{precision} {shape}: U median {np.median(eu):.2e} max {eu.max():.2e}; "
              f"V median {np.median(ev):.2e} max {ev.max():.2e}", flush=True)
        assert within(eu, prob.R.row_counts(), MIXED_TOL[precision]), shape
        assert within(ev, prob.R.col_counts(), MIXED_TOL[precision], factor=3.0), shape
        assert s.info()["fallback_rows"] == 0
        check_arith(prob, s, tape, precision, str(shape))
        del s


def test_sampler_with_automatic_shape_meets_the_oracle():
    """shape="auto" tunes on the sampler's own problem, keeps one of the
    timed candidates, and the sampler it builds meets the oracle."""
    from paper_1705_10633_amd import autotune
    K, precision = 32, "fp32"
    prob = _f32_start(_skewed(K, seed=21))
    tape = tape_for(prob, 1, seed=22)
    ref = O.gibbs(prob, tape, n_sweeps=1, nthreads=8)
    import torch
    from paper_1705_10633_amd.sampler import DeviceRatings, Sampler
    s = Sampler(DeviceRatings(prob.R, val_dtype="float32"), K, prob.U0.astype(np.float32),
                prob.V0.astype(np.float32), precision=precision, alpha=prob.alpha, beta0=prob.beta0,
                nu0=prob.nu0, mean_rating=prob.mean_rating, shape="auto")
    cands = autotune.candidate_shapes([prob.R.row_counts(), prob.R.col_counts()], K)
    assert [c for c, _ in s.tune_table] == cands and s.shape in cands
    print(f"kept {s.shape}", flush=True)
    s.sweep(1, tape=_dev(tape))
    torch.cuda.synchronize()
    eu = row_rel_err(s.U.cpu().numpy(), ref["U"], MIXED_FLOOR)
    ev = row_rel_err(s.V.cpu().numpy(), ref["V"], MIXED_FLOOR)
    assert within(eu, prob.R.row_counts(), MIXED_TOL[precision])
    assert within(ev, prob.R.col_counts(), MIXED_TOL[precision], factor=3.0)
    check_arith(prob, s, tape, precision, f"auto {s.shape}")
    with pytest.raises(ValueError):
        Sampler(DeviceRatings(prob.R, val_dtype="float32"), K, prob.U0.astype(np.float32),
                prob.V0.astype(np.float32), precision=precision, shape="fastest")
