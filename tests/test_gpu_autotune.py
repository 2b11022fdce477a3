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


@pytest.mark.parametrize("precision,variant", [(p, v) for p in ("fp32", "bf16") for v in (1, 2, 3)])
def test_every_kernel_variant_meets_the_oracle(precision, variant):
    """The code variants of the one-wavefront K = 64 kernel (trailing updates
    on matrix cores or vector units, 4 or 3 wavefronts per SIMD) sample the
    same conditional: each meets the oracle at the arithmetic bound, with
    heavy rows cut into pieces so the combine launch runs the variant too."""
    K = 64
    prob = _f32_start(_skewed(K, seed=K + 31))
    tape = tape_for(prob, 1, seed=K + 33)
    shape = {"kernel_variant": variant, "heavy_split": 1, "heavy_min_ratings": 1024, "piece_min_ratings": 256}
    import torch
    s = make_sampler(prob, precision=precision, with_test=False, shape=shape)
    assert s.info()["kernel_variant"] == variant and s.info()["heavy_rows"][0] == 6
    s.sweep(1, tape=_dev(tape))
    torch.cuda.synchronize()
    assert s.info()["fallback_rows"] == 0
    check_arith(prob, s, tape, precision, f"variant {variant}")


def test_autotune_returns_a_timed_candidate():
    """K = 64: the three kernel variants are timed with the built-in cuts and
    a cost model a rows + b ratings is fitted to each from its two row
    launches; then the cut candidates of the fastest variant that the model
    leaves in.  The kept shape is the fastest timed one."""
    from paper_1705_10633_amd import autotune
    from paper_1705_10633_amd.sampler import DeviceRatings
    prob = _skewed(64, seed=5)
    counts = [prob.R.row_counts(), prob.R.col_counts()]
    R = DeviceRatings(prob.R, val_dtype="float32")
    best, table = autotune.tune(R, prob.K, prob.U0.astype(np.float32), prob.V0.astype(np.float32),
                                counts, precision="bf16", sweeps=3, warmup=1, mean_rating=prob.mean_rating)
    fits = autotune.variant_fits()
    assert [f["variant"] for f in fits] == [1, 2, 3]
    assert [c for c, _ in table[:3]] == [{"kernel_variant": v} for v in (1, 2, 3)]
    for f in fits:
        print(f"variant {f['variant']}: {f['ms_per_sweep']:.3f} ms/sweep, a = {f['a_us_per_row']:.3g} us/row, "
              f"b = {f['b_us_per_rating']:.3g} us/rating", flush=True)
        assert f["ms_per_sweep"] > 0 and np.isfinite(f["a_us_per_row"]) and np.isfinite(f["b_us_per_rating"])
        assert len(f["launches"]) == 2
    fastest = min(fits, key=lambda f: f["ms_per_sweep"])["variant"]
    assert all(c.get("kernel_variant") == fastest for c, _ in table[3:])
    assert len(table) > 4 and all(ms > 0 for _, ms in table)
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
    import os
    os.environ["BPMF_TUNE_CACHE"] = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"bpmf_tune_{os.getpid()}.json")
    if os.path.exists(os.environ["BPMF_TUNE_CACHE"]):
        os.remove(os.environ["BPMF_TUNE_CACHE"])
    mk = lambda: Sampler(DeviceRatings(prob.R, val_dtype="float32"), K, prob.U0.astype(np.float32),
                         prob.V0.astype(np.float32), precision=precision, alpha=prob.alpha, beta0=prob.beta0,
                         nu0=prob.nu0, mean_rating=prob.mean_rating, shape="auto")
    s = mk()
    assert not s.tune_cached and s.shape in [c for c, _ in s.tune_table]
    print(f"kept {s.shape}", flush=True)
    # the second sampler of the same problem takes the cached shape without tuning
    again = mk()
    assert again.tune_cached and again.shape == s.shape and again.tune_table is None
    del again
    os.remove(os.environ.pop("BPMF_TUNE_CACHE"))
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
