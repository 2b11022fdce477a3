"""Sampled parity at full size, in the configuration the benchmark times.

One sweep of the MovieLens-shaped problem (138,493 x 26,744, 20M ratings,
K = 64, BF16 gathers and Gram, FP32 Cholesky, device Philox draws, HIP-graph
replay), of the ChEMBL-shaped one (483,500 x 5,775, 1.02M ratings, K = 32,
FP32) and of the Netflix-shaped one (480,189 x 17,770, 100M ratings, K = 128,
BF16, the blocked four-wavefront kernel), from the same library calls the
benchmark makes. The oracle
cannot redo a whole sweep in seconds, so it recomputes

  * both Normal-Wishart steps (Alg. 1, hyper-parameter draws) from the same
    start state and the same Philox draws, to the FP64 bar;
  * a sample of rows of each half-sweep: the heaviest rows, the lightest rows
    and a uniform sample, from the state the GPU saw and the hyper-parameters
    it drew (row conditional of section 2, Cholesky form of section 3.1);
  * a sample of the held-out predictions.

The row noise is the oracle's FP64 Box-Muller of the same Philox counters;
the mixed kernels make it in FP32, a relative difference of ~1e-7 that is far
below the mixed tolerances.

For the rows two comparisons are made. Against the FP32 state the error is
the mixed-precision error and is held to the one-sweep mixed tolerances.
Against the oracle fed what the kernels read (the FP32 rating offsets, and
in BF16 mode the gathered side rounded to BF16 with round to nearest even, as
the kernels store their BF16 copies) only the FP32 arithmetic is left, so the
bound is the FP32 arithmetic one: this separates rounding of the inputs from
mistakes in the arithmetic.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1705_10633_amd import synth

from .gpu_common import ARITH_TOL, MIXED_FLOOR, MIXED_TOL, _r_eff, bf16_round, make_sampler, row_rel_err, within

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
SEED = 0x5EED2024


def _pick(counts, n_uniform, n_ends, rng):
    order = np.argsort(counts, kind="stable")
    pick = np.concatenate([order[:n_ends], order[-n_ends:],
                           rng.choice(counts.size, size=n_uniform, replace=False)])
    return np.unique(pick)


def _sub_csr(ptr, idx, val, rows):
    cnt = ptr[rows + 1] - ptr[rows]
    sp = np.zeros(rows.size + 1, np.int64)
    np.cumsum(cnt, out=sp[1:])
    sel = np.concatenate([np.arange(ptr[i], ptr[i + 1]) for i in rows])
    return sp, idx[sel], val[sel]


def _oracle_rows(ptr, idx, val, rows, other, prob, Lam, mu, Z):
    sp, si, sv = _sub_csr(ptr, idx, val, rows)
    return O.half_sweep(sp, si, sv, other, prob.alpha, prob.mean_rating, Lam, mu, Z[rows], nthreads=8)


def _check_full_size(prob, precision, n_uniform=1500, n_ends=100):
    import torch
    K = prob.K
    U0 = prob.U0.astype(np.float32)
    V0 = prob.V0.astype(np.float32)
    s = make_sampler(prob, precision=precision, seed=SEED, use_graph=True)
    s.sweep(1)
    torch.cuda.synchronize()
    U1 = s.U.cpu().numpy()
    V1 = s.V.cpu().numpy()
    h = s.hyper()
    info = s.info()
    assert info["nonfinite_rows"] == 0
    assert np.all(np.isfinite(U1)) and np.all(np.isfinite(V1))

    # Normal-Wishart draws of both sides from the state they were drawn from;
    # a half-sweep's draws are [K chi^2][K(K-1)/2 Bartlett][K mean][n K row normals]
    R = prob.R
    nb = K * (K - 1) // 2
    Z = {}
    for side, X, n, hs in (("U", U0, R.M, 0), ("V", V0, R.N, 1)):
        blk = O.philox_block(SEED, hs, n, K, prob.nu0)
        chi2, zb, zm = blk[:K], blk[K:K + nb], blk[K + nb:2 * K + nb]
        Z[side] = blk[2 * K + nb:].reshape(n, K)
        Lam, mu = O.nw(X.astype(np.float64), prob.mu0, prob.beta0, prob.nu0, prob.W0, chi2, zb, zm)
        eL = np.max(np.abs(h["Lambda_" + side] - Lam)) / np.max(np.abs(Lam))
        em = np.max(np.abs(h["mu_" + side] - mu)) / max(1.0, np.max(np.abs(mu)))
        print(f"{prob.name} NW({side}) over {n} rows: rel err Lambda {eL:.2e} mu {em:.2e}")
        assert eL <= FP64_TOL and em <= FP64_TOL

    rng = np.random.default_rng(7)
    for side, ptr, idx, val, other, X1, n in (("U", R.row_ptr, R.col_idx, R.row_val, V0, U1, R.M),
                                              ("V", R.col_ptr, R.row_idx, R.col_val, U1, V1, R.N)):
        counts = ptr[1:] - ptr[:-1]
        rows = _pick(counts, min(n_uniform, n // 2), min(n_ends, n // 4), rng)
        Lam, mu = h["Lambda_" + side], h["mu_" + side]
        ref = _oracle_rows(ptr, idx, val, rows, other.astype(np.float64), prob, Lam, mu, Z[side])
        err = row_rel_err(X1[rows], ref, MIXED_FLOOR)
        print(f"{prob.name} {precision} {side}: {rows.size} rows (nnz {counts[rows].min()}..{counts[rows].max()}), "
              f"vs FP32 state median {np.median(err):.2e} max {err.max():.2e}")
        worst = np.argsort(err)[-5:]
        print("  worst rows (row, ratings, |x|, error): " +
              ", ".join(f"({rows[w]}, {counts[rows[w]]}, {np.linalg.norm(ref[w]):.3g}, {err[w]:.2e})" for w in worst))
        assert within(err, counts[rows], MIXED_TOL[precision], factor=1.0 if side == "U" else 3.0)
        g = (bf16_round(other) if precision == "bf16" else other.astype(np.float32)).astype(np.float64)
        ref_b = _oracle_rows(ptr, idx, _r_eff(val, prob.mean_rating), rows, g, prob, Lam, mu, Z[side])
        err_b = row_rel_err(X1[rows], ref_b, MIXED_FLOOR)
        print(f"ARITH {prob.name} {precision} {side}: vs the kernels' inputs median {np.median(err_b):.2e} "
              f"max {err_b.max():.2e}")
        assert within(err_b, counts[rows], ARITH_TOL[precision])

    # held-out predictions after one sweep (burn-in 0): U1 . V1 + rbar, FP64 accumulation
    mean, cnt = s.test_predictions()
    mean = mean.cpu().numpy()
    assert cnt == 1
    t = rng.choice(prob.test_rows.size, size=5000, replace=False)
    ref_p = O.predict(U1.astype(np.float64), V1.astype(np.float64), prob.test_rows[t], prob.test_cols[t],
                      prob.mean_rating)
    np.testing.assert_allclose(mean[t], ref_p, rtol=1e-12, atol=1e-12)


def test_movielens_shaped_bf16_sampled_parity():
    prob = synth.movielens_like(burnin=0)
    _check_full_size(prob, "bf16")


def test_chembl_shaped_fp32_sampled_parity():
    prob = synth.chembl_like(burnin=0)
    _check_full_size(prob, "fp32")


def test_netflix_shaped_bf16_sampled_parity():
    prob = synth.netflix_like(burnin=0)
    _check_full_size(prob, "bf16", n_uniform=600, n_ends=50)
