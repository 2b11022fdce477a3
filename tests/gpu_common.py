"""Helpers shared by the GPU tests: build a sampler for a synth.Problem and
compare against the oracle."""
import math

import numpy as np

from paper_1705_10633_amd import synth


def make_sampler(prob, precision="fp64", val_dtype=None, seed=0, use_graph=False, validate=True,
                 with_test=True, rbar=None, shape=None):
    import torch  # noqa: F401
    from paper_1705_10633_amd.sampler import DeviceRatings, Sampler
    if val_dtype is None:
        val_dtype = "float64" if precision == "fp64" else "float32"
    R = DeviceRatings(prob.R, val_dtype=val_dtype)
    U0, V0 = prob.U0, prob.V0
    if precision != "fp64":
        U0 = U0.astype(np.float32)
        V0 = V0.astype(np.float32)
    s = Sampler(R, prob.K, U0, V0, precision=precision, alpha=prob.alpha, beta0=prob.beta0,
                nu0=prob.nu0, mu0=prob.mu0, W0=prob.W0,
                mean_rating=prob.mean_rating if rbar is None else rbar, seed=seed,
                burnin=prob.burnin, test_rows=prob.test_rows if with_test else None,
                test_cols=prob.test_cols if with_test else None, use_graph=use_graph,
                validate=validate, shape=shape)
    return s


def row_rel_err(A, B, floor=1e-3):
    """Per-row ||A_i - B_i|| / max(||B_i||, floor sqrt(K) rms(B)): relative to
    the row's norm, floored at a fraction of a typical row norm (rounding
    errors scale with the terms a row sums, not with the result, so a row
    that happens to be near zero would otherwise show a large relative
    error; the FP64 bar uses floor = 1e-3 / sqrt(K), the mixed bounds 0.1)."""
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    rms = np.sqrt(np.mean(B * B)) if B.size else 1.0
    den = np.maximum(np.linalg.norm(B, axis=1), floor * math.sqrt(B.shape[1]) * rms)
    return np.linalg.norm(A - B, axis=1) / den


def row_rel_err_fp64(A, B):
    """The FP64 bar's per-row error: ||A_i - B_i|| / max(||B_i||, 1e-3 rms(B))."""
    B = np.asarray(B, np.float64)
    return row_rel_err(A, B, floor=1e-3 / math.sqrt(B.shape[1]))


# Floor of the mixed-precision row errors (a tenth of a typical row norm).
MIXED_FLOOR = 0.1


def tape_for(prob, n_sweeps, seed=7):
    return synth.make_tape(np.random.default_rng(seed), n_sweeps, prob.M, prob.N, prob.K, prob.nu0)


def bf16_round(x):
    """FP32 -> BF16 -> FP32 with round to nearest, ties to even (as the kernels
    store their BF16 copies)."""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32)


def _r_eff(vals, rbar):
    """Ratings whose offset r - rbar, taken in FP64 by the oracle, is the FP32
    value fl32(fl32(r) - fl32(rbar)) the kernels multiply."""
    r32 = np.asarray(vals, np.float64).astype(np.float32)
    d = (r32 - np.float32(rbar)).astype(np.float32)
    return rbar + d.astype(np.float64)


def arith_errors(prob, s, tape, precision, rbar=None):
    """Per-row relative errors of a mixed-precision sampler's U and V after one
    sweep from the tape's first sweep, against the FP64 oracle's two
    half-sweeps fed what the kernels read: the FP32 rating offsets, the
    gathered side as stored (the FP32 master, or its BF16 copy in BF16 mode,
    the movies' half gathering the GPU's own new U) and the GPU's
    hyper-parameters (themselves checked against the oracle at 1e-10
    elsewhere).  What is left is the FP32 arithmetic of the Gram, the
    factorisation and the solves, plus in BF16 mode the two-part BF16 form
    of r - rbar in the right-hand side (carried to about 2^-17)."""
    from oracle import oracle as O
    R, K = prob.R, prob.K
    rb = prob.mean_rating if rbar is None else rbar
    h = s.hyper()
    nb = K * (K - 1) // 2
    hb = 2 * K + nb
    Zu = tape[hb:hb + R.M * K].reshape(R.M, K)
    o = hb + R.M * K
    Zv = tape[o + hb:o + hb + R.N * K].reshape(R.N, K)
    G = bf16_round if precision == "bf16" else (lambda a: np.asarray(a, np.float32))
    U1 = s.U.cpu().numpy().astype(np.float32)
    V1 = s.V.cpu().numpy()
    U_ref = O.half_sweep(R.row_ptr, R.col_idx, _r_eff(R.row_val, rb), G(prob.V0).astype(np.float64),
                         prob.alpha, rb, h["Lambda_U"], h["mu_U"], Zu, nthreads=8)
    V_ref = O.half_sweep(R.col_ptr, R.row_idx, _r_eff(R.col_val, rb), G(U1).astype(np.float64),
                         prob.alpha, rb, h["Lambda_V"], h["mu_V"], Zv, nthreads=8)
    return row_rel_err(U1, U_ref, MIXED_FLOOR), row_rel_err(V1, V_ref, MIXED_FLOOR)


# The FP32 arithmetic bound for the errors arith_errors leaves: (median, max)
# over rows of the per-row relative error, the max scaled by
# max(1, sqrt(n_i / 100)) for a row with n_i ratings.  Derivation: the Gram
# and right-hand side are sums of n_i products in FP32 (unit roundoff
# u = 2^-24 = 6e-8) whose rounding errors grow like sqrt(n_i); the
# factorisation and the two solves add ~K u; the solution amplifies the
# relative error of P and b by cond(P), which is ~10..50 for these planted
# problems (prior plus alpha times the Gram of unit-variance rows).  With
# n_i ~ 100 that gives a typical relative error of a few u cond(P) ~ 1e-7 to
# 1e-6 and a worst row ~ 10x that.  BF16 mode also carries r - rbar as two
# BF16 parts (to ~2^-18 each) in the right-hand side of the one-wavefront and
# four-wavefront kernels: relative ~2e-6 on a sum of terms of random sign,
# more on a row whose sum cancels (up to 10x at the error floor).  Measured
# over every mixed GPU test (medians, maxima of the scaled errors): FP32
# 1e-7..2e-7 and <= 1e-6; BF16 2e-7..1.2e-6 and <= 3.4e-6 except K = 1
# (1.6e-5, a scalar row whose right-hand side cancels).
ARITH_TOL = {"fp32": (5e-7, 5e-6), "bf16": (2e-6, 3e-5)}


# One mixed sweep against the plain FP64 oracle, inputs rounded as the
# kernels round them (median, max as for ARITH_TOL).  FP32: the inputs are
# exact in FP32 except the ratings (rounded by 2^-24 relative), so the
# arithmetic bound.  BF16: every gathered entry is rounded by up to 2^-9
# relative (4e-3 between two BF16 neighbours, 2e-3 after rounding), which the
# Gram and the right-hand side carry and cond(P) amplifies.  Measured: BF16
# medians 8e-5..9e-4, maxima <= 1.8e-3.
MIXED_TOL = {"fp32": ARITH_TOL["fp32"], "bf16": (3e-3, 2e-2)}


def within(err, counts, tol, factor=1.0):
    """With e_i = err_i / max(1, sqrt(n_i / 100)) for a row of n_i ratings:
    median(e) <= factor tol[0] and max(e) <= factor tol[1]."""
    med, mx = tol
    e = np.asarray(err) / np.maximum(1.0, np.sqrt(np.asarray(counts, np.float64) / 100.0))
    return np.median(e) <= factor * med and np.all(e <= factor * mx)


def arith_bound_ok(err, counts, precision):
    return within(err, counts, ARITH_TOL[precision])


def check_arith(prob, s, tape, precision, what="", rows=None):
    eu, ev = arith_errors(prob, s, tape, precision)
    cu, cv = prob.R.row_counts(), prob.R.col_counts()
    if rows is not None:
        eu, cu = eu[rows], cu[rows]
    print(f"ARITH {precision} K={prob.K} {what}: U median {np.median(eu):.2e} max {eu.max():.2e}; "
          f"V median {np.median(ev):.2e} max {ev.max():.2e}", flush=True)
    assert arith_bound_ok(eu, cu, precision)
    assert arith_bound_ok(ev, cv, precision)
    return eu, ev
