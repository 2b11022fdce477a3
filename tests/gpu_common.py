"""Helpers shared by the GPU tests: build a sampler for a synth.Problem and
compare against the oracle."""
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


def row_rel_err(A, B):
    """Per-row ||A_i - B_i|| / max(||B_i||, 1e-3 rms(B))."""
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    rms = np.sqrt(np.mean(B * B)) if B.size else 1.0
    den = np.maximum(np.linalg.norm(B, axis=1), 1e-3 * rms)
    return np.linalg.norm(A - B, axis=1) / den


def tape_for(prob, n_sweeps, seed=7):
    return synth.make_tape(np.random.default_rng(seed), n_sweeps, prob.M, prob.N, prob.K, prob.nu0)
