"""ctypes wrapper for the FP64 CPU oracle (bpmf_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark; never by the product library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "bpmf_oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C, -O2, pthreads)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-Wno-unused-variable", "-o", tmp, SRC, "-lm", "-lpthread"])
        os.replace(tmp, LIB)
    return LIB


def build_sanitized(out: str) -> str:
    """Compile the oracle with AddressSanitizer and UndefinedBehaviorSanitizer
    (gcc, host code only) for the sanitizer test run; load it through the
    BPMF_ORACLE_LIB environment variable with libasan preloaded."""
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wno-unused-variable",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-o", out, SRC, "-lm", "-lpthread"])
    return out


def lib():
    global _lib
    if _lib is None:
        override = os.environ.get("BPMF_ORACLE_LIB")
        if override:
            _lib = C.CDLL(override)
        else:
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                build(force=True)
            _lib = C.CDLL(LIB)
        _declare(_lib)
    return _lib


P = C.c_void_p
I64 = C.c_int64
I32 = C.c_int
F64 = C.c_double
U32 = C.c_uint32
U64 = C.c_uint64


def _declare(L):
    L.oracle_cholesky.argtypes = [I32, P, P]
    L.oracle_spd_inverse.argtypes = [I32, P, P]
    L.oracle_row_update.argtypes = [I32, I64, P, P, P, F64, F64, P, P, P, P, P]
    L.oracle_half_sweep.argtypes = [I64, I32, P, P, P, P, F64, F64, P, P, P, P, I32]
    L.oracle_nw_posterior.argtypes = [I32, I64, P, P, F64, F64, P, P, P, P, P]
    L.oracle_nw.argtypes = [I32, I64, P, P, F64, F64, P, P, P, P, P, P]
    L.oracle_tape_block_len.argtypes = [I64, I32]
    L.oracle_tape_block_len.restype = I64
    L.oracle_gibbs.argtypes = [I64, I64, I32, P, P, P, P, P, P, F64, F64, P, F64, F64, P, P,
                               I32, I32, I32, P, P, I64, P, P, P, P, P, I32]
    L.oracle_predict.argtypes = [I32, I64, P, P, P, P, F64, P]
    L.oracle_predict.restype = None
    L.oracle_foldin.argtypes = [I32, I64, I32, F64, F64, P, P, P, I64, P, P, P, P, P, P, P]
    L.oracle_philox4x32_10.argtypes = [P, P, P]
    L.oracle_philox4x32_10.restype = None
    L.oracle_philox_row_normals.argtypes = [U64, U32, I64, I32, P]
    L.oracle_philox_row_normals.restype = None
    L.oracle_philox_block.argtypes = [U64, U32, I64, I32, F64, P]
    L.oracle_philox_block.restype = None
    L.oracle_philox_tape.argtypes = [U64, I32, I32, I64, I64, I32, F64, P]
    L.oracle_philox_tape.restype = None
    L.oracle_gamma_draws.argtypes = [U64, U32, F64, I64, P]
    L.oracle_gamma_draws.restype = None
    L.oracle_stream_normals.argtypes = [U64, U32, U32, I64, P]
    L.oracle_stream_normals.restype = None


class OracleError(RuntimeError):
    pass


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _p(a):
    return a.ctypes.data if a is not None else None


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc} ({'not SPD' if rc == 1 else 'error'})")


def cholesky(A):
    A = _f64(A)
    n = A.shape[0]
    L = np.empty_like(A)
    _check(lib().oracle_cholesky(n, _p(A), _p(L)), "cholesky")
    return L


def spd_inverse(A):
    A = _f64(A)
    out = np.empty_like(A)
    _check(lib().oracle_spd_inverse(A.shape[0], _p(A), _p(out)), "spd_inverse")
    return out


def row_update(other, idx, val, alpha, rbar, Lambda, mu, z):
    """One row's draw and conditional mean: returns (draw, mean)."""
    other = _f64(other)
    K = other.shape[1]
    idx = _i32(idx)
    val = _f64(val)
    Lambda = _f64(Lambda)
    Lmu = _f64(Lambda @ _f64(mu))
    z = _f64(z)
    out = np.empty(K)
    mean = np.empty(K)
    _check(lib().oracle_row_update(K, idx.size, _p(idx), _p(val), _p(other), alpha, rbar,
                                   _p(Lambda), _p(Lmu), _p(z), _p(out), _p(mean)), "row_update")
    return out, mean


def half_sweep(ptr, idx, val, other, alpha, rbar, Lambda, mu, Z, nthreads=1):
    ptr = _i64(ptr)
    idx = _i32(idx)
    val = _f64(val)
    other = _f64(other)
    K = other.shape[1]
    n = ptr.size - 1
    Lambda = _f64(Lambda)
    mu = _f64(mu)
    Z = _f64(Z).reshape(n, K)
    X = np.empty((n, K))
    _check(lib().oracle_half_sweep(n, K, _p(ptr), _p(idx), _p(val), _p(other), alpha, rbar,
                                   _p(Lambda), _p(mu), _p(Z), _p(X), nthreads), "half_sweep")
    return X


def nw_posterior(X, mu0, beta0, nu0, W0):
    X = _f64(X)
    n, K = X.shape
    mu0 = _f64(mu0)
    W0 = _f64(W0)
    mus = np.empty(K)
    bs = C.c_double()
    ns = C.c_double()
    Ws = np.empty((K, K))
    _check(lib().oracle_nw_posterior(K, n, _p(X), _p(mu0), beta0, nu0, _p(W0), _p(mus),
                                     C.byref(bs), C.byref(ns), _p(Ws)), "nw_posterior")
    return mus, bs.value, ns.value, Ws


def nw(X, mu0, beta0, nu0, W0, chi2, zb, zm):
    X = _f64(X)
    n, K = X.shape
    mu0 = _f64(mu0)
    W0 = _f64(W0)
    chi2 = _f64(chi2)
    zb = _f64(zb) if K > 1 else np.zeros(1)
    zm = _f64(zm)
    Lam = np.empty((K, K))
    mu = np.empty(K)
    _check(lib().oracle_nw(K, n, _p(X), _p(mu0), beta0, nu0, _p(W0), _p(chi2), _p(zb), _p(zm),
                           _p(Lam), _p(mu)), "nw")
    return Lam, mu


def tape_block_len(n_rows, K):
    return int(lib().oracle_tape_block_len(n_rows, K))


def gibbs(prob, tape, n_sweeps=None, U=None, V=None, sweep0=0, burnin=None, nthreads=1,
          rbar=None, pred_sum=None, pred_cnt=0, want_hyper=False):
    """Run the whole sampler on a synth.Problem.  Returns a dict with U, V,
    pred_sum, pred_cnt, pred_mean, rmse (and hyper if asked)."""
    R = prob.R
    K = prob.K
    n_sweeps = prob.n_sweeps if n_sweeps is None else n_sweeps
    burnin = prob.burnin if burnin is None else burnin
    rbar = prob.mean_rating if rbar is None else rbar
    U = _f64(prob.U0 if U is None else U).copy()
    V = _f64(prob.V0 if V is None else V).copy()
    tape = _f64(tape)
    need = n_sweeps * (tape_block_len(R.M, K) + tape_block_len(R.N, K))
    if tape.size < need:
        raise ValueError(f"tape too short: {tape.size} < {need}")
    rp, ci, rv = _i64(R.row_ptr), _i32(R.col_idx), _f64(R.row_val)
    cp, ri, cv = _i64(R.col_ptr), _i32(R.row_idx), _f64(R.col_val)
    tr, tc = _i32(prob.test_rows), _i32(prob.test_cols)
    ps = np.zeros(tr.size) if pred_sum is None else _f64(pred_sum).copy()
    cnt = C.c_int64(pred_cnt)
    hyper = np.empty(2 * K * K + 2 * K) if want_hyper else None
    mu0, W0 = _f64(prob.mu0), _f64(prob.W0)
    _check(lib().oracle_gibbs(R.M, R.N, K, _p(rp), _p(ci), _p(rv), _p(cp), _p(ri), _p(cv),
                              prob.alpha, rbar, _p(mu0), prob.beta0, prob.nu0, _p(W0),
                              _p(tape), n_sweeps, sweep0, burnin, _p(U), _p(V), tr.size,
                              _p(tr), _p(tc), _p(ps), C.byref(cnt), _p(hyper), nthreads), "gibbs")
    out = {"U": U, "V": V, "pred_sum": ps, "pred_cnt": cnt.value}
    if cnt.value > 0 and tr.size:
        out["pred_mean"] = ps / cnt.value
        out["rmse"] = float(np.sqrt(np.mean((out["pred_mean"] - prob.test_vals) ** 2)))
    if want_hyper:
        out["hyper"] = {"Lambda_U": hyper[:K * K].reshape(K, K).copy(),
                        "mu_U": hyper[K * K:K * K + K].copy(),
                        "Lambda_V": hyper[K * K + K:2 * K * K + K].reshape(K, K).copy(),
                        "mu_V": hyper[2 * K * K + K:].copy()}
    return out


def predict(U, V, rows, cols, rbar):
    U, V = _f64(U), _f64(V)
    rows, cols = _i32(rows), _i32(cols)
    out = np.empty(rows.size)
    lib().oracle_predict(U.shape[1], rows.size, _p(rows), _p(cols), _p(U), _p(V), rbar, _p(out))
    return out


def foldin(model, req, want_mean=False):
    """Oracle fold-in for synth.FoldinModel / synth.FoldinRequests."""
    S, N, K = model.S, model.N, model.K
    Vs = _f64(model.Vs)
    Lam = _f64(model.Lambda)
    mu = _f64(model.mu)
    ptr, cols, vals = _i64(req.ptr), _i32(req.cols), _f64(req.vals)
    qp, qc = _i64(req.q_ptr), _i32(req.q_cols)
    out = np.empty(qc.size)
    mean = np.empty((req.n, S, K)) if want_mean else None
    _check(lib().oracle_foldin(S, N, K, model.alpha, model.mean_rating, _p(Vs), _p(Lam), _p(mu),
                               req.n, _p(ptr), _p(cols), _p(vals), _p(qp), _p(qc), _p(out),
                               _p(mean)), "foldin")
    return (out, mean) if want_mean else out


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def philox_row_normals(seed, h, n_rows, K):
    out = np.empty((n_rows, K))
    lib().oracle_philox_row_normals(seed, h, n_rows, K, _p(out))
    return out


def philox_block(seed, h, n_rows, K, nu0):
    out = np.empty(tape_block_len(n_rows, K))
    lib().oracle_philox_block(seed, h, n_rows, K, nu0, _p(out))
    return out


def philox_tape(seed, sweep0, n_sweeps, M, N, K, nu0):
    out = np.empty(n_sweeps * (tape_block_len(M, K) + tape_block_len(N, K)))
    lib().oracle_philox_tape(seed, sweep0, n_sweeps, M, N, K, nu0, _p(out))
    return out


def gamma_draws(seed, h, a, n):
    out = np.empty(n)
    lib().oracle_gamma_draws(seed, h, a, n, _p(out))
    return out


def stream_normals(seed, h, tag, n):
    out = np.empty(n)
    lib().oracle_stream_normals(seed, h, tag, n, _p(out))
    return out
