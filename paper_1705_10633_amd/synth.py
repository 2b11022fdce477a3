"""Seeded synthetic workloads for the BPMF Gibbs row update.

This module makes inputs only: rating matrices with the shapes, count laws and
value maps of the paper's benchmarks (ChEMBL IC50 subset, MovieLens ml-20m and
Netflix, described in the Validation section, "Benchmarks"), planted low-rank
factors, initial states, the standard-normal / chi-square draw tape, and
fold-in serving requests.  It holds none of the sampler's arithmetic: it is the
one module that both the CPU oracle (tests) and the HIP library (product) read
inputs from.

Every generator takes a seed; a config's seed is split with
``numpy.random.SeedSequence.spawn`` into independent streams so that, e.g.,
changing the test-set size does not change the training ratings.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

STREAMS = ("factors", "counts", "columns", "values", "test", "init", "tape")


def streams(seed: int) -> dict:
    kids = np.random.SeedSequence(seed).spawn(len(STREAMS))
    return {name: np.random.Generator(np.random.PCG64(k)) for name, k in zip(STREAMS, kids)}


# ----------------------------------------------------------------------------
# Sparse rating matrix in both orientations
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Ratings:
    M: int
    N: int
    row_ptr: np.ndarray  # int64 [M+1]
    col_idx: np.ndarray  # int32 [nnz], sorted within each row
    row_val: np.ndarray  # float64 [nnz]
    col_ptr: np.ndarray  # int64 [N+1]
    row_idx: np.ndarray  # int32 [nnz], sorted within each column
    col_val: np.ndarray  # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def row_counts(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def col_counts(self) -> np.ndarray:
        return np.diff(self.col_ptr)


def from_coo(M: int, N: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> Ratings:
    """Build CSR and CSC from distinct (row, col, value) triples."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    key = rows * N + cols
    order = np.argsort(key, kind="stable")
    ks = key[order]
    if ks.size > 1 and np.any(ks[1:] == ks[:-1]):
        raise ValueError("duplicate (row, col) positions")
    r_sorted = rows[order]
    row_ptr = np.zeros(M + 1, dtype=np.int64)
    np.cumsum(np.bincount(r_sorted, minlength=M), out=row_ptr[1:])
    col_idx = cols[order].astype(np.int32)
    row_val = vals[order]
    ckey = cols * M + rows
    corder = np.argsort(ckey, kind="stable")
    c_sorted = cols[corder]
    col_ptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(np.bincount(c_sorted, minlength=N), out=col_ptr[1:])
    row_idx = rows[corder].astype(np.int32)
    col_val = vals[corder]
    return Ratings(M, N, row_ptr, col_idx, row_val, col_ptr, row_idx, col_val)


# ----------------------------------------------------------------------------
# Count laws
# ----------------------------------------------------------------------------
def _fix_total(counts: np.ndarray, total: int, lo: int, hi: int, rng) -> np.ndarray:
    """Add or remove single ratings on random rows (within [lo, hi]) to hit `total`."""
    counts = counts.copy()
    diff = int(total - counts.sum())
    while diff != 0:
        if diff > 0:
            cand = np.nonzero(counts < hi)[0]
        else:
            cand = np.nonzero(counts > lo)[0]
        if cand.size == 0:
            raise ValueError("cannot reach the requested total")
        pick = rng.choice(cand, size=min(abs(diff), cand.size), replace=False)
        counts[pick] += 1 if diff > 0 else -1
        diff = int(total - counts.sum())
    return counts


def zipf_rank_counts(M: int, s: float, cap: int, total: int, rng) -> np.ndarray:
    """Rank-frequency Zipf law: count(rank r) = clip(round(C r^-s), 1, cap).

    C is found by bisection so the counts sum to `total` (then trimmed by
    single ratings); the ranks are randomly permuted onto the rows.
    """
    r = np.arange(1, M + 1, dtype=np.float64)
    base = r ** (-s)

    def tot(C):
        return int(np.clip(np.rint(C * base), 1, cap).sum())

    lo, hi = 0.0, 1.0
    while tot(hi) < total:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if tot(mid) < total:
            lo = mid
        else:
            hi = mid
    counts = np.clip(np.rint(hi * base), 1, cap).astype(np.int64)
    counts = _fix_total(counts, total, 1, cap, rng)
    return rng.permutation(counts)


def lognormal_counts(M: int, sigma: float, cap: int, total: int, rng,
                     mu: Optional[float] = None) -> tuple:
    """Per-row counts clip(rint(exp(mu + sigma z)), 1, cap), z ~ N(0,1) i.i.d.

    With mu=None the location is fitted by bisection on the realised draws so
    that the counts sum to `total`.  Returns (counts, mu).
    """
    z = rng.standard_normal(M)

    def counts_for(m):
        return np.clip(np.rint(np.exp(m + sigma * z)), 1, cap).astype(np.int64)

    if mu is None:
        lo, hi = -10.0, 20.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if counts_for(mid).sum() < total:
                lo = mid
            else:
                hi = mid
        mu = hi
        counts = _fix_total(counts_for(mu), total, 1, cap, rng)
    else:
        counts = counts_for(mu)
    return counts, mu


def distinct_columns(counts: np.ndarray, N: int, rng) -> np.ndarray:
    """For each row, `counts[i]` distinct columns, uniform without replacement.

    Returns int64 columns in row-major order, sorted within each row.
    """
    counts = np.asarray(counts, dtype=np.int64)
    if np.any(counts > N):
        raise ValueError("a row asks for more columns than exist")
    M = counts.size
    nnz = int(counts.sum())
    ptr = np.zeros(M + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    rows = np.repeat(np.arange(M, dtype=np.int64), counts)
    cols = rng.integers(0, N, size=nnz, dtype=np.int64)
    dense = np.nonzero(counts > N // 4)[0]
    for r in dense:
        cols[ptr[r]:ptr[r + 1]] = rng.choice(N, size=int(counts[r]), replace=False)
    active = np.ones(nnz, dtype=bool)
    for r in dense:
        active[ptr[r]:ptr[r + 1]] = False
    # resample duplicates among the sparse rows until every row is duplicate-free
    sel = np.nonzero(active)[0]
    while sel.size:
        key = rows[sel] * N + cols[sel]
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup_sorted = np.zeros(sel.size, dtype=bool)
        dup_sorted[1:] = ks[1:] == ks[:-1]
        dup = sel[order[dup_sorted]]
        if dup.size == 0:
            break
        cols[dup] = rng.integers(0, N, size=dup.size, dtype=np.int64)
        # only rows that had a duplicate need re-checking
        bad_rows = np.unique(rows[dup])
        mask = np.zeros(M, dtype=bool)
        mask[bad_rows] = True
        sel = sel[mask[rows[sel]]]
    key = rows * N + cols
    key.sort()
    return key - rows * N


# ----------------------------------------------------------------------------
# Planted models
# ----------------------------------------------------------------------------
def planted_dot(U: np.ndarray, V: np.ndarray, rows: np.ndarray, cols: np.ndarray,
                chunk: int = 1 << 20) -> np.ndarray:
    """u_i . v_j for each (i, j) pair, in float64, chunked to bound memory."""
    out = np.empty(rows.size, dtype=np.float64)
    for a in range(0, rows.size, chunk):
        b = min(rows.size, a + chunk)
        out[a:b] = np.einsum("ij,ij->i", U[rows[a:b]], V[cols[a:b]])
    return out


def unobserved_positions(M: int, N: int, n: int, train_rows: np.ndarray,
                         train_cols: np.ndarray, rng) -> tuple:
    """n distinct uniform (i, j) positions not in the training set."""
    train_key = np.sort(train_rows.astype(np.int64) * N + train_cols.astype(np.int64))
    if M * N - train_key.size < n:
        raise ValueError("not enough unobserved positions")
    got = np.empty(0, dtype=np.int64)
    while got.size < n:
        need = n - got.size
        cand = rng.integers(0, M * N, size=2 * need + 16, dtype=np.int64)
        pos = np.searchsorted(train_key, cand)
        pos = np.minimum(pos, train_key.size - 1)
        fresh = cand[train_key[pos] != cand] if train_key.size else cand
        got = np.unique(np.concatenate([got, fresh]))
        if got.size > n:
            got = rng.permutation(got)[:n]
    got = rng.permutation(got)
    return got // N, got % N


@dataclasses.dataclass
class Problem:
    """One BPMF run: ratings, priors, initial state and a held-out test set."""
    name: str
    R: Ratings
    K: int
    alpha: float
    mu0: np.ndarray
    beta0: float
    nu0: float
    W0: np.ndarray
    n_sweeps: int
    burnin: int
    U0: np.ndarray
    V0: np.ndarray
    test_rows: np.ndarray
    test_cols: np.ndarray
    test_vals: np.ndarray
    seed: int
    mean_rating: float
    note: str = ""

    @property
    def M(self):
        return self.R.M

    @property
    def N(self):
        return self.R.N


def _finish(name, M, N, K, rows, cols, vals, test_rows, test_cols, test_vals, st, seed,
            n_sweeps, burnin, note="", alpha=2.0, beta0=2.0, nu0=None):
    R = from_coo(M, N, rows, cols, vals)
    nu0 = float(K) if nu0 is None else float(nu0)
    U0 = 0.1 * st["init"].standard_normal((M, K))
    V0 = 0.1 * st["init"].standard_normal((N, K))
    mean_rating = float(np.mean(R.row_val)) if R.nnz else 0.0
    return Problem(name, R, K, alpha, np.zeros(K), beta0, nu0, np.eye(K), n_sweeps, burnin,
                   U0, V0, test_rows.astype(np.int32), test_cols.astype(np.int32),
                   np.asarray(test_vals, dtype=np.float64), seed, mean_rating, note)


def uniform_planted(M=1000, N=500, K=10, nnz=20000, noise=0.5, seed=101, n_sweeps=20,
                    burnin=0, test_frac=0.1, rank=None) -> Problem:
    """Plain BPMF workload: distinct uniform positions, planted U V^T + Gaussian noise.

    Planted factor entries have variance 1/sqrt(rank) so that u.v has unit variance.
    """
    rank = K if rank is None else rank
    st = streams(seed)
    sd = (1.0 / math.sqrt(rank)) ** 0.5
    Up = sd * st["factors"].standard_normal((M, rank))
    Vp = sd * st["factors"].standard_normal((N, rank))
    key = st["columns"].choice(M * N, size=nnz, replace=False)
    rows, cols = key // N, key % N
    vals = planted_dot(Up, Vp, rows, cols) + noise * st["values"].standard_normal(nnz)
    ntest = int(round(test_frac * nnz))
    tr, tc = unobserved_positions(M, N, ntest, rows, cols, st["test"])
    tv = planted_dot(Up, Vp, tr, tc) + noise * st["test"].standard_normal(ntest)
    return _finish("uniform_planted", M, N, K, rows, cols, vals, tr, tc, tv, st, seed,
                   n_sweeps, burnin)


def _rows_from_counts(counts):
    return np.repeat(np.arange(counts.size, dtype=np.int64), counts)


def chembl_like(M=483500, N=5775, nnz=1023952, K=32, s=1.3, seed=102, n_sweeps=50,
                burnin=25, test_frac=0.1) -> Problem:
    """ChEMBL-IC50-shaped: rank-frequency Zipf row counts, planted rank-K + N(0,1)."""
    st = streams(seed)
    counts = zipf_rank_counts(M, s, N, nnz, st["counts"])
    rows = _rows_from_counts(counts)
    cols = distinct_columns(counts, N, st["columns"])
    sd = (1.0 / math.sqrt(K)) ** 0.5
    Up = sd * st["factors"].standard_normal((M, K))
    Vp = sd * st["factors"].standard_normal((N, K))
    vals = planted_dot(Up, Vp, rows, cols) + st["values"].standard_normal(rows.size)
    ntest = int(round(test_frac * nnz))
    tr, tc = unobserved_positions(M, N, ntest, rows, cols, st["test"])
    tv = planted_dot(Up, Vp, tr, tc) + st["test"].standard_normal(ntest)
    return _finish("chembl_like", M, N, K, rows, cols, vals, tr, tc, tv, st, seed,
                   n_sweeps, burnin)


def movielens_like(M=138493, N=26744, nnz=20_000_000, K=64, sigma=1.2, cap=9000, seed=103,
                   n_sweeps=20, burnin=10, test_frac=0.1, mu=None) -> Problem:
    """MovieLens-20M-shaped: log-normal row counts, half-star ratings from a planted rank-K model.

    r = clip(0.5 rint(2 (3.5 + u.v)), 0.5, 5.0).
    """
    st = streams(seed)
    cap = min(cap, N)
    counts, mu_fit = lognormal_counts(M, sigma, cap, nnz, st["counts"], mu)
    rows = _rows_from_counts(counts)
    cols = distinct_columns(counts, N, st["columns"])
    sd = (1.0 / math.sqrt(K)) ** 0.5
    Up = sd * st["factors"].standard_normal((M, K))
    Vp = sd * st["factors"].standard_normal((N, K))

    def quant(x):
        return np.clip(0.5 * np.rint(2.0 * (3.5 + x)), 0.5, 5.0)

    vals = quant(planted_dot(Up, Vp, rows, cols))
    ntest = int(round(test_frac * rows.size))
    tr, tc = unobserved_positions(M, N, ntest, rows, cols, st["test"])
    tv = quant(planted_dot(Up, Vp, tr, tc))
    return _finish("movielens_like", M, N, K, rows, cols, vals, tr, tc, tv, st, seed,
                   n_sweeps, burnin, note=f"lognormal location fitted mu={mu_fit:.4f}")


def netflix_like(M=480189, N=17770, nnz=100_000_000, K=128, s=1.1, cap=17000, seed=104,
                 n_sweeps=5, burnin=2, test_frac=0.1) -> Problem:
    """Netflix-shaped: rank-frequency Zipf row counts, integer 1..5 ratings, planted rank-K."""
    st = streams(seed)
    cap = min(cap, N)
    counts = zipf_rank_counts(M, s, cap, nnz, st["counts"])
    rows = _rows_from_counts(counts)
    cols = distinct_columns(counts, N, st["columns"])
    sd = (1.0 / math.sqrt(K)) ** 0.5
    Up = sd * st["factors"].standard_normal((M, K))
    Vp = sd * st["factors"].standard_normal((N, K))

    def quant(x):
        return np.clip(np.rint(3.0 + x), 1.0, 5.0)

    vals = quant(planted_dot(Up, Vp, rows, cols))
    ntest = int(round(test_frac * rows.size))
    tr, tc = unobserved_positions(M, N, ntest, rows, cols, st["test"])
    tv = quant(planted_dot(Up, Vp, tr, tc))
    return _finish("netflix_like", M, N, K, rows, cols, vals, tr, tc, tv, st, seed,
                   n_sweeps, burnin)


# ----------------------------------------------------------------------------
# Draw tape: the sampler's random numbers passed in as an input
# ----------------------------------------------------------------------------
def tape_block_len(n_rows: int, K: int) -> int:
    """Doubles consumed by one half-sweep over `n_rows` rows."""
    return K + K * (K - 1) // 2 + K + n_rows * K


def tape_sweep_len(M: int, N: int, K: int) -> int:
    return tape_block_len(M, K) + tape_block_len(N, K)


def make_tape(rng, n_sweeps: int, M: int, N: int, K: int, nu0: float) -> np.ndarray:
    """Host-generated draws for `n_sweeps` sweeps, users' half first.

    Per half-sweep over n rows: K chi-square draws with n + nu0 - k degrees of
    freedom (k = 0..K-1), K(K-1)/2 standard normals for the strict lower part of
    the Bartlett factor (row-major), K standard normals for the mean, and n*K
    standard normals for the rows (row-major).
    """
    parts = []
    for _ in range(n_sweeps):
        for n in (M, N):
            df = nu0 + n - np.arange(K, dtype=np.float64)
            parts.append(rng.chisquare(df))
            parts.append(rng.standard_normal(K * (K - 1) // 2))
            parts.append(rng.standard_normal(K))
            parts.append(rng.standard_normal(n * K))
    return np.concatenate(parts) if parts else np.zeros(0)


# ----------------------------------------------------------------------------
# Fold-in serving workload
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class FoldinModel:
    S: int
    N: int
    K: int
    alpha: float
    mean_rating: float
    Vs: np.ndarray        # [S, N, K] float32
    Lambda: np.ndarray    # [S, K, K] float64, SPD
    mu: np.ndarray        # [S, K] float64


def foldin_model(S=16, N=20000, K=64, alpha=2.0, seed=105, mean_rating=3.0) -> FoldinModel:
    """S posterior-like samples: a planted V plus per-sample jitter, and SPD user hypers."""
    st = streams(seed)
    sd = (1.0 / math.sqrt(K)) ** 0.5
    V = sd * st["factors"].standard_normal((N, K))
    Vs = (V[None] + 0.05 * st["factors"].standard_normal((S, N, K))).astype(np.float32)
    Lam = np.empty((S, K, K))
    mu = np.empty((S, K))
    for s in range(S):
        A = st["init"].standard_normal((K, 2 * K)) / math.sqrt(2 * K)
        Lam[s] = 2.0 * math.sqrt(K) * (A @ A.T + np.eye(K))
        mu[s] = 0.05 * st["init"].standard_normal(K)
    return FoldinModel(S, N, K, alpha, mean_rating, Vs, Lam, mu)


@dataclasses.dataclass
class FoldinRequests:
    n: int
    ptr: np.ndarray       # int64 [n+1] into cols/vals
    cols: np.ndarray      # int32
    vals: np.ndarray      # float32
    q_ptr: np.ndarray     # int64 [n+1] into q_cols
    q_cols: np.ndarray    # int32
    arrival: np.ndarray   # float64 seconds


def foldin_requests(n: int, N: int, seed=105, mu=3.0, sigma=1.5, cap=5000, Q=100,
                    rate=None, stream_offset=0, rating_mean=3.0) -> FoldinRequests:
    """New-user requests: log-normal rating counts over distinct random columns,
    ratings N(3, 1), Q query columns among the unrated ones, Poisson arrivals."""
    ss = np.random.SeedSequence([seed, 7, stream_offset])
    rng = np.random.Generator(np.random.PCG64(ss))
    cap = min(cap, N - Q)
    counts = np.clip(np.rint(np.exp(mu + sigma * rng.standard_normal(n))), 1, cap).astype(np.int64)
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    cols = np.empty(int(ptr[-1]), dtype=np.int32)
    q_ptr = np.arange(n + 1, dtype=np.int64) * Q
    q_cols = np.empty(n * Q, dtype=np.int32)
    for i in range(n):
        pick = rng.choice(N, size=int(counts[i]) + Q, replace=False)
        cols[ptr[i]:ptr[i + 1]] = np.sort(pick[:counts[i]])
        q_cols[i * Q:(i + 1) * Q] = pick[counts[i]:]
    vals = (rating_mean + rng.standard_normal(cols.size)).astype(np.float32)
    if rate is None:
        arrival = np.zeros(n)
    else:
        arrival = np.cumsum(rng.exponential(1.0 / rate, size=n))
    return FoldinRequests(n, ptr, cols, vals, q_ptr, q_cols, arrival)


def relabel_users_by_count(prob: Problem) -> Problem:
    """The same problem with the users renumbered in descending rating count
    (ties by the old index): the reordering of R's rows for locality that
    the paper applies before its runs (Section 3.1), here so that the users
    gathered most often on the movies' side share pages and cache sets.  U0
    and the held-out pairs are permuted with them; the posterior is the same
    up to the relabelling."""
    R = prob.R
    counts = R.row_counts()
    new_of_old = np.empty(R.M, np.int64)
    new_of_old[np.argsort(-counts, kind="stable")] = np.arange(R.M)
    rows = new_of_old[np.repeat(np.arange(R.M), counts)]
    R2 = from_coo(R.M, R.N, rows, R.col_idx.astype(np.int64), R.row_val)
    p = Problem(**{**prob.__dict__})
    p.R = R2
    U0 = np.empty_like(prob.U0)
    U0[new_of_old] = prob.U0
    p.U0 = U0
    p.test_rows = new_of_old[prob.test_rows].astype(np.int32)
    p.name = prob.name + "_users_by_count"
    return p


CONFIGS = {
    "uniform_planted": uniform_planted,
    "chembl_like": chembl_like,
    "movielens_like": movielens_like,
    "netflix_like": netflix_like,
}
