"""The algebra behind the rank-one row kernels, checked on the CPU against
direct factorisations (numpy, FP64).

A row with ratings v_1..v_m has the precision P = Lambda + alpha sum_t v_t v_t^T.
With L0 = chol(Lambda), chol(P) is reached by m rank-one updates (the
rank-one update the paper recommends for items with few ratings, Section 3.1):

* Givens form: for each column k, r = sqrt(L_kk^2 + w_k^2), c = L_kk / r,
  s = w_k / r, rows i >= k map (L_ik, w_i) to (c L_ik + s w_i, c w_i - s L_ik);
* closed form for one rating: chol(L0 L0^T + w w^T) = L0 chol(I + p p^T) with
  p = L0^{-1} w, and I + p p^T = U D U^T with t_j = 1 + sum_{m<=j} p_m^2,
  D = diag(t_j / t_{j-1}), U_ij = p_i p_j / t_j (i > j).  Solves with U and
  U^T reduce to running sums.

These are the formulas the kernels evaluate in FP32; here they are pinned in
FP64 against numpy's Cholesky and solves.
"""
import numpy as np
import pytest


def _spd(rng, K):
    A = rng.standard_normal((K, K + 3))
    return A @ A.T / K + 0.1 * np.eye(K)


def givens_update(L, w):
    L = L.copy()
    w = w.copy()
    K = L.shape[0]
    for k in range(K):
        r = np.hypot(L[k, k], w[k])
        c, s = L[k, k] / r, w[k] / r
        col = L[k:, k].copy()
        L[k:, k] = c * col + s * w[k:]
        w[k:] = c * w[k:] - s * col
    return L


def closed_form_factor(p):
    """chol(I + p p^T) from the LDL^T closed form."""
    K = p.size
    t = 1.0 + np.cumsum(p * p)
    tprev = np.concatenate([[1.0], t[:-1]])
    U = np.eye(K)
    for j in range(K):
        U[j + 1:, j] = p[j + 1:] * p[j] / t[j]
    return U * np.sqrt(t / tprev)[None, :]


def running_sum_sample(L0, p, c, z):
    """x = L0^{-T} Lt^{-T} (Lt^{-1} c + z) with Lt = chol(I + p p^T), by the
    prefix and suffix sums of the one-lane kernel."""
    K = p.size
    y = np.zeros(K)
    t_prev, S = 1.0, 0.0
    rs = np.zeros(K)
    for i in range(K):
        t = t_prev + p[i] ** 2
        y[i] = (c[i] - p[i] * S / t_prev) * np.sqrt(t_prev / t)
        S += p[i] * c[i]
        rs[i] = 1.0 / np.sqrt(t)
        t_prev = t
    g = y + z
    u = np.zeros(K)
    Q = 0.0
    for j in range(K - 1, -1, -1):
        rp = rs[j - 1] if j > 0 else 1.0
        h = g[j] * rs[j] / rp
        u[j] = h - p[j] * Q
        Q += p[j] * h * rp * rp
    return np.linalg.solve(L0.T, u)


@pytest.mark.parametrize("K,m", [(1, 1), (5, 1), (32, 1), (32, 3), (64, 2)])
def test_givens_updates_give_the_cholesky_factor(K, m):
    rng = np.random.default_rng(K * 10 + m)
    Lam = _spd(rng, K)
    alpha = 2.0
    V = rng.standard_normal((m, K))
    L = np.linalg.cholesky(Lam)
    for v in V:
        L = givens_update(L, np.sqrt(alpha) * v)
    P = Lam + alpha * V.T @ V
    ref = np.linalg.cholesky(P)
    assert np.allclose(np.triu(L, 1), 0.0)
    assert np.all(np.diag(L) > 0)
    np.testing.assert_allclose(L, ref, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("K", [1, 2, 10, 32])
def test_closed_form_factor_of_identity_plus_rank_one(K):
    rng = np.random.default_rng(K)
    p = rng.standard_normal(K) * 3.0
    Lt = closed_form_factor(p)
    np.testing.assert_allclose(Lt, np.linalg.cholesky(np.eye(K) + np.outer(p, p)), rtol=1e-12, atol=1e-13)
    # and L0 Lt is chol(L0 L0^T + w w^T)
    L0 = np.linalg.cholesky(_spd(rng, K))
    w = L0 @ p
    np.testing.assert_allclose(L0 @ Lt, np.linalg.cholesky(L0 @ L0.T + np.outer(w, w)), rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("K,scale", [(10, 1.0), (32, 1.0), (32, 30.0)])
def test_one_rating_sample_by_running_sums(K, scale):
    """The one-lane kernel's sample equals the direct Cholesky sample of the
    row conditional for the same normals."""
    rng = np.random.default_rng(K + int(scale))
    Lam = _spd(rng, K)
    mu = rng.standard_normal(K)
    alpha, r = 2.0, rng.standard_normal()
    v = scale * rng.standard_normal(K)
    z = rng.standard_normal(K)
    P = Lam + alpha * np.outer(v, v)
    b = Lam @ mu + alpha * r * v
    L = np.linalg.cholesky(P)
    x_ref = np.linalg.solve(L.T, np.linalg.solve(L, b) + z)
    L0 = np.linalg.cholesky(Lam)
    p = np.linalg.solve(L0, np.sqrt(alpha) * v)
    c = L0.T @ mu + np.sqrt(alpha) * r * p  # L0^{-1} b
    x = running_sum_sample(L0, p, c, z)
    np.testing.assert_allclose(x, x_ref, rtol=1e-9, atol=1e-10 * np.abs(x_ref).max())
    # pivots of chol(P): L0_kk^2 t_k / t_{k-1}
    t = 1.0 + np.cumsum(p * p)
    piv = np.diag(L0) ** 2 * t / np.concatenate([[1.0], t[:-1]])
    np.testing.assert_allclose(piv, np.diag(L) ** 2, rtol=1e-10)


def test_empty_row_is_the_prior_draw():
    """With p = 0 the one-lane formulas reduce to x = L0^{-T}(L0^T mu + z)."""
    rng = np.random.default_rng(7)
    K = 12
    L0 = np.linalg.cholesky(_spd(rng, K))
    mu, z = rng.standard_normal(K), rng.standard_normal(K)
    x = running_sum_sample(L0, np.zeros(K), L0.T @ mu, z)
    np.testing.assert_allclose(x, mu + np.linalg.solve(L0.T, z), rtol=1e-12, atol=1e-12)
