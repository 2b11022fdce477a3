"""Fold-in kernel against the oracle, and the continuous-batching server:
results alone == results in a mixed batch (bitwise), memory admission, and
real-time replay of a Poisson trace."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1705_10633_amd import synth

pytestmark = pytest.mark.gpu

# FP32 fold-in: the Gram, Cholesky and solves run in FP32 on FP32 samples;
# a prediction is rbar plus the average over S samples of a K-term dot
# product m_s . v_q, whose error is a few unit roundoffs (6e-8) of
# |m_s| |v_q| times cond(P) (< ~10 for these requests: prior plus alpha times
# the Gram of unit-variance rows) -> scaled bound 4e-6 (1 + |pred - rbar|).
# Measured over the fold-in tests: max 2.6e-7, median 5e-8.
FOLDIN_TOL = 4e-6


def _dev(a, dt=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    return t.to("cuda") if dt is None else t.to("cuda", dt)


def _foldin(model):
    from paper_1705_10633_amd.sampler import Foldin
    return Foldin(model.Vs, model.Lambda, model.mu, model.alpha, model.mean_rating)


def _run_direct(fm, req):
    import torch
    out = fm.run(_dev(req.ptr), _dev(req.cols), _dev(req.vals), _dev(req.q_ptr), _dev(req.q_cols))
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("K,N", [(10, 300), (33, 500), (64, 2000)])
def test_foldin_matches_oracle(K, N):
    model = synth.foldin_model(S=4, N=N, K=K, seed=K)
    req = synth.foldin_requests(40, N, seed=K, mu=3.0, sigma=1.5, cap=800, Q=7)
    fm = _foldin(model)
    got = _run_direct(fm, req)
    ref = O.foldin(model, req)
    err = np.abs(got - ref) / (1.0 + np.abs(ref - model.mean_rating))
    print(f"K={K}: max scaled err {err.max():.2e}, median {np.median(err):.2e}")
    assert err.max() <= FOLDIN_TOL


def test_foldin_empty_request_is_prior_mean():
    """A request with no ratings folds in at the prior mean mu_s."""
    model = synth.foldin_model(S=3, N=100, K=8, seed=2)
    req = synth.FoldinRequests(1, np.array([0, 0], np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32),
                               np.array([0, 5], np.int64), np.array([1, 7, 20, 50, 99], np.int32), np.zeros(1))
    got = _run_direct(_foldin(model), req)
    ref = model.mean_rating + np.mean([model.Vs[s].astype(np.float64)[req.q_cols] @ model.mu[s]
                                       for s in range(3)], axis=0)
    np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-5)


def test_server_alone_equals_mixed():
    from paper_1705_10633_amd.serving import FoldinServer
    model = synth.foldin_model(S=8, N=3000, K=64, seed=3)
    fm = _foldin(model)
    req = synth.foldin_requests(60, 3000, seed=9, Q=20)
    # each request alone, direct call
    alone = []
    for i in range(req.n):
        one = synth.FoldinRequests(1, req.ptr[i:i + 2] - req.ptr[i], req.cols[req.ptr[i]:req.ptr[i + 1]],
                                   req.vals[req.ptr[i]:req.ptr[i + 1]], req.q_ptr[i:i + 2] - req.q_ptr[i],
                                   req.q_cols[req.q_ptr[i]:req.q_ptr[i + 1]], np.zeros(1))
        alone.append(_run_direct(fm, one))
    # all of them through the server at once (mixed batches)
    srv = FoldinServer(fm, mem_budget_bytes=64 << 20, n_streams=3, max_batch=16)
    for i in range(req.n):
        srv.submit(i, req.cols[req.ptr[i]:req.ptr[i + 1]], req.vals[req.ptr[i]:req.ptr[i + 1]],
                   req.q_cols[req.q_ptr[i]:req.q_ptr[i + 1]])
    srv.drain()
    res = {}
    while len(res) < req.n:
        for rid, p, lat in srv.poll():
            res[rid] = p
            assert lat > 0
    st = srv.stats()
    srv.close()
    assert st["batches"] >= 4 and st["max_batch"] > 1  # requests really were batched together
    for i in range(req.n):
        assert np.array_equal(res[i], alone[i]), i
    # and the whole batch in one direct call too
    assert np.array_equal(_run_direct(fm, req), np.concatenate(alone))


def test_server_memory_admission():
    from paper_1705_10633_amd.serving import FoldinServer
    model = synth.foldin_model(S=16, N=4000, K=32, seed=4)
    fm = _foldin(model)
    budget = 2 * 220_000
    srv = FoldinServer(fm, mem_budget_bytes=budget, n_streams=2, max_batch=1000, max_inflight=1000)
    req = synth.foldin_requests(200, 4000, seed=4, Q=50, cap=400)
    for i in range(req.n):
        srv.submit(i, req.cols[req.ptr[i]:req.ptr[i + 1]], req.vals[req.ptr[i]:req.ptr[i + 1]],
                   req.q_cols[req.q_ptr[i]:req.q_ptr[i + 1]])
    srv.drain()
    st = srv.stats()
    got = {}
    while len(got) < req.n:
        for rid, p, _ in srv.poll():
            got[rid] = p
    srv.close()
    assert st["max_batch_bytes"] <= st["stream_capacity"] == budget // 2
    assert st["batches"] > 1
    ref = _run_direct(fm, req)
    for i in range(req.n):
        assert np.array_equal(got[i], ref[req.q_ptr[i]:req.q_ptr[i + 1]])
    # a request larger than one stream's share is refused, not dropped silently
    srv2 = FoldinServer(fm, mem_budget_bytes=budget, n_streams=2)
    # S * nq * 4 bytes of per-sample partials alone (16 * 3900 * 4 = 250 KB) exceed 220 KB
    big = np.arange(100, dtype=np.int32)
    from paper_1705_10633_amd._lib import BpmfError
    with pytest.raises(BpmfError):
        srv2.submit(0, big, np.ones(100, np.float32), np.arange(100, 4000, dtype=np.int32))
    with pytest.raises(BpmfError):
        srv2.submit(1, np.array([4000], np.int32), np.ones(1, np.float32), np.array([0], np.int32))
    srv2.close()


def test_server_replay_poisson_trace():
    from paper_1705_10633_amd.serving import FoldinServer
    model = synth.foldin_model(S=16, N=20000, K=64, seed=5)
    fm = _foldin(model)
    req = synth.foldin_requests(2000, 20000, seed=5, Q=100, rate=20000)
    srv = FoldinServer(fm, mem_budget_bytes=256 << 20, n_streams=4, max_batch=256)
    out, lat = srv.replay(req)
    st = srv.stats()
    srv.close()
    assert np.all(lat > 0) and lat.size == req.n
    print(f"20k req/s: p50 {np.percentile(lat, 50) * 1e3:.3f} ms p99 {np.percentile(lat, 99) * 1e3:.3f} ms, "
          f"batches {st['batches']}, max batch {st['max_batch']}")
    ref = _run_direct(fm, req)
    assert np.array_equal(out, ref)


def _sub_requests(req, pick):
    """The requests `pick` of a FoldinRequests, as one batch in that order."""
    cnt = req.ptr[pick + 1] - req.ptr[pick]
    qcnt = req.q_ptr[pick + 1] - req.q_ptr[pick]
    ptr = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    q_ptr = np.concatenate([[0], np.cumsum(qcnt)]).astype(np.int64)
    cols = np.concatenate([req.cols[req.ptr[i]:req.ptr[i + 1]] for i in pick])
    vals = np.concatenate([req.vals[req.ptr[i]:req.ptr[i + 1]] for i in pick])
    qc = np.concatenate([req.q_cols[req.q_ptr[i]:req.q_ptr[i + 1]] for i in pick])
    return synth.FoldinRequests(pick.size, ptr, cols.astype(np.int32), vals.astype(np.float32), q_ptr,
                                qc.astype(np.int32), np.zeros(pick.size))


def _pivot_failure_model(S, N, K, seed):
    """alpha = 1e9 makes P = Lambda + alpha sum v v^T of a request with fewer
    ratings than K rank-deficient up to Lambda: its largest diagonal is
    ~ alpha |v|^2 ~ 1e8 while the pivots past the rated directions are
    ~ Lambda_kk ~ 1e1, below 64 K 2^-24 max P_kk (~ 1e4), so the FP32
    Cholesky fails for every sample; requests with many more ratings than K
    stay well conditioned and pass in FP32."""
    m = synth.foldin_model(S=S, N=N, K=K, seed=seed)
    return synth.FoldinModel(m.S, m.N, m.K, 1e9, m.mean_rating, m.Vs, m.Lambda, m.mu)


def _pivot_failure_requests(N, seed, n=24, Q=9):
    """Alternating requests with 1..3 ratings (FP32 pivot fails) and 300."""
    rng = np.random.default_rng(seed)
    counts = np.where(np.arange(n) % 2 == 0, rng.integers(1, 4, n), 300)
    ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    cols, qcols = [], []
    for c in counts:
        pick = rng.choice(N, size=int(c) + Q, replace=False)
        cols.append(np.sort(pick[:c]))
        qcols.append(pick[c:])
    vals = (3.0 + rng.standard_normal(int(ptr[-1]))).astype(np.float32)
    return synth.FoldinRequests(n, ptr, np.concatenate(cols).astype(np.int32), vals,
                                np.arange(n + 1, dtype=np.int64) * Q,
                                np.concatenate(qcols).astype(np.int32), np.zeros(n))


# FP64 arithmetic on FP32 inputs, FP32 output: relative 6e-8 of the prediction
# plus cond(P) 2^-52 (cond ~ 1e8 here) -> 1e-6 with a margin.
FOLDIN_F64_TOL = 1e-6


@pytest.mark.parametrize("K", [16, 64])
def test_foldin_fp32_pivot_failure_recomputed_in_fp64(K):
    """(request, sample) pairs whose FP32 pivot fails are recomputed in FP64
    and agree with the FP64 oracle to FP64 accuracy; the FP32 Cholesky of such
    a P loses all digits in the unrated directions, so without the recompute
    the error would be O(1)."""
    N = 2000
    model = _pivot_failure_model(4, N, K, seed=K + 40)
    req = _pivot_failure_requests(N, seed=K)
    got = _run_direct(_foldin(model), req)
    ref = O.foldin(model, req)
    assert np.all(np.isfinite(got))
    err = np.abs(got - ref) / (1.0 + np.abs(ref - model.mean_rating))
    few = np.repeat((req.ptr[1:] - req.ptr[:-1]) < K, req.q_ptr[1:] - req.q_ptr[:-1])
    print(f"K={K}: requests with fewer ratings than K (FP64 recompute) max err {err[few].max():.2e}; "
          f"with 300 ratings (FP32) max err {err[~few].max():.2e}")
    assert err[few].max() <= FOLDIN_F64_TOL
    assert err[~few].max() <= FOLDIN_TOL


def test_foldin_serving_shape_against_oracle():
    """The serving workload's shape (S = 16 samples of 20,000 x 64, log-normal
    rating counts clipped at 5,000, Q = 100): the 12 largest requests of a
    2,000-request trace and 36 others, in one batch, against the oracle."""
    model = synth.foldin_model(S=16, N=20000, K=64, seed=5)
    req = synth.foldin_requests(2000, 20000, seed=5, Q=100, rate=20000)
    cnt = req.ptr[1:] - req.ptr[:-1]
    rng = np.random.default_rng(3)
    pick = np.unique(np.concatenate([np.argsort(cnt)[-12:], rng.choice(req.n, 36, replace=False)]))
    sub = _sub_requests(req, pick)
    got = _run_direct(_foldin(model), sub)
    ref = O.foldin(model, sub)
    err = np.abs(got - ref) / (1.0 + np.abs(ref - model.mean_rating))
    print(f"serving shape: {pick.size} requests, {int(cnt[pick].min())}..{int(cnt[pick].max())} ratings, "
          f"max scaled err {err.max():.2e}, median {np.median(err):.2e}")
    assert int(cnt[pick].max()) >= 1000
    assert err.max() <= FOLDIN_TOL
