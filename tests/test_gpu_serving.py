"""Fold-in kernel against the oracle, and the continuous-batching server:
results alone == results in a mixed batch (bitwise), memory admission, and
real-time replay of a Poisson trace."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1705_10633_amd import synth

pytestmark = pytest.mark.gpu

# FP32 fold-in: the Gram, Cholesky and solves run in FP32 on FP32 samples;
# relative error of m_s ~ cond(P) * K * 6e-8 with cond(P) < ~1e2 here, and a
# prediction is a K-term dot product -> bound 2e-4 * (1 + |pred - rbar|).
FOLDIN_TOL = 2e-4


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
