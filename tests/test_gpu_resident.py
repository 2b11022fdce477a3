"""Resident fold-in server (one persistent kernel, request slots in pinned
host memory): predictions bitwise equal to bpmf_foldin and within the fold-in
tolerance of the FP64 oracle, requests whose FP32 pivot fails recomputed in
FP64, the kernel's idle exit and relaunch, slot-size admission, and real-time
replay."""
import time

import numpy as np
import pytest

from paper_1705_10633_amd import synth

from oracle import oracle as O

from .test_gpu_serving import (FOLDIN_F64_TOL, FOLDIN_TOL, _foldin, _pivot_failure_model,
                               _pivot_failure_requests, _run_direct)

pytestmark = pytest.mark.gpu


def _submit_all(srv, req, ids=None):
    for i in range(req.n):
        srv.submit(i if ids is None else ids[i], req.cols[req.ptr[i]:req.ptr[i + 1]],
                   req.vals[req.ptr[i]:req.ptr[i + 1]], req.q_cols[req.q_ptr[i]:req.q_ptr[i + 1]])


def _collect(srv, n):
    got = {}
    t0 = time.time()
    while len(got) < n:
        for rid, p, lat in srv.poll():
            assert lat > 0
            got[rid] = p
        assert time.time() - t0 < 60
    return got


@pytest.mark.parametrize("S,K,N", [(8, 64, 3000), (16, 32, 4000), (3, 10, 500)])
def test_resident_server_equals_foldin(S, K, N):
    from paper_1705_10633_amd.serving import FoldinServer
    model = synth.foldin_model(S=S, N=N, K=K, seed=K)
    fm = _foldin(model)
    req = synth.foldin_requests(80, N, seed=K + 1, Q=20, cap=600)
    srv = FoldinServer(fm, resident=True, n_slots=8, max_nnz=600, max_q=20)
    _submit_all(srv, req)
    srv.drain()
    got = _collect(srv, req.n)
    st = srv.stats()
    srv.close()
    assert st["requests_done"] == req.n and st["max_inflight"] <= 8
    ref = _run_direct(fm, req)
    for i in range(req.n):
        assert np.array_equal(got[i], ref[req.q_ptr[i]:req.q_ptr[i + 1]]), i
    # and against the FP64 oracle
    ora = O.foldin(model, req)
    res = np.concatenate([got[i] for i in range(req.n)])
    err = np.abs(res - ora) / (1.0 + np.abs(ora - model.mean_rating))
    print(f"S={S} K={K}: resident vs oracle max scaled err {err.max():.2e}")
    assert err.max() <= FOLDIN_TOL


def test_resident_pivot_failure_recomputed_in_fp64():
    """A request whose FP32 pivot fails comes back from the resident kernel as
    NaN and is computed again in FP64 (through bpmf_foldin): the predictions
    equal batching mode's bitwise and the FP64 oracle's to FP64 accuracy."""
    from paper_1705_10633_amd.serving import FoldinServer
    N, K = 2000, 32
    model = _pivot_failure_model(8, N, K, seed=7)
    fm = _foldin(model)
    req = _pivot_failure_requests(N, seed=11, n=16, Q=9)
    srv = FoldinServer(fm, resident=True, n_slots=4, max_nnz=400, max_q=16)
    _submit_all(srv, req)
    srv.drain()
    got = _collect(srv, req.n)
    srv.close()
    ref = _run_direct(fm, req)
    ora = O.foldin(model, req)
    for i in range(req.n):
        sl = slice(req.q_ptr[i], req.q_ptr[i + 1])
        assert np.array_equal(got[i], ref[sl]), i
        err = np.abs(got[i] - ora[sl]) / (1.0 + np.abs(ora[sl] - model.mean_rating))
        bound = FOLDIN_F64_TOL if req.ptr[i + 1] - req.ptr[i] < K else FOLDIN_TOL
        assert err.max() <= bound, (i, err.max())


def test_resident_empty_request_and_slot_admission():
    from paper_1705_10633_amd.serving import FoldinServer
    from paper_1705_10633_amd._lib import BpmfError
    model = synth.foldin_model(S=4, N=200, K=16, seed=2)
    fm = _foldin(model)
    srv = FoldinServer(fm, resident=True, n_slots=2, max_nnz=10, max_q=5)
    q = np.array([1, 7, 20, 50, 99], np.int32)
    srv.submit(0, np.zeros(0, np.int32), np.zeros(0, np.float32), q)
    with pytest.raises(BpmfError):
        srv.submit(1, np.arange(11, dtype=np.int32), np.ones(11, np.float32), q)
    with pytest.raises(BpmfError):
        srv.submit(2, np.arange(3, dtype=np.int32), np.ones(3, np.float32), np.arange(6, dtype=np.int32))
    srv.drain()
    got = _collect(srv, 1)
    srv.close()
    one = synth.FoldinRequests(1, np.array([0, 0], np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32),
                               np.array([0, 5], np.int64), q, np.zeros(1))
    assert np.array_equal(got[0], _run_direct(fm, one))


def test_resident_server_with_a_slot_per_compute_unit():
    """256 slots of 16 wavefronts: one slot workgroup per CU of the chip (the
    most the device holds at once, else creation is refused)."""
    from paper_1705_10633_amd.serving import FoldinServer
    from paper_1705_10633_amd._lib import BpmfError
    model = synth.foldin_model(S=16, N=3000, K=64, seed=9)
    fm = _foldin(model)
    req = synth.foldin_requests(300, 3000, seed=9, Q=16, cap=400)
    try:
        srv = FoldinServer(fm, resident=True, n_slots=256, max_nnz=400, max_q=16, idle_polls=20000)
    except BpmfError as e:
        assert "holds at once" in str(e)
        pytest.skip("device holds fewer than 256 slot workgroups")
    _submit_all(srv, req)
    srv.drain()
    got = _collect(srv, req.n)
    srv.close()
    ref = _run_direct(fm, req)
    for i in range(req.n):
        assert np.array_equal(got[i], ref[req.q_ptr[i]:req.q_ptr[i + 1]]), i


def test_resident_kernel_ends_when_idle_and_is_relaunched():
    """With a short idle limit the kernel ends between the two bursts; the
    second burst is served by a new launch with the same results."""
    from paper_1705_10633_amd.serving import FoldinServer
    model = synth.foldin_model(S=8, N=2000, K=64, seed=6)
    fm = _foldin(model)
    req = synth.foldin_requests(40, 2000, seed=6, Q=10, cap=300)
    srv = FoldinServer(fm, resident=True, n_slots=4, max_nnz=300, max_q=10, idle_polls=2000)
    _submit_all(srv, req)
    srv.drain()
    first = _collect(srv, req.n)
    time.sleep(0.3)  # far longer than 2000 idle polls: the kernel has ended
    _submit_all(srv, req, ids=[req.n + i for i in range(req.n)])
    srv.drain()
    second = _collect(srv, req.n)
    srv.close()
    ref = _run_direct(fm, req)
    for i in range(req.n):
        want = ref[req.q_ptr[i]:req.q_ptr[i + 1]]
        assert np.array_equal(first[i], want) and np.array_equal(second[req.n + i], want), i


def test_resident_replay_poisson_trace():
    from paper_1705_10633_amd.serving import FoldinServer
    model = synth.foldin_model(S=16, N=20000, K=64, seed=5)
    fm = _foldin(model)
    req = synth.foldin_requests(2000, 20000, seed=5, Q=100, rate=20000)
    srv = FoldinServer(fm, resident=True, n_slots=32, max_nnz=5000, max_q=100)
    out, lat = srv.replay(req)
    srv.close()
    assert np.all(lat > 0) and lat.size == req.n
    print(f"resident, 20k req/s: p50 {np.percentile(lat, 50) * 1e3:.3f} ms "
          f"p99 {np.percentile(lat, 99) * 1e3:.3f} ms")
    assert np.array_equal(out, _run_direct(fm, req))
