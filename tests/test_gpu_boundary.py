"""The C ABI's remaining paths on the GPU: bpmf_init's validation of the
rating matrix and the held-out pairs (each invalid input is refused with
BPMF_E_INVALID and no context is created), and bpmf_snapshot feeding fold-in
end to end (sampler -> sweeps -> snapshots into S slots -> bpmf_foldin,
against the FP64 oracle's fold-in on the snapshotted samples)."""
import ctypes as C

import numpy as np
import pytest

from oracle import oracle as O
from paper_1705_10633_amd import _lib, synth

from .gpu_common import make_sampler
from .test_gpu_serving import FOLDIN_TOL, _run_direct

pytestmark = pytest.mark.gpu

BPMF_E_INVALID = 1


def _raw_init(prob, arrays, test_rows=None, test_cols=None, validate=1):
    """bpmf_init straight through the C ABI on the given CSR/CSC arrays
    (dict of numpy arrays); returns (status, ctx pointer, message)."""
    import torch
    lib = _lib.load()
    dev = {k: torch.as_tensor(np.ascontiguousarray(v), device="cuda") for k, v in arrays.items()}
    K = prob.K
    R = _lib.Ratings(prob.M, prob.N, int(arrays["row_ptr"][-1]), dev["row_ptr"].data_ptr(),
                     dev["col_idx"].data_ptr(), dev["row_val"].data_ptr(), dev["col_ptr"].data_ptr(),
                     dev["row_idx"].data_ptr(), dev["col_val"].data_ptr(), 0)
    mu0 = np.zeros(K)
    W0 = np.eye(K)
    p = _lib.Params(K, _lib.BPMF_FP32, 2.0, 2.0, float(K), mu0.ctypes.data, W0.ctypes.data, 3.0, 1, 0, 0, validate)
    n_test = 0 if test_rows is None else len(test_rows)
    tr = torch.as_tensor(np.asarray(test_rows if n_test else [0], np.int32), device="cuda")
    tc = torch.as_tensor(np.asarray(test_cols if n_test else [0], np.int32), device="cuda")
    nb = C.c_size_t()
    st = lib.bpmf_workspace_size(C.byref(R), C.byref(p), n_test, C.byref(nb))
    assert st == 0
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    U = torch.zeros(prob.M, K, dtype=torch.float32, device="cuda")
    V = torch.zeros(prob.N, K, dtype=torch.float32, device="cuda")
    ctx = C.c_void_p(12345)
    st = lib.bpmf_init(C.byref(ctx), C.byref(R), C.byref(p), U.data_ptr(), V.data_ptr(), ws.data_ptr(),
                       C.c_size_t(nb.value), n_test, tr.data_ptr(), tc.data_ptr(), None)
    msg = lib.bpmf_last_error().decode()
    if st == 0:
        lib.bpmf_destroy(ctx)
    return st, ctx.value, msg


def _arrays(R):
    return {"row_ptr": R.row_ptr.astype(np.int64), "col_idx": R.col_idx.astype(np.int32),
            "row_val": R.row_val.astype(np.float32), "col_ptr": R.col_ptr.astype(np.int64),
            "row_idx": R.row_idx.astype(np.int32), "col_val": R.col_val.astype(np.float32)}


def _first_row_with(ptr, n):
    return int(np.flatnonzero(ptr[1:] - ptr[:-1] >= n)[0])


def _corrupt(kind, R):
    a = _arrays(R)
    i = _first_row_with(a["row_ptr"], 3)
    b = int(a["row_ptr"][i])
    if kind == "unsorted":
        a["col_idx"][b], a["col_idx"][b + 1] = a["col_idx"][b + 1], a["col_idx"][b]
    elif kind == "duplicate":
        a["col_idx"][b + 1] = a["col_idx"][b]
    elif kind == "col_out_of_range":
        a["col_idx"][int(a["row_ptr"][i + 1]) - 1] = R.N
    elif kind == "row_out_of_range":
        j = _first_row_with(a["col_ptr"], 1)
        a["row_idx"][int(a["col_ptr"][j + 1]) - 1] = R.M
    elif kind == "csr_ne_csc":
        a["col_val"][7] += 0.5
    elif kind == "nan_rating":
        # the same NaN in both orientations, so only the value check can refuse it
        c = int(a["col_idx"][b])
        u = int(a["col_ptr"][c]) + int(np.flatnonzero(a["row_idx"][a["col_ptr"][c]:a["col_ptr"][c + 1]] == i)[0])
        a["row_val"][b] = np.nan
        a["col_val"][u] = np.nan
    elif kind == "pointer_decreases":
        a["row_ptr"][i + 1], a["row_ptr"][i + 2] = a["row_ptr"][i + 2], a["row_ptr"][i + 1]
    else:
        raise ValueError(kind)
    return a


@pytest.mark.parametrize("kind,validate", [("unsorted", 1), ("duplicate", 1), ("col_out_of_range", 1),
                                           ("row_out_of_range", 1), ("csr_ne_csc", 1), ("nan_rating", 1),
                                           ("pointer_decreases", 0)])
def test_init_refuses_invalid_ratings(kind, validate):
    prob = synth.uniform_planted(M=120, N=80, K=8, nnz=2000, seed=31, n_sweeps=1)
    st, ctx, msg = _raw_init(prob, _corrupt(kind, prob.R), validate=validate)
    print(f"{kind}: status {st} ({msg})")
    assert st == BPMF_E_INVALID and not ctx
    # the library is unharmed: the valid matrix still initialises
    st, ctx, _ = _raw_init(prob, _arrays(prob.R))
    assert st == 0 and ctx


@pytest.mark.parametrize("pair", [(120, 3), (5, 80), (-1, 0)])
def test_init_refuses_test_pair_out_of_range(pair):
    prob = synth.uniform_planted(M=120, N=80, K=8, nnz=2000, seed=32, n_sweeps=1)
    rows = np.array([0, 1, pair[0]], np.int32)
    cols = np.array([2, 3, pair[1]], np.int32)
    st, ctx, msg = _raw_init(prob, _arrays(prob.R), rows, cols)
    assert st == BPMF_E_INVALID and not ctx, msg
    st, ctx, _ = _raw_init(prob, _arrays(prob.R), rows[:2], cols[:2])
    assert st == 0 and ctx


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_snapshot_feeds_foldin(precision):
    """S = 3 snapshots, one sweep apart, of a sampler's own V and user hypers;
    new users folded in against them agree with the FP64 oracle's fold-in on
    the same snapshotted samples, and each snapshot is bitwise the sampler's
    state at that sweep."""
    import torch
    from paper_1705_10633_amd.sampler import Foldin
    prob = synth.uniform_planted(M=400, N=300, K=16, nnz=12000, seed=33, n_sweeps=5, burnin=0)
    s = make_sampler(prob, precision=precision, seed=77, with_test=False)
    S, N, K = 3, prob.N, prob.K
    Vs = torch.empty(S, N, K, dtype=torch.float32, device="cuda")
    Lam = torch.empty(S, K, K, dtype=torch.float64, device="cuda")
    mu = torch.empty(S, K, dtype=torch.float64, device="cuda")
    s.sweep(2)
    for k in range(S):
        s.sweep(1)
        s.snapshot(Vs[k], Lam[k], mu[k])
        torch.cuda.synchronize()
        h = s.hyper()
        assert torch.equal(Vs[k], s.V.to(torch.float32))
        assert np.array_equal(Lam[k].cpu().numpy(), h["Lambda_U"])
        assert np.array_equal(mu[k].cpu().numpy(), h["mu_U"])
    assert not torch.equal(Vs[0], Vs[2])
    model = synth.FoldinModel(S, N, K, prob.alpha, prob.mean_rating, Vs.cpu().numpy(), Lam.cpu().numpy(),
                              mu.cpu().numpy())
    req = synth.foldin_requests(30, N, seed=4, Q=12, cap=200)
    fm = Foldin(model.Vs, model.Lambda, model.mu, model.alpha, model.mean_rating)
    got = _run_direct(fm, req)
    ref = O.foldin(model, req)
    err = np.abs(got - ref) / (1.0 + np.abs(ref - model.mean_rating))
    print(f"{precision}: snapshot fold-in max scaled err {err.max():.2e}")
    assert err.max() <= FOLDIN_TOL
