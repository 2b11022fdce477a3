"""The C ABI without a GPU: every function include/bpmf.h declares is exported
by libbpmf.so, and the host-side validation of parameters returns the
documented status codes (these calls never touch the device)."""
import ctypes as C
import json
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bpmf.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1705_10633_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1705_10633_amd import build
        build.build()
    return _lib.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bpmf_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("bpmf_init", "bpmf_sweep", "bpmf_predict", "bpmf_foldin", "bpmf_workspace_size",
                     "bpmf_server_create", "bpmf_server_replay"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and the Python binding declares argument types for all of them
    from paper_1705_10633_amd import _lib
    assert set(declared_functions()) <= set(_lib.EXPORTS), set(declared_functions()) - set(_lib.EXPORTS)


def test_timing_classes_match_the_header():
    """The binding's timing structure has the header's number of kernel classes."""
    from paper_1705_10633_amd import _lib
    n = int(re.search(r"#define BPMF_TIMING_CLASSES (\d+)", open(HEADER).read()).group(1))
    assert len(_lib.TIMING_CLASSES) == n
    assert C.sizeof(_lib.Timing) == 16 * n


def test_status_strings(lib):
    for code in range(7):
        assert lib.bpmf_status_string(code)
    assert lib.bpmf_version().startswith(b"bpmf")


def _params(K=4, nu0=None, W0=None, mu0=None, alpha=2.0, beta0=2.0, precision=0):
    from paper_1705_10633_amd import _lib
    mu0 = np.zeros(K) if mu0 is None else mu0
    W0 = np.eye(K) if W0 is None else W0
    keep = (np.ascontiguousarray(mu0, np.float64), np.ascontiguousarray(W0, np.float64))
    p = _lib.Params(K, precision, alpha, beta0, float(K) if nu0 is None else nu0, keep[0].ctypes.data,
                    keep[1].ctypes.data, float("nan"), 0, 0, 0, 0)
    return p, keep


def _ratings(M=10, N=8, nnz=20):
    from paper_1705_10633_amd import _lib
    fake = 0x1000  # never dereferenced by bpmf_workspace_size
    return _lib.Ratings(M, N, nnz, fake, fake, fake, fake, fake, fake, 0)


def _ws(lib, R, p, n_test=0):
    n = C.c_size_t()
    st = lib.bpmf_workspace_size(C.byref(R), C.byref(p), n_test, C.byref(n))
    return st, n.value


def test_workspace_size_validates_parameters(lib):
    R = _ratings()
    p, keep = _params()
    st, n = _ws(lib, R, p)
    assert st == 0 and n > 0
    st, n2 = _ws(lib, R, p, n_test=1000)
    assert st == 0 and n2 >= n + 8 * 1000
    for K in (0, 129):
        p, keep = _params(K=max(K, 1))
        p.K = K
        assert _ws(lib, R, p)[0] == 1, K
    p, keep = _params(K=4, nu0=2.9)          # nu0 must exceed K - 1
    assert _ws(lib, R, p)[0] == 1
    p, keep = _params(alpha=0.0)
    assert _ws(lib, R, p)[0] == 1
    p, keep = _params(beta0=-1.0)
    assert _ws(lib, R, p)[0] == 1
    p, keep = _params(mu0=np.array([0.0, math.nan, 0.0, 0.0]))
    assert _ws(lib, R, p)[0] == 1
    W = np.eye(4)
    W[0, 1] = 0.3
    p, keep = _params(W0=W)                   # not symmetric
    assert _ws(lib, R, p)[0] == 2
    W = np.eye(4)
    W[3, 3] = -1.0
    p, keep = _params(W0=W)                   # not positive definite
    assert _ws(lib, R, p)[0] == 2
    assert b"positive definite" in lib.bpmf_last_error()
    p, keep = _params(precision=3)
    assert _ws(lib, R, p)[0] == 1
    p, keep = _params()
    bad = _ratings(M=0)
    assert _ws(lib, bad, p)[0] == 1
    from paper_1705_10633_amd import _lib
    nulls = _lib.Ratings(10, 8, 20, 0x1000, None, None, 0x1000, None, None, 0)
    assert _ws(lib, nulls, p)[0] == 1
    # BF16 addresses gathered rows with 32-bit offsets: sides below 2^24 rows
    big = _ratings(M=1 << 24)
    p, keep = _params(precision=2)
    assert _ws(lib, big, p)[0] == 1 and b"2^24" in lib.bpmf_last_error()
    p, keep = _params(precision=1)
    assert _ws(lib, big, p)[0] == 0


def test_null_context_is_rejected(lib):
    assert lib.bpmf_sweep(None, 1, None, 0, None) == 4
    assert lib.bpmf_predict(None, 0, None, None, None, None) == 4
    assert lib.bpmf_destroy(None) == 0
    assert lib.bpmf_server_destroy(None) == 0
    assert lib.bpmf_server_submit(None, 0, 0, None, None, 0, None) == 4


def test_foldin_and_server_argument_checks(lib):
    from paper_1705_10633_amd import _lib
    fake = 0x1000
    m = _lib.FoldinModel(16, 64, 20000, 2.0, 3.0, fake, fake, fake)
    n = C.c_size_t()
    assert lib.bpmf_foldin_workspace_size(C.byref(m), 100, C.byref(n)) == 0
    assert n.value == 4 * 16 * 100
    bad = _lib.FoldinModel(16, 65, 20000, 2.0, 3.0, fake, fake, fake)   # K > 64
    assert lib.bpmf_foldin(C.byref(bad), 1, fake, fake, fake, fake, fake, 1, fake, fake, 1 << 20, None) == 1
    srv = C.c_void_p()
    assert lib.bpmf_server_create(C.byref(srv), C.byref(bad), 1 << 20, 2, 8, 8) == 1
    assert lib.bpmf_server_create(C.byref(srv), C.byref(m), 1 << 20, 0, 8, 8) == 1     # no streams
    assert lib.bpmf_server_create(C.byref(srv), C.byref(m), 64, 1, 8, 8) == 1          # budget too small
    # the no-allocation fold-in refuses what its fixed array cannot hold, before any device work
    cap = lib.bpmf_foldin_noalloc_max_partials()
    assert cap == 1 << 20
    assert lib.bpmf_foldin_noalloc(C.byref(m), 1, fake, fake, fake, fake, fake, cap // 16 + 1, fake, None) == 1
    assert lib.bpmf_foldin_noalloc(C.byref(bad), 1, fake, fake, fake, fake, fake, 1, fake, None) == 1
    assert lib.bpmf_foldin_noalloc(C.byref(m), -1, fake, fake, fake, fake, fake, 1, fake, None) == 1
    assert lib.bpmf_foldin_noalloc(C.byref(m), 0, None, None, None, None, None, 0, None, None) == 0


def test_launch_shape_fields_are_validated(lib):
    """bpmf_launch_shape: 0 keeps the built-in choice; out-of-range fields
    are rejected before any device work."""
    from paper_1705_10633_amd import _lib
    R = _ratings()
    good = [{}, {"heavy_min_ratings": 64, "piece_min_ratings": 64, "heavy_split": 1},
            {"heavy_split": -1, "rank1_max_ratings": -1}, {"rank1_max_ratings": 4, "rank1_split": 1},
            {"rank1_split": -1}, {"kernel_variant": 1}, {"kernel_variant": 2}, {"kernel_variant": 3}]
    bad = [{"heavy_min_ratings": 63}, {"heavy_min_ratings": -5}, {"piece_min_ratings": 1},
           {"heavy_split": 2}, {"rank1_split": -2}, {"rank1_max_ratings": 5},
           {"rank1_max_ratings": -2}, {"kernel_variant": 4}, {"kernel_variant": -1}]
    for fields, want in [(f, 0) for f in good] + [(f, 1) for f in bad]:
        p, keep = _params(precision=2)
        shp = _lib.LaunchShape(**fields)
        p.shape = C.pointer(shp)
        assert _ws(lib, R, p)[0] == want, fields
        if want:
            assert b"shape." in lib.bpmf_last_error()


def test_autotune_candidates_follow_the_counts():
    """The tuner varies only the knobs that change this matrix's launches,
    puts the built-in choice first, and lists no shape twice."""
    from paper_1705_10633_amd.autotune import candidate_shapes
    plain = candidate_shapes([np.full(100, 50), np.full(40, 125)], 64)
    assert plain == [{}, {"heavy_split": -1, "rank1_max_ratings": -1}]
    mixed = candidate_shapes([np.array([1, 2, 3, 9000, 50]), np.array([700, 20])], 32)
    assert mixed[0] == {}
    assert len(mixed) == len({json.dumps(c, sort_keys=True) for c in mixed})
    assert {"heavy_split": 1, "heavy_min_ratings": 4096, "piece_min_ratings": 256,
            "rank1_max_ratings": 3, "rank1_split": 1} in mixed
    assert not any(c.get("rank1_max_ratings") == 4 for c in mixed)   # no row has 4 ratings
    assert all(c.get("heavy_min_ratings", 0) <= 9000 for c in mixed)
    assert candidate_shapes([np.array([1, 9000])], 100) == [{}]     # K > 64: one launch shape
    # a chosen kernel variant is kept in every candidate; without heavy splits none is listed
    v = candidate_shapes([np.array([1, 2, 3, 9000, 50]), np.array([700, 20])], 64, heavy=False, variant=2)
    assert v[0] == {"kernel_variant": 2} and all(c["kernel_variant"] == 2 for c in v)
    assert not any(c.get("heavy_split") == 1 for c in v)


def test_autotune_cost_model():
    """The fixed-plus-per-rating fit recovers a, b from two launches, and the
    heavy-split test asks whether the heaviest row outlasts its launch's share
    (Section 4.2's workload model)."""
    from paper_1705_10633_amd import autotune
    a, b = autotune.fit_cost([(138493, 20_000_000, 0.004 * 138493 + 1.4e-5 * 2e7),
                              (26744, 20_000_000, 0.004 * 26744 + 1.4e-5 * 2e7)])
    assert abs(a - 0.004) < 1e-9 and abs(b - 1.4e-5) < 1e-12
    flat = [np.full(100000, 150)]
    assert not autotune.heavy_split_pays(flat, a, b)
    assert autotune.heavy_split_pays([np.concatenate([np.full(1000, 3), [9000]])], a, b)
    # a fit that is not a cost (negative per-rating or per-row part) prunes nothing
    assert autotune.heavy_split_pays(flat, 0.0167, -4.3e-5)
    assert autotune.heavy_split_pays(flat, -0.001, 1.4e-5)
    info = {"heavy_rows": (1, 0), "rank1_rows": (2, 0), "pieces": (4, 0)}
    assert autotune.launch_rows([np.array([1, 1, 50, 9000]), np.array([3, 4])], info) == [(5, 9050), (2, 7)]


def test_autotune_cache_keys(tmp_path):
    """The cache answers only for the same GPU architecture, K, precision and
    count histogram."""
    from paper_1705_10633_amd import autotune
    counts = [np.array([0, 1, 5, 900]), np.array([3, 903])]
    key = autotune.problem_key(counts, 64, "bf16", "gfx950")
    path = str(tmp_path / "cache.json")
    assert autotune.cache_lookup(key, path) is None
    autotune.cache_store(key, {"kernel_variant": 2}, [({}, 1.5)], [], path)
    assert autotune.cache_lookup(key, path) == {"kernel_variant": 2}
    assert autotune.cache_lookup(autotune.problem_key(counts, 64, "bf16", "gfx942"), path) is None
    assert autotune.cache_lookup(autotune.problem_key(counts, 32, "bf16", "gfx950"), path) is None
    other = [np.array([0, 1, 5, 9000]), np.array([3, 9003])]
    assert autotune.cache_lookup(autotune.problem_key(other, 64, "bf16", "gfx950"), path) is None
    autotune.cache_store(key, {"kernel_variant": 3}, [], [], path)
    assert autotune.cache_lookup(key, path) == {"kernel_variant": 3}


def test_autotune_result_round_trips(tmp_path):
    """A stored tuning result is returned only for the problem key it was
    tuned on."""
    from paper_1705_10633_amd import autotune
    key = {"M": 10, "N": 8, "nnz": 20, "K": 32, "precision": "fp32"}
    shape = {"heavy_split": 1, "heavy_min_ratings": 1024, "piece_min_ratings": 1024}
    path = str(tmp_path / "shape.json")
    autotune.save(path, shape, [({}, 0.36), (shape, 0.30)], key)
    assert autotune.load(path, key) == shape
    assert autotune.load(path, {**key, "K": 64}) is None
    assert autotune.load(str(tmp_path / "missing.json"), key) is None
