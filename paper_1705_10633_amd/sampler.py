"""Python front end of the BPMF sampler: torch owns the device buffers and the
stream; every computation is a call into libbpmf.so (see include/bpmf.h).
"""
from __future__ import annotations

import ctypes as C
import math
from typing import Optional

import numpy as np

from . import _lib
from ._lib import call


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("a ROCm GPU is required: the sampler has no CPU path")
    return torch


def _stream(torch, stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class DeviceRatings:
    """CSR + CSC of a synth.Ratings (or equivalent arrays) copied to the GPU."""

    def __init__(self, R, device="cuda", val_dtype="float32"):
        torch = _torch()
        dt = torch.float64 if val_dtype == "float64" else torch.float32
        self.M, self.N, self.nnz = int(R.M), int(R.N), int(R.row_ptr[-1])
        self.row_ptr = torch.as_tensor(np.asarray(R.row_ptr, np.int64), device=device)
        self.col_idx = torch.as_tensor(np.asarray(R.col_idx, np.int32), device=device)
        self.row_val = torch.as_tensor(np.asarray(R.row_val), device=device).to(dt)
        self.col_ptr = torch.as_tensor(np.asarray(R.col_ptr, np.int64), device=device)
        self.row_idx = torch.as_tensor(np.asarray(R.row_idx, np.int32), device=device)
        self.col_val = torch.as_tensor(np.asarray(R.col_val), device=device).to(dt)
        self.val_is_f64 = 1 if val_dtype == "float64" else 0

    def cstruct(self):
        return _lib.Ratings(self.M, self.N, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(),
                            self.row_val.data_ptr(), self.col_ptr.data_ptr(), self.row_idx.data_ptr(),
                            self.col_val.data_ptr(), self.val_is_f64)


class Sampler:
    """Gibbs sampler for BPMF on one GPU (one context of libbpmf)."""

    def __init__(self, ratings: DeviceRatings, K: int, U0, V0, precision: str = "fp64",
                 alpha: float = 2.0, beta0: float = 2.0, nu0: Optional[float] = None,
                 mu0=None, W0=None, mean_rating: float = float("nan"), seed: int = 0,
                 burnin: int = 0, test_rows=None, test_cols=None, use_graph: bool = False,
                 validate: bool = False, stream=None, shape=None):
        torch = _torch()
        self.torch = torch
        self.tune_table = None
        self.tune_cached = False
        if isinstance(shape, str):
            # "auto": the cached shape of this problem (GPU architecture, K, precision,
            # rating-count histogram), else time the candidates on this problem first
            # and keep (and cache) the fastest; only the mixed-precision kernels for
            # K <= 64 have shapes to choose
            if shape not in ("auto", "auto-nocache"):
                raise ValueError("shape must be None, a dict of bpmf_launch_shape fields or 'auto'")
            use_cache = shape == "auto"
            shape = {}
            if precision != "fp64" and K <= 64:
                from . import autotune
                counts = [torch.diff(ratings.row_ptr).cpu().numpy(), torch.diff(ratings.col_ptr).cpu().numpy()]
                arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName
                key = autotune.problem_key(counts, K, precision, arch)
                cached = autotune.cache_lookup(key) if use_cache else None
                if cached is not None:
                    shape, self.tune_cached = cached, True
                else:
                    shape, self.tune_table = autotune.tune(
                        ratings, K, U0, V0, counts, precision=precision, alpha=alpha, beta0=beta0, nu0=nu0,
                        mu0=mu0, W0=W0, mean_rating=mean_rating, seed=seed)
                    if use_cache:
                        autotune.cache_store(key, shape, self.tune_table, autotune.variant_fits())
        self.R = ratings
        self.K = K
        self.precision = precision
        prec = _lib.PRECISIONS[precision]
        xdt = torch.float64 if prec == _lib.BPMF_FP64 else torch.float32
        self.U = torch.as_tensor(np.asarray(U0), device="cuda").to(xdt).contiguous().clone()
        self.V = torch.as_tensor(np.asarray(V0), device="cuda").to(xdt).contiguous().clone()
        assert self.U.shape == (ratings.M, K) and self.V.shape == (ratings.N, K)
        nu0 = float(K) if nu0 is None else float(nu0)
        self._mu0 = np.ascontiguousarray(np.zeros(K) if mu0 is None else mu0, dtype=np.float64)
        self._W0 = np.ascontiguousarray(np.eye(K) if W0 is None else W0, dtype=np.float64)
        self.params = _lib.Params(K, prec, alpha, beta0, nu0, self._mu0.ctypes.data,
                                  self._W0.ctypes.data, mean_rating, seed, burnin,
                                  1 if use_graph else 0, 1 if validate else 0)
        # launch shape of the mixed-precision sweep (bpmf_launch_shape); fields left out keep
        # the library's built-in choice
        self.shape = dict(shape or {})
        if shape:
            self._shape = _lib.LaunchShape(**self.shape)
            self.params.shape = C.pointer(self._shape)
        self._rs = ratings.cstruct()
        if test_rows is not None:
            self.test_rows = torch.as_tensor(np.asarray(test_rows, np.int32), device="cuda")
            self.test_cols = torch.as_tensor(np.asarray(test_cols, np.int32), device="cuda")
            n_test = int(self.test_rows.numel())
        else:
            self.test_rows = self.test_cols = None
            n_test = 0
        self.n_test = n_test
        nbytes = C.c_size_t()
        call("bpmf_workspace_size", C.byref(self._rs), C.byref(self.params), n_test, C.byref(nbytes))
        self.ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device="cuda")
        self.ctx = C.c_void_p()
        call("bpmf_init", C.byref(self.ctx), C.byref(self._rs), C.byref(self.params), _ptr(self.U),
             _ptr(self.V), _ptr(self.ws), C.c_size_t(self.ws.numel()), n_test,
             _ptr(self.test_rows), _ptr(self.test_cols), _stream(torch, stream))

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx:
            try:
                _lib.load().bpmf_destroy(ctx)
            except Exception:
                pass
            self.ctx = None

    def sweep(self, n: int = 1, tape=None, stream=None):
        """n Gibbs sweeps; `tape` (device float64 tensor) supplies every draw."""
        if tape is None:
            call("bpmf_sweep", self.ctx, n, None, 0, _stream(self.torch, stream))
        else:
            call("bpmf_sweep", self.ctx, n, _ptr(tape), int(tape.numel()), _stream(self.torch, stream))

    def predict(self, rows, cols, stream=None):
        torch = self.torch
        r = torch.as_tensor(np.asarray(rows, np.int32), device="cuda")
        c = torch.as_tensor(np.asarray(cols, np.int32), device="cuda")
        out = torch.empty(r.numel(), dtype=torch.float64, device="cuda")
        call("bpmf_predict", self.ctx, r.numel(), _ptr(r), _ptr(c), _ptr(out), _stream(torch, stream))
        return out

    def test_predictions(self, stream=None):
        torch = self.torch
        out = torch.empty(max(self.n_test, 1), dtype=torch.float64, device="cuda")
        cnt = C.c_int64()
        call("bpmf_test_predictions", self.ctx, _ptr(out), C.byref(cnt), _stream(torch, stream))
        return out[: self.n_test], cnt.value

    def hyper(self, stream=None):
        K = self.K
        buf = np.empty(2 * K * K + 2 * K)
        call("bpmf_get_hyper", self.ctx, buf.ctypes.data, _stream(self.torch, stream))
        o = K * K + K
        return {"Lambda_U": buf[:K * K].reshape(K, K), "mu_U": buf[K * K:o],
                "Lambda_V": buf[o:o + K * K].reshape(K, K), "mu_V": buf[o + K * K:]}

    def info(self, stream=None):
        i = _lib.Info()
        call("bpmf_get_info", self.ctx, C.byref(i), _stream(self.torch, stream))
        return {"sweeps_done": i.sweeps_done, "fallback_rows": i.fallback_rows,
                "nonfinite_rows": i.nonfinite_rows, "mean_rating": i.mean_rating,
                "rank1_rows": tuple(i.rank1_rows), "heavy_rows": tuple(i.heavy_rows),
                "pieces": tuple(i.pieces), "kernel_variant": i.kernel_variant}

    def set_timing(self, enable: bool):
        """Bracket every launch with HIP events (sweeps then run without graph replay)."""
        call("bpmf_set_timing", self.ctx, 1 if enable else 0)

    def timing(self, reset: bool = True):
        """Accumulated per-kernel-class milliseconds and launch counts."""
        t = _lib.Timing()
        call("bpmf_get_timing", self.ctx, C.byref(t), 1 if reset else 0)
        return {name: (t.ms[i], t.launches[i]) for i, name in enumerate(_lib.TIMING_CLASSES)}

    def snapshot(self, V_slot, Lambda_slot, mu_slot, stream=None):
        call("bpmf_snapshot", self.ctx, _ptr(V_slot), _ptr(Lambda_slot), _ptr(mu_slot),
             _stream(self.torch, stream))

    def save_state(self, stream=None) -> bytes:
        n = C.c_size_t()
        call("bpmf_state_size", self.ctx, C.byref(n))
        buf = C.create_string_buffer(n.value)
        call("bpmf_state_save", self.ctx, buf, n, _stream(self.torch, stream))
        return buf.raw

    def restore_state(self, blob: bytes, stream=None):
        buf = C.create_string_buffer(blob, len(blob))
        call("bpmf_state_restore", self.ctx, buf, C.c_size_t(len(blob)), _stream(self.torch, stream))


class Foldin:
    """Stored posterior samples for fold-in of new users (device tensors)."""

    def __init__(self, Vs, Lambda, mu, alpha: float, mean_rating: float):
        torch = _torch()
        self.torch = torch
        self.Vs = torch.as_tensor(np.asarray(Vs, np.float32), device="cuda").contiguous()
        self.Lambda = torch.as_tensor(np.asarray(Lambda, np.float64), device="cuda").contiguous()
        self.mu = torch.as_tensor(np.asarray(mu, np.float64), device="cuda").contiguous()
        S, N, K = self.Vs.shape
        self.model = _lib.FoldinModel(S, K, N, alpha, mean_rating, self.Vs.data_ptr(),
                                      self.Lambda.data_ptr(), self.mu.data_ptr())

    def workspace_bytes(self, n_queries: int) -> int:
        n = C.c_size_t()
        call("bpmf_foldin_workspace_size", C.byref(self.model), n_queries, C.byref(n))
        return n.value

    def run(self, ptr, cols, vals, q_ptr, q_cols, out=None, ws=None, stream=None):
        """All arguments are device tensors (int64 ptr/q_ptr, int32 cols/q_cols, float32 vals)."""
        torch = self.torch
        n_req = int(ptr.numel()) - 1
        n_q = int(q_cols.numel())
        if out is None:
            out = torch.empty(max(n_q, 1), dtype=torch.float32, device="cuda")
        if ws is None:
            ws = torch.empty(self.workspace_bytes(n_q), dtype=torch.uint8, device="cuda")
        call("bpmf_foldin", C.byref(self.model), n_req, _ptr(ptr), _ptr(cols), _ptr(vals), _ptr(q_ptr),
             _ptr(q_cols), n_q, _ptr(out), _ptr(ws), C.c_size_t(ws.numel()), _stream(torch, stream))
        return out[:n_q]

    def run_noalloc(self, ptr, cols, vals, q_ptr, q_cols, out, stream=None):
        """bpmf_foldin_noalloc: the same as run() with the partials in the
        library's own device array (no workspace, nothing allocated)."""
        n_req = int(ptr.numel()) - 1
        n_q = int(q_cols.numel())
        call("bpmf_foldin_noalloc", C.byref(self.model), n_req, _ptr(ptr), _ptr(cols), _ptr(vals), _ptr(q_ptr),
             _ptr(q_cols), n_q, _ptr(out), _stream(self.torch, stream))
        return out[:n_q]
