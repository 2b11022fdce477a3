"""Fold-in serving: the native continuous-batching engine of libbpmf
(bpmf_server_*), its Python handle, and the latency benchmark of the
S = 16 x 20,000 x 64 fold-in workload."""
from __future__ import annotations

import ctypes as C
import time

import numpy as np

from . import _lib
from ._lib import call


class FoldinServer:
    """Continuous-batching fold-in server over stored posterior samples
    (a sampler.Foldin holding the device arrays)."""

    def __init__(self, foldin, mem_budget_bytes=256 << 20, n_streams=4, max_batch=256,
                 max_inflight=4096, resident=False, n_slots=32, max_nnz=5000, max_q=128, idle_polls=0):
        """resident=True: one persistent kernel serves n_slots requests at a
        time (bpmf_server_create_resident) instead of a launch per batch."""
        self.foldin = foldin  # keeps the model's device arrays alive
        self.srv = C.c_void_p()
        if resident:
            call("bpmf_server_create_resident", C.byref(self.srv), C.byref(foldin.model), n_slots, max_nnz,
                 max_q, int(idle_polls))
        else:
            call("bpmf_server_create", C.byref(self.srv), C.byref(foldin.model), C.c_size_t(mem_budget_bytes),
                 n_streams, max_batch, max_inflight)

    def close(self):
        if self.srv:
            _lib.load().bpmf_server_destroy(self.srv)
            self.srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, rid, cols, vals, q_cols):
        cols = np.ascontiguousarray(cols, np.int32)
        vals = np.ascontiguousarray(vals, np.float32)
        q = np.ascontiguousarray(q_cols, np.int32)
        call("bpmf_server_submit", self.srv, int(rid), cols.size, cols.ctypes.data, vals.ctypes.data,
             q.size, q.ctypes.data)

    def drain(self):
        call("bpmf_server_drain", self.srv)

    def poll(self, max_results=4096, pred_capacity=1 << 22):
        ids = np.empty(max_results, np.int64)
        off = np.empty(max_results + 1, np.int64)
        preds = np.empty(pred_capacity, np.float32)
        lat = np.empty(max_results)
        n = C.c_int32()
        call("bpmf_server_poll", self.srv, max_results, ids.ctypes.data, off.ctypes.data, preds.ctypes.data,
             pred_capacity, lat.ctypes.data, C.byref(n))
        k = n.value
        return [(int(ids[i]), preds[off[i]:off[i + 1]].copy(), float(lat[i])) for i in range(k)]

    def stats(self):
        st = _lib.ServerStats()
        call("bpmf_server_get_stats", self.srv, C.byref(st))
        return {f: getattr(st, f) for f, _ in st._fields_}

    def replay(self, req):
        """Replays a synth.FoldinRequests trace in real time; returns (predictions, latencies)."""
        n = req.n
        out = np.empty(max(int(req.q_ptr[-1]), 1), np.float32)
        lat = np.empty(max(n, 1))
        arr = np.ascontiguousarray(req.arrival, np.float64)
        ptr = np.ascontiguousarray(req.ptr, np.int64)
        cols = np.ascontiguousarray(req.cols, np.int32)
        vals = np.ascontiguousarray(req.vals, np.float32)
        qp = np.ascontiguousarray(req.q_ptr, np.int64)
        qc = np.ascontiguousarray(req.q_cols, np.int32)
        call("bpmf_server_replay", self.srv, n, arr.ctypes.data, ptr.ctypes.data, cols.ctypes.data,
             vals.ctypes.data, qp.ctypes.data, qc.ctypes.data, out.ctypes.data, lat.ctypes.data)
        return out[: int(req.q_ptr[-1])], lat[:n]


def bench_foldin(seconds=2.0, rates=(5000, 10000, 20000, 50000), S=16, N=20000, K=64, Q=100,
                 n_streams=4, mem_budget=256 << 20, max_batch=256, log=print, resident_rate=20000,
                 saturating_batch=4096):
    """p50 / p99 latency of Poisson request streams against S stored samples
    (batched server at each rate, the resident-kernel server at one), and the
    fold-in kernel's FP32 work rate on one saturating batch."""
    from . import synth
    from .sampler import Foldin
    model = synth.foldin_model(S=S, N=N, K=K)
    fm = Foldin(model.Vs, model.Lambda, model.mu, model.alpha, model.mean_rating)
    out = {"model": f"S={S} samples of V ({N} x {K}, FP32) resident on device",
           "request": "log-normal(3, 1.5) ratings clipped to 1..5000 over distinct columns, "
                      f"ratings N(3,1), Q={Q} query columns",
           "memory_budget_bytes": mem_budget, "n_streams": n_streams, "max_batch": max_batch,
           "rates": {}}
    for rate in rates:
        n = int(rate * seconds)
        t0 = time.perf_counter()
        req = synth.foldin_requests(n, N, seed=105, Q=Q, rate=rate, stream_offset=rate)
        gen = time.perf_counter() - t0
        srv = FoldinServer(fm, mem_budget_bytes=mem_budget, n_streams=n_streams, max_batch=max_batch)
        # warm-up burst
        warm = synth.foldin_requests(64, N, seed=7, Q=Q, rate=rate, stream_offset=1)
        srv.replay(warm)
        t0 = time.perf_counter()
        _, lat = srv.replay(req)
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        lat_ms = lat * 1e3
        rec = {"requests": n, "offered_rps": rate, "achieved_rps": n / wall,
               "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
               "p999_ms": float(np.percentile(lat_ms, 99.9)), "max_ms": float(lat_ms.max()),
               "batches": st["batches"], "mean_batch": st["requests_done"] / max(st["batches"], 1),
               "max_batch": st["max_batch"], "max_inflight": st["max_inflight"]}
        out["rates"][str(rate)] = rec
        log(f"[serve] {rate:6d} req/s: p50 {rec['p50_ms']:.3f} ms p99 {rec['p99_ms']:.3f} ms "
            f"(mean batch {rec['mean_batch']:.1f}, achieved {rec['achieved_rps']:.0f} req/s, gen {gen:.1f} s)")
    if resident_rate:
        n = int(resident_rate * seconds)
        req = synth.foldin_requests(n, N, seed=105, Q=Q, rate=resident_rate, stream_offset=resident_rate)
        srv = FoldinServer(fm, resident=True, n_slots=32, max_nnz=5000, max_q=Q)
        srv.replay(synth.foldin_requests(64, N, seed=7, Q=Q, rate=resident_rate, stream_offset=1))
        _, lat = srv.replay(req)
        srv.close()
        lat_ms = lat * 1e3
        out["resident"] = {"rate": resident_rate, "slots": 32, "requests": n,
                           "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99))}
        log(f"[serve] resident kernel, {resident_rate} req/s: p50 {out['resident']['p50_ms']:.3f} ms "
            f"p99 {out['resident']['p99_ms']:.3f} ms")
    if saturating_batch:
        out["saturating_batch"] = foldin_batch_throughput(fm, N, K, S, Q, saturating_batch)
        sb = out["saturating_batch"]
        log(f"[serve] batch of {saturating_batch}: {sb['ms_per_batch']:.3f} ms, {sb['requests_per_s']:.3g} req/s, "
            f"{sb['achieved_TFLOPs']:.2f} TFLOP/s = {100 * sb['frac']:.1f} % of FP32 peak")
    return out


def foldin_batch_throughput(fm, N, K, S, Q, n_req, reps=10, seed=106):
    """One bpmf_foldin call over n_req requests, timed with HIP events on the
    launch stream; algorithmic FP32 work per (request, sample): the Gram and
    rhs nnz (K^2 + 3K), the Cholesky K^3 / 3, the two solves 2 K^2 and the
    query dot products 2 K Q."""
    import torch
    from . import synth
    req = synth.foldin_requests(n_req, N, seed=seed, Q=Q)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    args = [dev(req.ptr), dev(req.cols), dev(req.vals), dev(req.q_ptr), dev(req.q_cols)]
    out = torch.empty(max(int(req.q_cols.size), 1), dtype=torch.float32, device="cuda")
    ws = torch.empty(fm.workspace_bytes(int(req.q_cols.size)), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(2):
        fm.run(*args, out=out, ws=ws, stream=stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fm.run(*args, out=out, ws=ws, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nnz = np.diff(req.ptr).astype(np.float64)
    nq = np.diff(req.q_ptr).astype(np.float64)
    flops = S * float(np.sum(nnz * (K * K + 3 * K) + K ** 3 / 3.0 + 2 * K * K + 2 * K * nq))
    tf = flops / (ms * 1e-3) / 1e12
    return {"requests": n_req, "ms_per_batch": ms, "requests_per_s": n_req / (ms * 1e-3),
            "algorithmic_flop_per_batch": flops, "achieved_TFLOPs": tf, "peak_TFLOPs": 157.3,
            "frac": tf / 157.3, "bound": "alu"}
