#!/usr/bin/env python3
"""Benchmark of the BPMF Gibbs sampler on one MI355X.

Metric: Gibbs rows sampled per second at K = 64 (users + movies per sweep,
whole sweeps including the hyper-parameter steps and the test predictions),
next to the plain FP64 one-workgroup-per-row path on the same data, plus the
p50 / p99 latency of batched fold-in serving.

Workload (one step = one Gibbs sweep): the MovieLens-20M-shaped synthetic
matrix, 138,493 x 26,744 with 20,000,000 ratings (log-normal row counts,
half-star ratings from a planted rank-64 model), K = 64, BF16 gathers and
Gram on matrix cores with FP32 accumulation, FP32 Cholesky, FP64 hyper step,
device Philox draws, whole sweep replayed from a HIP graph.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Progress goes to stderr; one JSON line goes to stdout.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X = {"hbm_GBs": 8000.0, "fp32_TFLOPs": 157.3, "bf16_TFLOPs": 2500.0, "fp64_TFLOPs": 78.6}

# HBM traffic of the row kernel, taken with rocprofv3 FETCH_SIZE / WRITE_SIZE
# counters and stored as text beside the sources it was measured on; it is
# reported only while those sources are unchanged.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "rows_mixed_kernel_k64_bf16_movielens_hbm.txt")
ROW_KERNEL_SOURCES = ("kernels_mixed.hip", "rowsolve.hpp", "rng.hpp", "common.hpp")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rows_kernel_flops(rows, nnz, K):
    """Algorithmic work of `rows` row updates with `nnz` ratings in all.

    FP32 (vector units or FP32 matrix cores): Cholesky K^3/3, two triangular
    solves 2 K^2, forming P K(K+1), right-hand side 2 nnz K.  BF16 matrix
    cores: the symmetric Gram nnz K(K+1).
    """
    valu = rows * (K ** 3 / 3.0 + 2.0 * K * K + K * (K + 1)) + 2.0 * nnz * K
    mfma = float(nnz) * K * (K + 1)
    return valu, mfma


def full_kernel_rows(counts, rank1_rows):
    """(rows, ratings) of one side that the full row kernel handles (the
    one-wavefront launch, with the heavy rows' pieces and their combine
    launch): every row but the rank-one tail of the count order."""
    c = np.sort(np.asarray(counts, np.int64))[::-1]
    keep = c[:c.size - int(rank1_rows)]
    return int(keep.size), int(keep.sum())


# The workloads of the paper's benchmarks (synthetic stand-ins); the metric
# is quoted on the MovieLens-shaped one, the others are opt-in.
WORKLOADS = {
    "movielens": dict(gen="movielens_like", precision="bf16",
                      text="MovieLens-20M-shaped synthetic: 138,493 x 26,744, 20M ratings, K=64, "
                           "BF16 gathers/Gram + FP32 Cholesky + FP64 hyper step, HIP-graph sweep"),
    "chembl": dict(gen="chembl_like", precision="fp32",
                   text="ChEMBL-shaped synthetic: 483,500 x 5,775, 1,023,952 ratings (97% of rows with one), K=32, "
                        "FP32 gathers/Gram/Cholesky + FP64 hyper step, HIP-graph sweep"),
    "netflix": dict(gen="netflix_like", precision="bf16",
                    text="Netflix-shaped synthetic: 480,189 x 17,770, 100M ratings, K=128, BF16 gathers/Gram on "
                         "matrix cores + FP32 Cholesky (four wavefronts per row) + FP64 hyper step, HIP-graph sweep"),
}


def row_kernel_digest():
    """sha256 over the sources the BF16 row kernel is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for name in ROW_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1705_10633_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """(HBM bytes per row-kernel launch, note) from the stored counter summary, or
    (None, reason) when it is missing or was taken on other kernel sources."""
    if not os.path.exists(TRAFFIC_PROFILE):
        return None, "no counter summary"
    fields = {}
    with open(TRAFFIC_PROFILE) as f:
        for line in f:
            m = re.match(r"^([a-z_0-9]+):\s*(\S+)", line)
            if m:
                fields[m.group(1)] = m.group(2)
    if fields.get("kernel_sources_sha256") != row_kernel_digest():
        return None, "row kernel changed since the counters were taken"
    return float(fields["hbm_bytes_per_launch"]), "FETCH_SIZE x %s + WRITE_SIZE x %s, mean of both launches" % (
        fields.get("fetch_scale", "?"), fields.get("write_scale", "?"))


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def time_sweeps(sampler, steps, warmup):
    import torch
    if warmup > 0:
        sampler.sweep(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    sampler.sweep(steps)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(stop) / steps, wall / steps * 1e3


def cpu_baseline(prob, n_sweeps=3, seed=2024, budget_s=15.0):
    """The FP64 oracle as it stands on the same workload, all host threads
    (row loops threaded, everything else serial): three whole sweeps when
    they fit the time budget, else the row updates of a uniform sample of the
    rows of both halves of one sweep."""
    from oracle import oracle as O
    nth = os.cpu_count() or 1
    R, K = prob.R, prob.K
    # ~4 GFLOP/s per thread for the plain loops: nnz K^2 + rows K^3/3 per half-sweep
    flops = 2.0 * R.nnz * K * K + (R.M + R.N) * K ** 3 / 3.0
    est = n_sweeps * flops / (4e9 * nth)
    if est <= budget_s:
        tape = O.philox_tape(seed, 0, n_sweeps, prob.M, prob.N, prob.K, prob.nu0)
        t0 = time.perf_counter()
        O.gibbs(prob, tape, n_sweeps=n_sweeps, burnin=0, nthreads=nth)
        t = time.perf_counter() - t0
        rows = n_sweeps * (prob.M + prob.N)
        return {"value": rows / t, "unit": "rows/s", "cores": nth, "kind": "oracle",
                "sample": f"{n_sweeps} whole FP64 oracle sweeps of the full workload (both halves, both "
                          f"Normal-Wishart steps and {prob.test_rows.size} held-out predictions per sweep): "
                          f"{rows} rows in {t:.1f} s wall on {nth} threads"}
    return row_sample(prob, nth, budget_s, seed, flops)


def row_sample(prob, nth, budget_s, seed, flops):
    """Oracle row updates of a uniform sample of the rows of both halves of one
    sweep, sized to about budget_s on nth threads."""
    from oracle import oracle as O
    R, K = prob.R, prob.K
    frac = min(1.0, max(1e-4, budget_s / (flops / (4e9 * nth))))
    rng = np.random.default_rng(seed)
    Lam = np.eye(K) * 2.0
    mu = np.zeros(K)
    total_rows, total_t = 0, 0.0
    for ptr, idx, val, other, n in ((R.row_ptr, R.col_idx, R.row_val, prob.V0, R.M),
                                    (R.col_ptr, R.row_idx, R.col_val, prob.U0, R.N)):
        pick = np.sort(rng.choice(n, size=max(1, int(frac * n)), replace=False))
        cnt = ptr[pick + 1] - ptr[pick]
        sp = np.zeros(pick.size + 1, np.int64)
        np.cumsum(cnt, out=sp[1:])
        sel = np.concatenate([np.arange(ptr[i], ptr[i + 1]) for i in pick])
        Z = rng.standard_normal((pick.size, K))
        t0 = time.perf_counter()
        O.half_sweep(sp, idx[sel], val[sel], other, prob.alpha, prob.mean_rating, Lam, mu, Z, nthreads=nth)
        total_t += time.perf_counter() - t0
        total_rows += pick.size
    return {"value": total_rows / total_t, "unit": "rows/s", "cores": nth, "kind": "oracle",
            "sample": f"FP64 oracle row updates of a uniform {frac * 100:.2g}% sample of the rows of both halves "
                      f"of one sweep ({total_rows} rows, {total_t:.1f} s wall, {nth} threads)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="movielens",
                    help="synthetic workload (the metric is quoted on movielens)")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--autotune", action="store_true",
                    help="time every candidate launch shape first and sweep with the fastest")
    ap.add_argument("--shape", default=None,
                    help="launch shape to sweep with, as JSON (bpmf_launch_shape fields)")
    ap.add_argument("--users-by-count", action="store_true",
                    help="renumber the users in descending rating count first (reordering of R for locality)")
    ap.add_argument("--only-timed", action="store_true",
                    help="run only warm-up and timed sweeps (for profiler runs)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.calib_copy:
        import torch
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": 1 << 30, "copies": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the sampler runs on one GPU only; --gpus must be 1"}))
        log("bench.py: the sampler and its kernels run on one GPU; multi-GPU sharding is not built")
        sys.exit(2)

    if args.autotune and args.shape:
        log("bench.py: --autotune and --shape exclude each other")
        sys.exit(2)

    import torch
    from paper_1705_10633_amd import synth
    from paper_1705_10633_amd.sampler import DeviceRatings, Sampler

    wl = WORKLOADS[args.workload]
    t0 = time.perf_counter()
    prob = getattr(synth, wl["gen"])()
    if args.users_by_count:
        prob = synth.relabel_users_by_count(prob)
    K = prob.K
    prec = wl["precision"]
    log(f"[bench] workload generated in {time.perf_counter() - t0:.1f} s: M={prob.M} N={prob.N} "
        f"nnz={prob.R.nnz} K={K} ({prob.note})")

    R32 = DeviceRatings(prob.R, val_dtype="float32")
    shape, tune_table, tune_fits = (json.loads(args.shape) if args.shape else {}), None, None
    if args.autotune:
        from paper_1705_10633_amd import autotune
        t0 = time.perf_counter()
        shape, tune_table = autotune.tune(
            R32, K, prob.U0.astype(np.float32), prob.V0.astype(np.float32),
            [prob.R.row_counts(), prob.R.col_counts()], precision=prec, sweeps=args.steps, warmup=3,
            alpha=prob.alpha, beta0=prob.beta0, nu0=prob.nu0, mean_rating=prob.mean_rating, seed=2024)
        tune_fits = autotune.variant_fits()
        for f in tune_fits:
            log(f"[bench] autotune variant {f['variant']}: {f['ms_per_sweep']:.3f} ms/sweep, row cost fit "
                f"a = {f['a_us_per_row']:.4g} us/row + b = {f['b_us_per_rating']:.4g} us/rating per launch")
        for c, ms in tune_table:
            log(f"[bench] autotune {ms:8.3f} ms/sweep  {c}")
        log(f"[bench] autotune: {len(tune_table)} shapes in {time.perf_counter() - t0:.1f} s, "
            f"kept {shape}")
    s = Sampler(R32, K, prob.U0.astype(np.float32), prob.V0.astype(np.float32), precision=prec,
                alpha=prob.alpha, beta0=prob.beta0, nu0=prob.nu0, mean_rating=prob.mean_rating,
                seed=2024, burnin=0, test_rows=prob.test_rows, test_cols=prob.test_cols,
                use_graph=True, shape=shape)
    rows_per_sweep = prob.M + prob.N
    ms_dev, ms_wall = time_sweeps(s, args.steps, args.warmup)
    value = rows_per_sweep / (ms_wall * 1e-3)
    log(f"[bench] {prec} graph sweeps: {ms_wall:.3f} ms/sweep wall ({ms_dev:.3f} ms by events) "
        f"-> {value:.4g} rows/s")
    if args.only_timed:
        print(json.dumps({"metric": f"Gibbs rows sampled/sec at K={K}", "value": value, "ms_per_step": ms_wall,
                          "workload": args.workload, "launch_shape": shape,
                          "autotune": None if tune_table is None else
                          {"timed": [{"shape": c, "ms_per_sweep": ms} for c, ms in tune_table],
                           "kernel_variant_fits": tune_fits}}))
        return

    # four more runs of the same number of sweeps, for the spread between runs
    runs = [ms_wall] + [time_sweeps(s, args.steps, 0)[1] for _ in range(4)]
    log(f"[bench] five runs of {args.steps} sweeps: " + " ".join(f"{r:.3f}" for r in runs) +
        f" ms/sweep (median {float(np.median(runs)):.3f})")

    # per-kernel durations over the same number of sweeps, events on the launch
    # stream; the pass runs twice and the second is kept (after any idle gap the
    # clocks ramp up during the first, which then reads up to ~10 % slow)
    s.set_timing(True)
    s.sweep(args.steps)
    s.timing(reset=True)
    s.sweep(args.steps)
    tm = s.timing(reset=True)
    s.set_timing(False)
    info = s.info()
    for k, (ms, n) in tm.items():
        log(f"[bench]   {k:15s} {ms / max(n, 1) * 1e3:9.1f} us/launch x {n}")
    rc, cc = prob.R.row_counts(), prob.R.col_counts()
    # The dominant kernel: the full row kernel (one wavefront per row at K <= 64,
    # four at K = 128), its users' and movies' launches and, where heavy rows are
    # cut into pieces, their combine launch; the rank-one tail runs in kernels of
    # its own and is neither timed nor counted here.
    per_launch = {}
    valu = mfma = 0.0
    t_rows = 0.0
    launches = 0
    for side, cls, counts in ((0, "rows_users", rc), (1, "rows_movies", cc)):
        rows, nnz = full_kernel_rows(counts, info["rank1_rows"][side])
        v, m = rows_kernel_flops(rows, nnz, K)
        ms, n = tm[cls]
        us = ms / max(n, 1) * 1e3
        per_launch[cls] = {"rows": rows, "ratings": nnz, "avg_us": us, "fp32_flop": v, "bf16_mfma_flop": m,
                           "fp32_TFLOPs": v / (us * 1e-6) / 1e12 if us > 0 else None,
                           "fp32_frac": v / (us * 1e-6) / 1e12 / MI355X["fp32_TFLOPs"] if us > 0 else None,
                           "bf16_mfma_frac": m / (us * 1e-6) / 1e12 / MI355X["bf16_TFLOPs"] if us > 0 else None}
        valu += v
        mfma += m
        t_rows += ms / args.steps
        launches += n / args.steps
    if tm["rows_heavy"][1]:
        t_rows += tm["rows_heavy"][0] / args.steps
        launches += tm["rows_heavy"][1] / args.steps
        per_launch["rows_heavy"] = {"avg_us": tm["rows_heavy"][0] / tm["rows_heavy"][1] * 1e3,
                                    "note": "factorisation of the heavy rows whose Gram ran in pieces"}
    avg_launch_ms = t_rows / launches
    achieved = (valu / launches) / (avg_launch_ms * 1e-3) / 1e12
    mfma_achieved = (mfma / launches) / (avg_launch_ms * 1e-3) / 1e12
    traffic, traffic_note = measured_traffic() if args.workload == "movielens" else (
        None, "counter summary is for the MovieLens-shaped row kernel only")
    peak = MI355X["fp32_TFLOPs"]
    roofline = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": traffic}
    if K <= 64:
        kname = f"rows_mixed_kernel<{32 if K <= 32 else 64},{prec}>"
    else:
        kname = "rows_mixed128_kernel"
    detail = {"kernel": kname, "avg_launch_us": avg_launch_ms * 1e3,
              "valu_flop_per_sweep": valu, "mfma_bf16_flop_per_sweep": mfma,
              "mfma_bf16_achieved_TFLOPs": mfma_achieved,
              "mfma_bf16_frac": mfma_achieved / MI355X["bf16_TFLOPs"],
              "fp32_frac_of_unpacked_peak": achieved / (MI355X["fp32_TFLOPs"] / 2),
              "per_launch": per_launch,
              "per_kernel_us": {k: v[0] / max(v[1], 1) * 1e3 for k, v in tm.items()},
              "launch_shape_info": {k: info[k] for k in ("rank1_rows", "heavy_rows", "pieces", "kernel_variant")},
              "fallback_rows": info["fallback_rows"],
              "traffic_note": traffic_note,
              "hbm_GBs_at_traffic": (traffic / (avg_launch_ms * 1e-3) / 1e9) if traffic else None}

    fp64 = None
    if not args.no_fp64:
        del s
        torch.cuda.empty_cache()
        R64 = DeviceRatings(prob.R, val_dtype="float64")
        s64 = Sampler(R64, K, prob.U0, prob.V0, precision="fp64", alpha=prob.alpha, beta0=prob.beta0,
                      nu0=prob.nu0, mean_rating=prob.mean_rating, seed=2024, burnin=0,
                      test_rows=prob.test_rows, test_cols=prob.test_cols, use_graph=True)
        ms64_dev, ms64 = time_sweeps(s64, args.fp64_steps, 1)
        fp64 = {"value": rows_per_sweep / (ms64 * 1e-3), "unit": "rows/s", "ms_per_step": ms64,
                "path": "plain FP64, one 256-thread workgroup per row"}
        log(f"[bench] fp64 plain sweeps: {ms64:.2f} ms/sweep -> {fp64['value']:.4g} rows/s "
            f"(bf16 path is {value / fp64['value']:.1f}x)")
        del s64, R64
        torch.cuda.empty_cache()

    serving = None
    if not args.no_serving:
        try:
            from paper_1705_10633_amd import serving as srv
            serving = srv.bench_foldin(seconds=args.serve_seconds, log=log)
        except (ImportError, AttributeError) as e:
            log(f"[bench] serving skipped: {e}")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(prob)
        log(f"[bench] cpu baseline: {cpu['value']:.4g} rows/s ({cpu['sample']})")
        R = prob.R
        one = row_sample(prob, 1, 4.0, 2025, 2.0 * R.nnz * K * K + (R.M + R.N) * K ** 3 / 3.0)
        cpu["value_1core"] = one["value"]
        cpu["sample_1core"] = one["sample"]
        cpu["host_cpu"] = host_cpu_model()
        log(f"[bench] cpu baseline, one thread: {one['value']:.4g} rows/s ({one['sample']}); host {cpu['host_cpu']}")

    out = {
        "metric": "Gibbs rows sampled/sec at K=64 (vs plain FP64 path) + p50/p99 fold-in latency",
        "value": value, "unit": "rows/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_wall, "ms_per_step_runs": runs, "ms_per_step_median_of_runs": float(np.median(runs)),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic",
        "config": {"workload": wl["text"],
                   "M": prob.M, "N": prob.N, "nnz": prob.R.nnz, "K": K,
                   "rows_per_step": rows_per_sweep, "n_test": int(prob.test_rows.size)},
        "roofline": roofline,
        "roofline_detail": detail,
        "cpu_baseline": cpu,
        "fp64_plain": fp64,
        "speedup_vs_fp64_plain": (value / fp64["value"]) if fp64 else None,
        "serving": serving,
        "launch_shape": shape,
    }
    if tune_table is not None:
        out["autotune"] = {"timed": [{"shape": c, "ms_per_sweep": ms} for c, ms in tune_table],
                           "kernel_variant_fits": tune_fits}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
