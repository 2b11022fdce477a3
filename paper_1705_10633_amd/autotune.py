"""Autotuner of the mixed-precision sweep: kernel variant and launch shape.

What depends on the rating matrix is (bpmf_launch_shape):
  * the code variant of the one-wavefront row kernel at 32 < K <= 64
    (kernel_variant: where the Cholesky's trailing updates run, and the
    register budget: 1 matrix cores / 4 wavefronts per SIMD, 2 vector units,
    3 matrix cores / 3 wavefronts per SIMD);
  * how the rating-count-ordered row table is cut into launches: which heavy
    rows are split into pieces and how long the pieces are, and which rows
    with few ratings take the rank-one kernels.

The paper models the cost of updating an item as a fixed part plus a part per
rating (Section 4.2).  The tuner fits that model, t = a rows + b ratings, to
each kernel variant's two row launches (users and movies, timed with events
on the sampler's stream), keeps the variant that sweeps fastest, and uses
its fitted a, b to decide whether heavy rows need splitting at all: a launch
over rows sorted by count, spread over S concurrent wavefront slots, ends
no earlier than max(total cost / S, cost of its heaviest row), so splits are
candidates only when the heaviest row's predicted cost a + b n_max exceeds
the launch's share total / S.  The remaining candidates run whole sweeps on
the device and the fastest is kept.

Every candidate samples the same conditionals; results differ only within
FP32 rounding (summation order of the pieces, rank-one updates against a
fresh factorisation, the order of the trailing updates), so the tuned shape
is a speed choice, not a numerical one.  Tuning changes nothing in the
library: the caller passes the chosen shape to the Sampler it keeps.  A
result can be cached in a JSON file keyed by the GPU architecture, K, the
precision and the problem's rating-count histogram; Sampler(shape="auto")
consults the cache before tuning and records what it tuned.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from .sampler import DeviceRatings, Sampler

# the largest rank1_max_ratings the library accepts
RANK1_MAX = 4
# kernel_variant values of the one-wavefront row kernel at 32 < K <= 64
VARIANTS = (1, 2, 3)
# concurrent one-wavefront rows on the device (256 CUs x 4 SIMDs x 4 waves)
WAVE_SLOTS = 4096


def kernel_variants(K: int) -> List[int]:
    return list(VARIANTS) if 32 < K <= 64 else [0]


def candidate_shapes(row_counts: Sequence[np.ndarray], K: int, heavy: bool = True,
                     variant: int = 0) -> List[dict]:
    """Candidate launch shapes for a matrix with the given per-side rating
    counts (users' and movies'), the built-in choice ({} or just the variant)
    first.  Only knobs that change the launches of this matrix are varied:
    heavy-row splits when some row has >= 1024 ratings (and `heavy`), rank-one
    limits at counts that occur."""
    if K > 64:
        return [{}]
    counts = np.concatenate([np.asarray(c, np.int64) for c in row_counts])
    top = int(counts.max()) if counts.size else 0
    heavy_c: List[dict] = [{"heavy_split": -1}]
    if heavy:
        for hmin, piece in itertools.product((1024, 2048, 4096), (256, 512, 1024)):
            if top >= hmin:
                heavy_c.append({"heavy_split": 1, "heavy_min_ratings": hmin, "piece_min_ratings": piece})
    small: List[dict] = [{"rank1_max_ratings": -1}]
    for lim in range(1, RANK1_MAX + 1):
        # a limit with no row at exactly that count launches as the one below it
        if (counts == lim).any():
            small.append({"rank1_max_ratings": lim, "rank1_split": 1})
    base = {"kernel_variant": variant} if variant else {}
    out = [dict(base)]
    for h, s in itertools.product(heavy_c, small):
        c = {**base, **h, **s}
        if c not in out:
            out.append(c)
    return out


def _sampler(ratings: DeviceRatings, K: int, U0, V0, shape: dict, precision: str, **kw) -> Sampler:
    return Sampler(ratings, K, U0, V0, precision=precision, use_graph=True, shape=shape, **kw)


def time_shape(ratings: DeviceRatings, K: int, U0, V0, shape: dict, precision: str = "bf16",
               sweeps: int = 10, warmup: int = 3, **sampler_kw) -> float:
    """Milliseconds per sweep of a sampler built with this launch shape
    (device generator, graph replay), from the same starting state."""
    import torch
    s = _sampler(ratings, K, U0, V0, shape, precision, **sampler_kw)
    stream = torch.cuda.current_stream()
    s.sweep(warmup)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    s.sweep(sweeps)
    t1.record(stream)
    t1.synchronize()
    ms = t0.elapsed_time(t1) / sweeps
    del s
    return ms


def launch_rows(row_counts: Sequence[np.ndarray], info: dict) -> List[Tuple[int, int]]:
    """(entries, ratings) of the users' and the movies' one-wavefront launches
    under the launch shape a sampler reported in info(): rows in descending
    count order without the rank-one tail; a heavy row counts as its pieces
    (whose sums are factored in a launch of their own)."""
    out = []
    for side, c in enumerate(row_counts):
        c = np.sort(np.asarray(c, np.int64))[::-1]
        lo, hi = int(info["heavy_rows"][side]), c.size - int(info["rank1_rows"][side])
        # the heavy rows' pieces gather and multiply in the same launch
        out.append((hi - lo + int(info["pieces"][side]), int(c[:hi].sum())))
    return out


def fit_cost(points: Sequence[Tuple[int, int, float]]) -> Tuple[float, float]:
    """Least-squares a, b of t = a rows + b ratings over (rows, ratings, t)
    points (t in microseconds); a in us per row, b in us per rating."""
    A = np.array([[r, n] for r, n, _ in points], np.float64)
    t = np.array([x for _, _, x in points], np.float64)
    (a, b), *_ = np.linalg.lstsq(A, t, rcond=None)
    return float(a), float(b)


def time_variant(ratings: DeviceRatings, K: int, U0, V0, row_counts, variant: int, precision: str,
                 sweeps: int, warmup: int, **sampler_kw) -> dict:
    """Whole-sweep time of a kernel variant with the built-in cuts, and its
    fitted fixed-plus-per-rating row cost from per-launch event timings."""
    import torch
    shape = {"kernel_variant": variant} if variant else {}
    s = _sampler(ratings, K, U0, V0, shape, precision, **sampler_kw)
    stream = torch.cuda.current_stream()
    s.sweep(warmup)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    s.sweep(sweeps)
    t1.record(stream)
    t1.synchronize()
    ms = t0.elapsed_time(t1) / sweeps
    s.set_timing(True)
    s.sweep(sweeps)
    tm = s.timing(reset=True)
    s.set_timing(False)
    pts = []
    for (rows, nnz), cls in zip(launch_rows(row_counts, s.info()), ("rows_users", "rows_movies")):
        total, n = tm[cls]
        if n and rows:
            pts.append((rows, nnz, total / n * 1e3))
    del s
    a, b = fit_cost(pts) if len(pts) == 2 else (float("nan"), float("nan"))
    return {"variant": variant, "ms_per_sweep": ms, "a_us_per_row": a, "b_us_per_rating": b,
            "launches": [{"rows": r, "ratings": n, "us": t} for r, n, t in pts]}


def heavy_split_pays(row_counts: Sequence[np.ndarray], a: float, b: float, slots: int = WAVE_SLOTS) -> bool:
    """Whether some side's heaviest row outlasts its launch's share of the
    work under the cost model (a per row, b per rating, `slots` rows at once).
    A fit that is not a cost (not finite, a < 0 or b <= 0: the two launches
    did not follow the model, e.g. when rows of very different kinds share a
    launch) rules nothing out."""
    if not (np.isfinite(a) and np.isfinite(b)) or a < 0 or b <= 0:
        return True
    for c in row_counts:
        c = np.asarray(c, np.float64)
        if c.size == 0:
            continue
        cost = a + b * c
        if cost.max() > cost.sum() / slots:
            return True
    return False


def tune(ratings: DeviceRatings, K: int, U0, V0, row_counts: Sequence[np.ndarray],
         precision: str = "bf16", candidates: Optional[List[dict]] = None, sweeps: int = 10,
         warmup: int = 3, **sampler_kw) -> Tuple[dict, List[Tuple[dict, float]]]:
    """Returns (fastest shape, [(shape, ms per sweep)] of every shape timed).
    Without `candidates`: the kernel variants first (built-in cuts, with the
    cost model fitted to each; see variant_fits()), then the cut candidates
    of the fastest variant that the model leaves in.  Ties keep the earlier
    candidate, so the built-in choice wins unless a shape is strictly faster."""
    global _last_fits
    table: List[Tuple[dict, float]] = []
    _last_fits = []
    if candidates is None:
        variants = kernel_variants(K)
        for v in variants:
            f = time_variant(ratings, K, U0, V0, row_counts, v, precision, sweeps, warmup, **sampler_kw)
            _last_fits.append(f)
            table.append(({"kernel_variant": v} if v else {}, f["ms_per_sweep"]))
        best_v = min(range(len(variants)), key=lambda i: (_last_fits[i]["ms_per_sweep"], i))
        fv = _last_fits[best_v]
        candidates = [c for c in candidate_shapes(row_counts, K,
                                                   heavy=heavy_split_pays(row_counts, fv["a_us_per_row"],
                                                                          fv["b_us_per_rating"]),
                                                   variant=fv["variant"])
                      if c not in [t[0] for t in table]]
    for c in candidates:
        table.append((c, time_shape(ratings, K, U0, V0, c, precision, sweeps, warmup, **sampler_kw)))
    best = min(range(len(table)), key=lambda i: (table[i][1], i))
    return table[best][0], table


_last_fits: List[dict] = []


def variant_fits() -> List[dict]:
    """The kernel-variant timings and fitted a, b of the last tune() call."""
    return list(_last_fits)


def problem_key(row_counts: Sequence[np.ndarray], K: int, precision: str, arch: str) -> Dict:
    """Cache key: GPU architecture, K, precision, sizes and a digest of both
    sides' rating-count histograms (counts binned by powers of two)."""
    h = hashlib.sha256()
    sizes = []
    for c in row_counts:
        c = np.asarray(c, np.int64)
        sizes.append(int(c.size))
        bins = np.bincount(np.floor(np.log2(np.maximum(c, 1))).astype(np.int64) + (c > 0), minlength=32)
        h.update(bins.astype(np.int64).tobytes())
    return {"arch": arch, "K": int(K), "precision": precision, "rows": sizes,
            "ratings": int(np.asarray(row_counts[0]).sum()), "histogram": h.hexdigest()[:16]}


def cache_path() -> str:
    return os.environ.get("BPMF_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "bpmf",
                                                             "launch_shapes.json")


def cache_lookup(key: Dict, path: Optional[str] = None) -> Optional[dict]:
    """The cached shape for this key, or None."""
    try:
        with open(path or cache_path()) as f:
            entries = json.load(f)
    except (OSError, ValueError):
        return None
    for e in entries if isinstance(entries, list) else []:
        if e.get("key") == key:
            return e.get("shape")
    return None


def cache_store(key: Dict, shape: dict, table: List[Tuple[dict, float]], fits: List[dict],
                path: Optional[str] = None) -> None:
    """Adds (or replaces) the entry for this key."""
    path = path or cache_path()
    try:
        with open(path) as f:
            entries = json.load(f)
        if not isinstance(entries, list):
            entries = []
    except (OSError, ValueError):
        entries = []
    entries = [e for e in entries if e.get("key") != key]
    entries.append({"key": key, "shape": shape, "fits": fits,
                    "table": [{"shape": c, "ms_per_sweep": ms} for c, ms in table]})
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(entries, f, indent=1)
    os.replace(tmp, path)


def save(path: str, shape: dict, table: List[Tuple[dict, float]], key: Dict) -> None:
    """Writes one tuning result (the problem's key, the chosen shape and every
    timing) as JSON."""
    with open(path, "w") as f:
        json.dump({"key": key, "shape": shape,
                   "table": [{"shape": c, "ms_per_sweep": ms} for c, ms in table]}, f, indent=1)


def load(path: str, key: Dict) -> Optional[dict]:
    """The stored shape if the file's key matches, else None."""
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    return d["shape"] if d.get("key") == key else None
