"""Launch-shape autotuner for the mixed-precision sweep.

The row kernels' tiles are fixed by K (padded to 32, 64 or 128) and by the
register budget of one wavefront per row; what depends on the rating matrix
is how the rating-count-ordered row table is cut into launches
(bpmf_launch_shape): which heavy rows are split into pieces and how long the
pieces are, and which rows with few ratings take the rank-one kernels.  The
paper models a row's cost as a fixed part plus a part per rating and splits
heavy items across workers (Section 4.2); the best cut on a GPU depends on
the count distribution, so it is measured rather than modelled: every
candidate shape runs whole sweeps on the device, timed with events on the
sampler's stream, and the fastest is kept.

Every candidate samples the same conditionals; results differ only within
FP32 rounding (summation order of the pieces, rank-one updates against a
fresh factorisation), so the tuned shape is a speed choice, not a numerical
one.  Tuning changes nothing in the library: the caller passes the chosen
shape to the Sampler it keeps.
"""
from __future__ import annotations

import itertools
import json
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from .sampler import DeviceRatings, Sampler

# the largest rank1_max_ratings the library accepts
RANK1_MAX = 4


def candidate_shapes(row_counts: Sequence[np.ndarray], K: int) -> List[dict]:
    """Candidate launch shapes for a matrix with the given per-side rating
    counts (users' and movies'), the built-in choice ({}) first.  Only knobs
    that change the launches of this matrix are varied: heavy-row splits when
    some row has >= 1024 ratings, rank-one limits at counts that occur."""
    if K > 64:
        return [{}]
    counts = np.concatenate([np.asarray(c, np.int64) for c in row_counts])
    top = int(counts.max()) if counts.size else 0
    heavy: List[dict] = [{"heavy_split": -1}]
    for hmin, piece in itertools.product((1024, 2048, 4096), (256, 512, 1024)):
        if top >= hmin:
            heavy.append({"heavy_split": 1, "heavy_min_ratings": hmin, "piece_min_ratings": piece})
    small: List[dict] = [{"rank1_max_ratings": -1}]
    for lim in range(1, RANK1_MAX + 1):
        # a limit with no row at exactly that count launches as the one below it
        if (counts == lim).any():
            small.append({"rank1_max_ratings": lim, "rank1_split": 1})
    out = [{}]
    for h, s in itertools.product(heavy, small):
        c = {**h, **s}
        if c not in out:
            out.append(c)
    return out


def time_shape(ratings: DeviceRatings, K: int, U0, V0, shape: dict, precision: str = "bf16",
               sweeps: int = 10, warmup: int = 3, **sampler_kw) -> float:
    """Milliseconds per sweep of a sampler built with this launch shape
    (device generator, graph replay), from the same starting state."""
    import torch
    s = Sampler(ratings, K, U0, V0, precision=precision, use_graph=True, shape=shape, **sampler_kw)
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


def tune(ratings: DeviceRatings, K: int, U0, V0, row_counts: Sequence[np.ndarray],
         precision: str = "bf16", candidates: Optional[List[dict]] = None, sweeps: int = 10,
         warmup: int = 3, **sampler_kw) -> Tuple[dict, List[Tuple[dict, float]]]:
    """Times every candidate shape and returns (fastest, [(shape, ms per sweep)]).
    Ties keep the earlier candidate, so the built-in choice wins unless a
    shape is strictly faster."""
    if candidates is None:
        candidates = candidate_shapes(row_counts, K)
    table = []
    for c in candidates:
        table.append((c, time_shape(ratings, K, U0, V0, c, precision, sweeps, warmup, **sampler_kw)))
    best = min(range(len(table)), key=lambda i: (table[i][1], i))
    return table[best][0], table


def save(path: str, shape: dict, table: List[Tuple[dict, float]], key: Dict) -> None:
    """Writes a tuning result (the problem's key, the chosen shape and every
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
