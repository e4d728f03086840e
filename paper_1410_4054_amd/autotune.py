"""Autotuner for the batched solver's launch shape.

The batched kernel has three shape parameters: the workgroup size (rows a
workgroup sweeps per step: 256, 512 or 1024 threads), the row limit under
which a system keeps its work vectors in LDS (which also fixes how many
workgroups fit on a CU), and the team size (workgroups that solve one large
system together; 1 = every system alone).  tune() times every candidate on
the batch itself (same right-hand side, same start) and keeps the fastest;
results are cached in a JSON file keyed by device and batch shape, so a
batch of the same shape is tuned once.

    best = tune(batch, b, x0, rtol=1e-10)   # {'workgroup': ..., 'lds_rows': ..., 'team': ...}
"""
from __future__ import annotations

import json
import os
import time

CANDIDATES = ([{"workgroup": wg, "lds_rows": lds, "team": 1} for wg in (256, 512, 1024) for lds in (0, 2048, -1)]
              + [{"workgroup": 1024, "lds_rows": 0, "team": t} for t in (4, 8, 16, 32)])


def default_cache_path() -> str:
    return os.environ.get("FK_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "fk", "autotune.json")


def batch_key(batch, rtol: float) -> str:
    import torch

    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    sizes = batch.sys_ptr[1:] - batch.sys_ptr[:-1]
    return (f"{dev}|batch-v2|count={batch.count}|n={batch.n}|max_rows={int(sizes.max())}"
            f"|min_rows={int(sizes.min())}|rtol={rtol:g}")


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def tune(batch, b, x0, rtol: float = 1e-10, candidates=None, reps: int = 1, cache_path: str | None = None,
         use_cache: bool = True) -> dict:
    """Fastest {'workgroup', 'lds_rows', 'team'} for this batch; also returns the
    timings under 'seconds' (candidate index -> seconds) when measured."""
    import torch

    cache_path = cache_path or default_cache_path()
    key = batch_key(batch, rtol)
    cache = _load(cache_path)
    if use_cache and key in cache:
        return dict(cache[key], cached=True)
    candidates = candidates or CANDIDATES
    x = torch.empty_like(x0)
    timings = []
    for cand in candidates:
        best = float("inf")
        for _ in range(max(1, reps)):
            x.copy_(x0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            batch.solve(b, x, rtol=rtol, **cand)
            best = min(best, time.perf_counter() - t0)
        timings.append(best)
    i = min(range(len(candidates)), key=lambda k: timings[k])
    result = dict(candidates[i])
    result["seconds"] = {json.dumps(c): t for c, t in zip(candidates, timings)}
    cache[key] = {k: v for k, v in result.items()}
    try:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1)
    except OSError:
        pass
    result["cached"] = False
    return result
