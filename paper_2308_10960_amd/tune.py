"""Autotuner of the launch parameters (schedule, unroll depth, panel order,
persistent grids).

For one device-resident matrix it times every candidate with the library's
own HIP-event kernel timing, keeps the fastest, and can store the choice in
a tune cache (one "key params" line per kind of matrix) that hm_build_plan
reads when the plan is built with tune=1.
"""

from __future__ import annotations

import os

from . import hm

CANDIDATES = ["schedule=0 unroll=4 order=0 persist=0", "schedule=0 unroll=8 order=0 persist=0",
              "schedule=0 unroll=8 order=1 persist=0", "schedule=0 unroll=8 order=1 persist=4",
              "schedule=0 unroll=8 order=1 persist=8", "schedule=1 unroll=4 order=0 persist=0",
              "schedule=1 unroll=8 order=0 persist=0", "schedule=1 unroll=8 order=0 persist=8"]
# the batched path only depends on the row-panel order
BATCH_CANDIDATES = ["schedule=0 unroll=8 order=0 persist=0", "schedule=0 unroll=8 order=1 persist=0"]


def _time(D, step, reps: int) -> float:
    import torch
    hm.hm_profile_begin(D.handle, reps)
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    ms, calls = hm.hm_profile_end(D.handle)
    return sum(ms) / max(calls, 1)


def tune(D, step, candidates=CANDIDATES, reps: int = 10, warmup: int = 3):
    """Time every candidate on matrix D with the callable ``step`` (one
    product); leave D on the fastest and return (best, {params: ms})."""
    import torch
    times = {}
    for c in candidates:
        hm.hm_matrix_set_launch(D.handle, c)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        times[c] = _time(D, step, reps)
    best = min(times, key=times.get)
    hm.hm_matrix_set_launch(D.handle, best)
    return best, times


def write_cache(path: str, key: str, params: str) -> None:
    """Insert or replace the line for ``key`` in the tune cache at ``path``."""
    lines = []
    if os.path.exists(path):
        with open(path) as f:
            lines = [l for l in f.read().splitlines() if l and not l.startswith(key + " ")]
    lines.append(f"{key} {params}")
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.write("\n".join(lines) + "\n")
    os.replace(tmp, path)
