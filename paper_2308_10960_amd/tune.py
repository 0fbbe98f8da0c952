"""Autotuner of the launch parameters (schedule, unroll depth, panel order,
persistent grids) and of the column-tile shape (rows per column chunk,
groups per tile, one or several storage formats per tile) with the way
column tiles are spread over waves.

For one device-resident matrix it times every launch candidate with the
library's own HIP-event kernel timing and keeps the fastest; tile shapes
change the store layout, so each shape candidate is a plan and an upload of
its own.  The choice goes into a tune cache (one "key params" line per kind
of matrix) that hm_build_plan reads when the plan is built with tune=1.
"""

from __future__ import annotations

import os

from . import hm

CANDIDATES = ["schedule=0 unroll=4 order=0 persist=0", "schedule=0 unroll=8 order=0 persist=0",
              "schedule=0 unroll=4 order=1 persist=0",
              "schedule=0 unroll=8 order=1 persist=0", "schedule=0 unroll=8 order=1 persist=4",
              "schedule=0 unroll=8 order=1 persist=8", "schedule=1 unroll=4 order=0 persist=0",
              "schedule=1 unroll=8 order=0 persist=0", "schedule=1 unroll=8 order=0 persist=8"]
# the batched path: row-panel order, and FP32 column tiles as 8-byte slots
# (colb=0) or 16-byte groups (colb=1) per lane; none changes a bit
BATCH_CANDIDATES = ["schedule=0 unroll=8 order=0 persist=0 colb=0", "schedule=0 unroll=8 order=1 persist=0 colb=0",
                    "schedule=0 unroll=8 order=0 persist=0 colb=1", "schedule=0 unroll=8 order=1 persist=0 colb=1"]
# column-tile shapes (chunk rows, tile groups, tile_mix: 1 one format per
# tile, 2 up to four; the same store for a matrix of one format)
SHAPE_CANDIDATES = [(512, 64, 1), (256, 64, 1), (128, 64, 1), (64, 64, 1), (512, 32, 1), (256, 32, 1),
                    (512, 64, 2), (256, 64, 2), (128, 64, 2)]
# single-RHS column tiles on a workgroup each, per launch class, or on a
# wave each (timed for every shape: the best choice depends on tile size)
COLW_VARIANTS = ("colw=0", "colw=1", "colw=2")


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


def tune_shape(make, step_of, launch: str, candidates=SHAPE_CANDIDATES, variants=("",), reps: int = 10,
               warmup: int = 3):
    """Time every tile shape: ``make(chunk, tile, mix)`` builds and uploads
    the matrix with that shape, ``step_of(D)`` returns one product of it.
    Each runs with the launch parameters ``launch``, followed by each of
    ``variants`` (extra launch parameters, "" for none).  Returns (best
    (chunk, tile, mix, variant), {(chunk, tile, mix, variant): ms}); the
    matrices are released."""
    import torch
    times = {}
    for chunk, tile, mix in candidates:
        D = make(chunk, tile, mix)
        try:
            step = step_of(D)
            for v in variants:
                hm.hm_matrix_set_launch(D.handle, (launch + " " + v).strip())
                for _ in range(warmup):
                    step()
                torch.cuda.synchronize()
                times[(chunk, tile, mix, v)] = _time(D, step, reps)
        finally:
            D.close()
            torch.cuda.empty_cache()
    return min(times, key=times.get), times


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
