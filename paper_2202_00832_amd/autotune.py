"""Tile-shape autotuner for the batched full-route evaluation (lo_batch_*).

The tile shape of a system in a batch is its number of Cholesky vectors per
work item ("chunk").  Small chunks balance the persistent kernel's work list
better; large ones spend less per item on the staging prologue and the
exchange epilogue.  Systems are grouped in buckets of similar shape
(orbital blocks NB = ceil(n/16), basis size rounded up to 64, Cholesky count
rounded up to 256).  Starting from the planner's default, the tuner visits the
buckets in decreasing order of work and, for each, times the whole batch with
the bucket's chunks scaled by a few factors, keeping the fastest (coordinate
descent; every configuration tried is a valid plan, so the result is never
slower than the default on the measurements taken).  The table maps bucket
keys to chunk lengths and can be stored as JSON and reused.
"""
from __future__ import annotations

import json
import math

import numpy as np

from . import lofqmc


def bucket_key(M: int, n: int, X: int) -> str:
    return "nb%d-m%d-x%d" % ((n + 15) // 16, 64 * math.ceil(M / 64), 256 * math.ceil(X / 256))


def _shape(sd):
    X, M, n = sd["lbar"].shape
    return M, n, X, sd["theta"].shape[0]


def time_batch(ctx, systems, chunk, reps: int = 3) -> float:
    """Milliseconds per evaluation (best of `reps`, after one untimed run)."""
    import torch
    b = lofqmc.Batch(ctx, systems, chunk)
    try:
        b.execute()
        best = float("inf")
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            b.execute()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best
    finally:
        b.close()


def tune(ctx, systems, factors=(0.25, 0.5, 2.0, 4.0), reps: int = 3, log=None) -> dict:
    """Returns {"table": {bucket: chunk}, "chunk": [per system], "ms": best,
    "default_ms": time of the planner's default, "trials": [...]}."""
    base = lofqmc.Batch(ctx, systems)
    default = base.info()["chunk"].astype(np.int64)
    base.close()
    shapes = [_shape(sd) for sd in systems]
    keys = [bucket_key(M, n, X) for (M, n, X, _) in shapes]
    work = {}
    for (M, n, X, nw), k in zip(shapes, keys):
        work[k] = work.get(k, 0.0) + M * ((n + 15) // 16) ** 2 * X * nw
    chunk = default.copy()
    best = time_batch(ctx, systems, chunk, reps)
    default_ms = best
    trials = [{"bucket": None, "factor": 1.0, "ms": best}]
    for k in sorted(work, key=lambda q: -work[q]):
        idx = [i for i, kk in enumerate(keys) if kk == k]
        keep = chunk.copy()
        for f in factors:
            cand = keep.copy()
            for i in idx:
                X = shapes[i][2]
                cand[i] = int(min(max(1, round(keep[i] * f)), X))
            if np.array_equal(cand, keep):
                continue
            ms = time_batch(ctx, systems, cand, reps)
            trials.append({"bucket": k, "factor": f, "ms": ms})
            if log:
                log("autotune %s x%g: %.3f ms" % (k, f, ms))
            if ms < best:
                best, chunk = ms, cand
    table = {keys[i]: int(chunk[i]) for i in range(len(systems))}
    return {"table": table, "chunk": [int(c) for c in chunk], "ms": best, "default_ms": default_ms,
            "trials": trials}


def chunks_from_table(systems, table: dict):
    """Chunk per system from a stored table (None for buckets it lacks)."""
    out = []
    for sd in systems:
        M, n, X, _ = _shape(sd)
        out.append(int(table.get(bucket_key(M, n, X), 0)))
    return out


def save_table(path: str, table: dict):
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


def load_table(path: str) -> dict:
    with open(path) as f:
        return json.load(f)
