"""Tile size per size bucket for the batched factorisation.

Every problem of a batch runs in one workgroup, so the best tile size depends
on the problem's size only: small tiles waste less zero padding, large ones
run more of the work on the matrix cores.  ``tune`` times each candidate tile
size on sample problems of every bucket (a batch of same-bucket problems, the
median of a few launches) and keeps the fastest; ``tile_for`` reads the table
(a tuned one if given, else the built-in one).  Buckets are by n (columns),
the dimension that sets the number of tile columns and the panel length.
"""
from __future__ import annotations

import json
import math
import time
from typing import Callable, Sequence

# (lowest n of the bucket, tile size); buckets run up to the next entry's n
DEFAULT_TABLE = [(0, 16), (32, 32), (64, 64)]
CANDIDATES = (16, 32, 64, 128)
BUCKETS = (0, 16, 32, 64, 128, 256)


def tile_for(n: int, table: Sequence[tuple[int, int]] | None = None) -> int:
    tab = sorted(table or DEFAULT_TABLE)
    b = tab[0][1]
    for lo, tb in tab:
        if n >= lo:
            b = tb
    return b


def tune(sample: Callable[[int, int], list[tuple[int, int]]], time_batch: Callable[[list, int], float],
         candidates: Sequence[int] = CANDIDATES, buckets: Sequence[int] = BUCKETS, reps: int = 3) -> list[tuple[int, int]]:
    """sample(lo, hi) -> shapes with lo <= n < hi; time_batch(shapes, b) ->
    seconds for one launch of those shapes all with tile size b.  Returns a
    table for tile_for, with neighbouring buckets of the same choice merged."""
    table = []
    edges = list(buckets) + [math.inf]
    for lo, hi in zip(edges[:-1], edges[1:]):
        shapes = sample(lo, hi)
        if not shapes:
            continue
        best, best_t = None, math.inf
        for b in candidates:
            ts = sorted(time_batch(shapes, b) for _ in range(reps))
            t = ts[len(ts) // 2]
            if t < best_t:
                best, best_t = b, t
        if not table or table[-1][1] != best:
            table.append((lo, best))
    return table


def save(table, path: str) -> None:
    with open(path, "w") as f:
        json.dump({"table": [list(e) for e in table], "when": time.strftime("%Y-%m-%d %H:%M:%S")}, f)


def load(path: str) -> list[tuple[int, int]]:
    with open(path) as f:
        return [tuple(e) for e in json.load(f)["table"]]


TABLE_PATH = __import__("os").path.join(__import__("os").path.dirname(__file__), "batch_tiles.json")


def current_table() -> list[tuple[int, int]]:
    """The tuned table if one was saved next to this module, else the default."""
    import os
    return load(TABLE_PATH) if os.path.exists(TABLE_PATH) else list(DEFAULT_TABLE)


def main() -> None:
    """Tunes on the GPU with problems of the batched workload (m log-uniform
    in [16, 512], n uniform in [8, m]) and saves the table next to this
    module."""
    import torch
    from . import tqr, workloads
    pool = workloads.batch_shapes(20000, seed=21)

    def sample(lo, hi):
        return [s for s in pool if lo <= s[1] < hi][:1500]

    def time_batch(shapes, b):
        bt = tqr.Batch(shapes, [b] * len(shapes))
        workloads.fill_normal_device(bt.A, 5)
        bt.factor()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        workloads.fill_normal_device(bt.A, 5)
        e0.record()
        bt.factor()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    table = tune(sample, time_batch)
    save(table, TABLE_PATH)
    print("tile table:", table, flush=True)


if __name__ == "__main__":
    main()
