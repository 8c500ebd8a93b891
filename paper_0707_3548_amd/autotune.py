"""(tile_b, inner_ib) per size bucket for the batched factorisation.

Every problem of a batch runs in one workgroup, so the best tiling depends on
the problem's size only: small tiles waste less zero padding, large ones run
more of the work on the matrix cores, and the inner block trades the panel's
length against the size of the trailing products.  ``tune`` times each
candidate (tile_b, inner_ib) pair on sample problems of every bucket (a
batch of same-bucket problems, the median of a few launches) and keeps the
fastest; ``tiling_for`` reads the table (a tuned one if given, else the
built-in one).  Buckets are by n (columns), the dimension that sets the
number of tile columns and the panel length.  The FP64 and FP32-update
batches are tuned separately (the FP32 tier supports inner_ib 16 only).
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Callable, Sequence

# (lowest n of the bucket, tile size, inner block); buckets run up to the next entry's n
DEFAULT_TABLE = [(0, 16, 16), (32, 32, 16), (64, 64, 16)]
CANDIDATES = ((16, 16), (32, 16), (32, 32), (64, 16), (64, 32), (64, 64), (128, 16), (128, 32))
CANDIDATES_FP32 = ((16, 16), (32, 16), (64, 16), (128, 16))
BUCKETS = (0, 16, 32, 64, 128, 256)


def _norm(table):
    """Entries as (lo, b, ib); two-element entries (older tables) mean ib 16."""
    return sorted((int(e[0]), int(e[1]), int(e[2]) if len(e) > 2 else 16) for e in table)


def tiling_for(n: int, table: Sequence[Sequence[int]] | None = None) -> tuple[int, int]:
    tab = _norm(table or DEFAULT_TABLE)
    b, ib = tab[0][1], tab[0][2]
    for lo, tb, tib in tab:
        if n >= lo:
            b, ib = tb, tib
    return b, ib


def tile_for(n: int, table: Sequence[Sequence[int]] | None = None) -> int:
    return tiling_for(n, table)[0]


def tune(sample: Callable[[int, int], list[tuple[int, int]]], time_batch: Callable[[list, int, int], float],
         candidates: Sequence[tuple[int, int]] = CANDIDATES, buckets: Sequence[int] = BUCKETS,
         reps: int = 3) -> list[tuple[int, int, int]]:
    """sample(lo, hi) -> shapes with lo <= n < hi; time_batch(shapes, b, ib)
    -> seconds for one launch of those shapes all with that tiling.  Returns
    a table for tiling_for, with neighbouring buckets of the same choice
    merged."""
    table = []
    edges = list(buckets) + [math.inf]
    for lo, hi in zip(edges[:-1], edges[1:]):
        shapes = sample(lo, hi)
        if not shapes:
            continue
        best, best_t = None, math.inf
        for b, ib in candidates:
            ts = sorted(time_batch(shapes, b, ib) for _ in range(reps))
            t = ts[len(ts) // 2]
            if t < best_t:
                best, best_t = (b, ib), t
        if not table or table[-1][1:] != best:
            table.append((lo, *best))
    return table


TABLE_PATH = os.path.join(os.path.dirname(__file__), "batch_tiles.json")


def save(tables: dict, path: str = TABLE_PATH) -> None:
    out = {k: [list(e) for e in v] for k, v in tables.items()}
    out["when"] = time.strftime("%Y-%m-%d %H:%M:%S")
    with open(path, "w") as f:
        json.dump(out, f)


def load(path: str = TABLE_PATH, precision: str = "fp64") -> list[tuple[int, int, int]]:
    with open(path) as f:
        d = json.load(f)
    key = "table" if precision == "fp64" else "table_fp32"
    return _norm(d[key]) if key in d else list(DEFAULT_TABLE)


def current_table(precision: str = "fp64") -> list[tuple[int, int, int]]:
    """The tuned table for "fp64" or "fp32" if one was saved next to this
    module, else the default."""
    return load(TABLE_PATH, precision) if os.path.exists(TABLE_PATH) else list(DEFAULT_TABLE)


def main() -> None:
    """Tunes on the GPU with problems of the batched workload (m log-uniform
    in [16, 512], n uniform in [8, m]), for FP64 and FP32-update batches, and
    saves the tables next to this module."""
    import torch
    from . import tqr, workloads
    pool = workloads.batch_shapes(20000, seed=21)

    def sample(lo, hi):
        return [s for s in pool if lo <= s[1] < hi][:1500]

    def timer(precision):
        def time_batch(shapes, b, ib):
            bt = tqr.Batch(shapes, [b] * len(shapes), [ib] * len(shapes), precision=precision)
            workloads.fill_normal_device(bt.A, 5)
            bt.factor()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            workloads.fill_normal_device(bt.A, 5)
            e0.record()
            bt.factor()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / 1e3
        return time_batch

    tables = {"table": tune(sample, timer(tqr.PRECISION_FP64)),
              "table_fp32": tune(sample, timer(tqr.PRECISION_FP32_UPDATES), candidates=CANDIDATES_FP32)}
    save(tables)
    print("tilings:", tables, flush=True)


if __name__ == "__main__":
    main()
