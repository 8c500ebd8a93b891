"""The task graph of Algorithm 1 (Buttari et al., Sec. 3.3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``algorithm1(p, q)`` -- the tasks in the order Algorithm 1 issues them.
* ``accesses(task)`` -- what each elementary operation of Sec. 3.1 reads and
  writes.  The diagonal tile is two data items: its strict lower part (V_kk)
  and its upper triangle (R_kk), because DTSQT2 only rewrites R_kk while
  DLARFB only reads V_kk.
* ``hazard_edges`` -- a generic read/write hazard analysis of the sequential
  task list (read-after-write, write-after-write, write-after-read).  It
  knows nothing of the algorithm's structure, so it is an independent check
  of any closed-form dependency rule.
* ``closed_form_preds`` -- the dependency rules of the flat elimination tree
  written out by hand.
* priorities (Sec. 3.3): DGEQT2 highest, then DTSQT2, DLARFB, DSSRFB.
* ``simulate`` -- a discrete-event list scheduler with W workers and
  priority-ordered ready queues, the CPU stand-in for a dynamic scheduler.
* operation counts of Sec. 3.2.

Task tuples are ``(kind, i, j, k)`` with 0-based tile indices:
GEQRT(k) = (GEQRT, k, k, k), LARFB(k, j) = (LARFB, k, j, k),
TSQRT(i, k) = (TSQRT, i, k, k), SSRFB(i, j, k) = (SSRFB, i, j, k).
"""
from __future__ import annotations

import heapq
from collections import defaultdict
from fractions import Fraction

GEQRT, TSQRT, LARFB, SSRFB = 0, 1, 2, 3  # numeric value = priority level (0 highest)
NAMES = {GEQRT: "GEQRT", TSQRT: "TSQRT", LARFB: "LARFB", SSRFB: "SSRFB"}


def algorithm1(p: int, q: int):
    out = []
    for k in range(min(p, q)):
        out.append((GEQRT, k, k, k))
        for j in range(k + 1, q):
            out.append((LARFB, k, j, k))
        for i in range(k + 1, p):
            out.append((TSQRT, i, k, k))
            for j in range(k + 1, q):
                out.append((SSRFB, i, j, k))
    return out


def _tile_items(i, j):
    return [("A", i, j, "V"), ("A", i, j, "R")] if i == j else [("A", i, j, "F")]


def accesses(task):
    """(reads, writes) of one task, as sets of data items."""
    kind, i, j, k = task
    if kind == GEQRT:
        r = set(_tile_items(k, k))
        w = set(_tile_items(k, k)) | {("T", k, k)}
    elif kind == LARFB:
        r = {("A", k, k, "V"), ("T", k, k)} | set(_tile_items(k, j))
        w = set(_tile_items(k, j))
    elif kind == TSQRT:
        r = {("A", k, k, "R")} | set(_tile_items(i, k))
        w = {("A", k, k, "R"), ("T", i, k)} | set(_tile_items(i, k))
    elif kind == SSRFB:
        r = set(_tile_items(k, j)) | set(_tile_items(i, j)) | set(_tile_items(i, k)) | {("T", i, k)}
        w = set(_tile_items(k, j)) | set(_tile_items(i, j))
    else:
        raise ValueError(kind)
    return r, w


def hazard_edges(tasks):
    """All hazard edges (u, v), u < v, of a sequential task list."""
    last_writer = {}
    readers = defaultdict(list)
    edges = set()
    for v, t in enumerate(tasks):
        r, w = accesses(t)
        for item in r:
            if item in last_writer:
                edges.add((last_writer[item], v))
        for item in w:
            if item in last_writer:
                edges.add((last_writer[item], v))
            for u in readers[item]:
                if u != v:
                    edges.add((u, v))
        for item in r:
            readers[item].append(v)
        for item in w:
            last_writer[item] = v
            readers[item] = []
    return edges


def closed_form_preds(task, p: int, q: int):
    """Direct predecessors of a task under the flat elimination tree."""
    kind, i, j, k = task
    preds = []
    prev = (lambda x, y: _last_update(x, y, k - 1)) if k > 0 else (lambda x, y: None)
    if kind == GEQRT:
        preds.append(prev(k, k))
    elif kind == LARFB:
        preds += [(GEQRT, k, k, k), prev(k, j)]
    elif kind == TSQRT:
        preds.append((GEQRT, k, k, k) if i == k + 1 else (TSQRT, i - 1, k, k))
        preds.append(prev(i, k))
    elif kind == SSRFB:
        preds.append((TSQRT, i, k, k))
        preds.append((LARFB, k, j, k) if i == k + 1 else (SSRFB, i - 1, j, k))
        preds.append(prev(i, j))
    return [x for x in preds if x is not None]


def _last_update(i, j, k):
    """The task of step k that last writes tile (i, j) (i, j > k)."""
    return (SSRFB, i, j, k)


def closed_form_edges(p: int, q: int):
    tasks = algorithm1(p, q)
    index = {t: n for n, t in enumerate(tasks)}
    return {(index[u], index[t]) for t in tasks for u in closed_form_preds(t, p, q)}


def successors(edges, n):
    succ = [set() for _ in range(n)]
    for u, v in edges:
        succ[u].add(v)
    return succ


def transitive_closure(edges, n):
    succ = successors(edges, n)
    reach = [set() for _ in range(n)]
    for u in reversed(range(n)):  # tasks are topologically ordered by index
        for v in succ[u]:
            reach[u].add(v)
            reach[u] |= reach[v]
    return {(u, v) for u in range(n) for v in reach[u]}


def transitive_reduction(edges, n):
    succ = successors(edges, n)
    closure = transitive_closure(edges, n)
    red = set()
    for u, v in edges:
        if not any((w, v) in closure for w in succ[u] if w != v):
            red.add((u, v))
    return red


def task_counts(p: int, q: int):
    K = min(p, q)
    return {
        GEQRT: K,
        LARFB: sum(q - 1 - k for k in range(K)),
        TSQRT: sum(p - 1 - k for k in range(K)),
        SSRFB: sum((p - 1 - k) * (q - 1 - k) for k in range(K)),
    }


# --- operation counts (Sec. 3.2) ----------------------------------------------

PAPER_FLOPS_B3 = {GEQRT: Fraction(2), LARFB: Fraction(3), TSQRT: Fraction(10, 3), SSRFB: Fraction(5)}


def paper_total_flops(p: int, q: int, b: int) -> float:
    """The sum of Eq. (opcount): per step k, one DGEQT2, q-k DLARFB, p-k DTSQT2
    and (p-k)(q-k) DSSRFB at 2, 3, 10/3 and 5 b^3 flops."""
    c = task_counts(p, q)
    return float(sum(PAPER_FLOPS_B3[kd] * c[kd] for kd in c)) * b ** 3


def kernel_flops(kind: int, b: int, ib: int) -> float:
    """Flops a kernel executes when it exploits the unit/zero structure of V
    and the triangular T, with inner blocks of ib columns.  At ib == b the
    leading terms are the paper's 2, 3, 10/3 and 5 b^3."""
    nb = b // ib
    if kind == SSRFB:
        # per block: W = A_kj[s] + V_s^T A_ij (2 ib b^2), T^T W (ib^2 b),
        # A_kj[s] -= W, A_ij -= V_s W (2 ib b^2)
        return nb * (4.0 * ib * b * b + ib * ib * b)
    if kind == LARFB:
        # block s acts on rows s*ib..b-1 (h rows) with a unit-lower V_s:
        # V_s^T C and V_s W cost (2 h ib - ib^2) b each, T^T W costs ib^2 b
        tot = 0.0
        for s in range(nb):
            h = b - s * ib
            tot += 2 * (2.0 * h * ib - ib * ib) * b + ib * ib * b
        return tot
    if kind == TSQRT:
        tot = 0.0
        for s in range(nb):
            rest = b - (s + 1) * ib
            # panel: column jj updates ib-1-jj panel columns over b+1 rows (4 flops/row/col)
            tot += sum(4.0 * (b + 1) * (ib - 1 - jj) + 3.0 * b for jj in range(ib))
            # T: column jj needs V^T v (2 b jj) and a triangular product (jj^2)
            tot += sum(2.0 * b * jj + jj * jj for jj in range(ib))
            # trailing update of the remaining columns
            tot += (4.0 * ib * b + ib * ib + 2 * ib) * rest
        return tot
    if kind == GEQRT:
        tot = 0.0
        for s in range(nb):
            h = b - s * ib
            rest = b - (s + 1) * ib
            tot += sum(4.0 * (h - jj) * (ib - 1 - jj) + 3.0 * (h - jj) for jj in range(ib))
            tot += sum(2.0 * (h - jj) * jj + jj * jj for jj in range(ib))
            tot += (2 * (2.0 * h * ib - ib * ib) + ib * ib) * rest
        return tot
    raise ValueError(kind)


def executed_flops(p: int, q: int, b: int, ib: int) -> float:
    c = task_counts(p, q)
    return sum(kernel_flops(kd, b, ib) * c[kd] for kd in c)


# --- a CPU model of a dynamic scheduler ---------------------------------------

def simulate(p: int, q: int, workers: int, duration=None):
    """List-schedule the graph on ``workers`` identical workers.  A worker
    that becomes free takes the ready task with the best (priority level, k,
    i, j); a task becomes ready when its last predecessor finishes.
    Returns (start, finish, worker) per task index, in Algorithm 1 order."""
    tasks = algorithm1(p, q)
    n = len(tasks)
    edges = closed_form_edges(p, q)
    succ = successors(edges, n)
    indeg = [0] * n
    for _, v in edges:
        indeg[v] += 1
    dur = [1.0 if duration is None else float(duration(t)) for t in tasks]

    def key(v):
        kind, i, j, k = tasks[v]
        return (kind, k, i, j)

    ready = [(key(v), v) for v in range(n) if indeg[v] == 0]
    heapq.heapify(ready)
    events = []  # (time, worker, task)
    free = list(range(workers))
    start = [None] * n
    finish = [None] * n
    where = [None] * n
    now = 0.0
    done = 0
    while done < n:
        while ready and free:
            _, v = heapq.heappop(ready)
            w = free.pop(0)
            start[v] = now
            where[v] = w
            heapq.heappush(events, (now + dur[v], w, v))
        if not events:
            raise RuntimeError("deadlock: no running task and nothing ready")
        now, w, v = heapq.heappop(events)
        finish[v] = now
        done += 1
        free.append(w)
        free.sort()
        for s in succ[v]:
            indeg[s] -= 1
            if indeg[s] == 0:
                heapq.heappush(ready, (key(s), s))
    return start, finish, where


def critical_path(p: int, q: int, duration=None) -> float:
    tasks = algorithm1(p, q)
    n = len(tasks)
    edges = closed_form_edges(p, q)
    preds = defaultdict(list)
    for u, v in edges:
        preds[v].append(u)
    dur = [1.0 if duration is None else float(duration(t)) for t in tasks]
    fin = [0.0] * n
    for v in range(n):
        fin[v] = dur[v] + max((fin[u] for u in preds[v]), default=0.0)
    return max(fin, default=0.0)
