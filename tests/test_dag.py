"""The task graph of Algorithm 1: closed-form rules against a generic hazard
analysis, the p = q = 3 graph, the recursive sub-graph property of Sec. 3.3,
task and operation counts of Sec. 3.2, and the list-scheduler model.  CPU."""
import os
from fractions import Fraction

import pytest

from conftest import GOLDEN
from oracle import dag


def _parse_task(tok):
    kind = {"G": dag.GEQRT, "L": dag.LARFB, "T": dag.TSQRT, "S": dag.SSRFB}[tok[0]]
    nums = [int(x) - 1 for x in tok[1:]]
    if kind == dag.GEQRT:
        k, = nums
        return (kind, k, k, k)
    if kind == dag.LARFB:
        k, j = nums
        return (kind, k, j, k)
    if kind == dag.TSQRT:
        i, k = nums
        return (kind, i, k, k)
    i, j, k = nums
    return (kind, i, j, k)


def test_p3q3_graph_matches_fixture():
    edges = set()
    with open(os.path.join(GOLDEN, "dag_p3q3.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            a, b = line.split("->")
            edges.add((_parse_task(a.split()), _parse_task(b.split())))
    tasks = dag.algorithm1(3, 3)
    n = len(tasks)
    assert n == 14
    red = dag.transitive_reduction(dag.hazard_edges(tasks), n)
    assert {(tasks[u], tasks[v]) for u, v in red} == edges
    assert len(edges) == 21


@pytest.mark.parametrize("p,q", [(p, q) for p in range(1, 8) for q in range(1, 8)])
def test_closed_form_equals_hazard_analysis(p, q):
    tasks = dag.algorithm1(p, q)
    n = len(tasks)
    he = dag.hazard_edges(tasks)
    ce = dag.closed_form_edges(p, q)
    assert dag.transitive_closure(he, n) == dag.transitive_closure(ce, n)
    assert dag.transitive_reduction(he, n) == dag.transitive_reduction(ce, n)


def test_recursive_subgraph_property():
    big = dag.algorithm1(6, 5)
    big_edges = {(big[u], big[v]) for u, v in dag.closed_form_edges(6, 5)}
    for p2 in range(1, 7):
        for q2 in range(1, 6):
            small = dag.algorithm1(p2, q2)
            assert set(small) <= set(big)
            edges = {(small[u], small[v]) for u, v in dag.closed_form_edges(p2, q2)}
            assert edges <= big_edges


@pytest.mark.parametrize("p,q,total", [(3, 3, 14), (8, 8, 204), (32, 32, 11440), (256, 4, 2550), (64, 16, 8024)])
def test_task_counts(p, q, total):
    c = dag.task_counts(p, q)
    assert sum(c.values()) == total
    if p * q <= 1024:
        tasks = dag.algorithm1(p, q)
        assert len(tasks) == total
        for kind in c:
            assert sum(1 for t in tasks if t[0] == kind) == c[kind]


def test_operation_counts_of_the_paper():
    want = {}
    with open(os.path.join(GOLDEN, "opcount.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, num, den = line.split()
            want[name] = Fraction(int(num), int(den))
    names = {v: k for k, v in dag.NAMES.items()}
    for name, val in want.items():
        assert dag.PAPER_FLOPS_B3[names[name]] == val
        # the executed-flop model at ib == b has the paper's leading term
        b = 2048
        assert dag.kernel_flops(names[name], b, b) / b ** 3 == pytest.approx(float(val), rel=2e-3)
    assert dag.paper_total_flops(3, 3, 1) == 50.0
    # Eq. (opcount): 5/2 n^2 (m - n/3) to leading order in the tile counts
    p = q = 400
    assert dag.paper_total_flops(p, q, 1) / (2.5 * q * q * (p - q / 3)) == pytest.approx(1.0, rel=1e-2)


def test_inner_blocking_flop_model():
    """SSRFB executes 4 b^3 + ib b^2 flops with inner blocks of ib columns;
    ib -> 1 approaches the LAPACK count (4 b^3 per b x b update pair)."""
    b = 256
    assert dag.kernel_flops(dag.SSRFB, b, 32) == 4 * b ** 3 + 32 * b * b
    assert dag.kernel_flops(dag.SSRFB, b, 1) / (4 * b ** 3) == pytest.approx(1.0, rel=1e-2)


@pytest.mark.parametrize("workers", [1, 2, 3, 7, 16, 64])
def test_list_scheduler_respects_edges_and_priorities(workers):
    p, q = 6, 5
    tasks = dag.algorithm1(p, q)
    dur = lambda t: {dag.GEQRT: 2, dag.TSQRT: 3, dag.LARFB: 3, dag.SSRFB: 5}[t[0]]
    start, finish, where = dag.simulate(p, q, workers, dur)
    for u, v in dag.closed_form_edges(p, q):
        assert start[v] >= finish[u]
    # a worker never runs two tasks at once
    by_w = {}
    for v in range(len(tasks)):
        by_w.setdefault(where[v], []).append((start[v], finish[v]))
    for spans in by_w.values():
        spans.sort()
        for (s0, f0), (s1, f1) in zip(spans, spans[1:]):
            assert s1 >= f0
    if workers == 1:
        assert max(finish) == sum(dur(t) for t in tasks)
    assert max(finish) >= dag.critical_path(p, q, dur)
