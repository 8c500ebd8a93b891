"""The product's operation counts (paper_0707_3548_amd/flops.py), which the
benchmark's rates and roofline use, pinned against the oracle's task-graph
flop model (oracle/dag.py, itself pinned to the counts of Sec. 3.2) and
against closed forms: the standard count 2n^2(m - n/3) of Sec. 2.1 and the
tiled count 2n^2(m - n/3)(1 + ib/(4b)) to leading order."""
import pytest

from oracle import dag
from paper_0707_3548_amd import flops

KINDS = {"GEQRT": dag.GEQRT, "TSQRT": dag.TSQRT, "LARFB": dag.LARFB, "SSRFB": dag.SSRFB}


@pytest.mark.parametrize("b,ib", [(16, 16), (64, 16), (64, 64), (128, 32), (256, 16), (256, 32), (200, 200)])
def test_kernel_flops_equal_the_oracle_model(b, ib):
    for name, kind in KINDS.items():
        assert flops.kernel_flops(name, b, ib) == dag.kernel_flops(kind, b, ib), (name, b, ib)


def test_paper_leading_terms_at_ib_equal_b():
    # Sec. 3.2: GEQRT 2 b^3 (4/3 + 2/3 for T), LARFB 3 b^3, TSQRT 10/3 b^3, SSRFB 5 b^3
    b = 2000
    for name, lead in (("GEQRT", 2.0), ("LARFB", 3.0), ("TSQRT", 10.0 / 3.0), ("SSRFB", 5.0)):
        assert abs(flops.kernel_flops(name, b, b) / b ** 3 - lead) < 0.01 * lead, name


def test_standard_and_target_counts():
    assert flops.standard(8192, 8192) == pytest.approx(7.330e11, rel=1e-3)
    assert flops.standard(65536, 1024) == pytest.approx(1.367e11, rel=1e-3)
    assert flops.standard(16384, 4096) == pytest.approx(5.039e11, rel=1e-3)
    for m, n in ((8192, 8192), (65536, 1024), (300, 7)):
        assert flops.bj_formula(m, n) == pytest.approx(2.0 * flops.standard(m, n), rel=1e-12)


@pytest.mark.parametrize("m,n,b,ib", [(8192, 8192, 256, 16), (65536, 1024, 256, 16), (512, 512, 64, 16),
                                      (16384, 4096, 256, 16)])
def test_tiled_total(m, n, b, ib):
    p, q = -(-m // b), -(-n // b)
    assert flops.tiled(m, n, b, ib) == pytest.approx(dag.executed_flops(p, q, b, ib), rel=1e-12)
    # leading order 2n^2(m - n/3)(1 + ib/(4b)); the lower-order terms are
    # within a few percent at these sizes
    lead = flops.standard(m, n) * (1 + ib / (4.0 * b))
    assert abs(flops.tiled(m, n, b, ib) / lead - 1) < 0.05
