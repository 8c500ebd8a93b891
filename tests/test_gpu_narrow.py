"""Narrow right-hand sides (1 to 4 columns, tile_b >= 64, inner_ib 16): Q^T B,
Q B and the least-squares solve run as pipelines of workgroups (one per row
tile, one per 64-row block of R) instead of task graphs (GPU).

* tqr_apply_qt against the tiled model of Algorithm 1 (oracle/tiled.py: the
  same transformations applied in numpy), elementwise; tqr_apply_q undoes it.
* tqr_solve_ls against the oracle's least-squares solution (unblocked
  Householder QR of Sec. 2.1, Q^T b, back substitution) and its normwise
  backward error.
The shapes cover ragged edges (m, n not multiples of b), square grids (the
last tile row is also a diagonal tile), one-tile-row problems, and every
block width (1, 2, 3 -> 4, 4).
"""
import numpy as np
import pytest

import oracle
from oracle import tiled

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)


APPLY = [(1000, 700, 64, 1), (777, 500, 128, 2), (1300, 600, 256, 3), (2048, 512, 256, 4), (300, 300, 128, 4),
         (65, 64, 64, 1), (256, 256, 256, 2), (900, 130, 64, 3)]


@pytest.mark.parametrize("m,n,b,nrhs", APPLY)
def test_narrow_apply_matches_tiled_model(m, n, b, nrhs):
    torch = _torch()
    from paper_0707_3548_amd import tqr, workloads
    ib = 16
    _say(f"case narrow apply m={m} n={n} b={b} nrhs={nrhs}")
    A = workloads.gaussian(m, n, seed=21)
    Bh = workloads.gaussian(m, nrhs, seed=22)
    dA = tqr.fortran(torch.from_numpy(A).cuda())
    ws = tqr.Workspace(m, n, nrhs, b, ib)
    tqr.factor(dA, b, ib, ws)
    dB = tqr.fortran(torch.from_numpy(Bh).cuda())
    tqr.apply_qt(dA, ws.T, dB, b, ib, ws)
    torch.cuda.synchronize()
    tiles, Tm = tiled.factor(A, b, ib)
    C_model = tiled.apply_qt(tiles, Tm, Bh)
    assert oracle.rel_fro(dB.cpu().numpy(), C_model) < 1e-12
    tqr.apply_q(dA, ws.T, dB, b, ib, ws)
    torch.cuda.synchronize()
    assert oracle.rel_fro(dB.cpu().numpy(), Bh) < 1e-13


SOLVE = [(2000, 900, 256, 1, 1e4), (1500, 1500, 128, 3, 1e3), (3000, 700, 64, 4, 1e5), (515, 300, 256, 2, 1e2),
         (4096, 1024, 256, 1, 1e6)]


@pytest.mark.parametrize("m,n,b,nrhs,cond", SOLVE)
def test_narrow_solve_ls_matches_oracle(m, n, b, nrhs, cond):
    torch = _torch()
    from paper_0707_3548_amd import tqr, workloads
    ib = 16
    _say(f"case narrow solve_ls m={m} n={n} b={b} nrhs={nrhs} cond={cond:g}")
    A, Bh, _ = workloads.ls_problem(m, n, cond, seed=23, nrhs=nrhs)
    dA = tqr.fortran(torch.from_numpy(A).cuda())
    dB = tqr.fortran(torch.from_numpy(Bh).cuda())
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    _, info = tqr.solve_ls(dA, dB, b, ib, status=status)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    assert int(status.item()) == 0
    X = dB.cpu().numpy()[:n]
    Xo, _ = oracle.lstsq(A, Bh, omp=True)
    assert np.linalg.norm(X - Xo) / np.linalg.norm(Xo) < cond * 1e-13
    for c in range(nrhs):
        assert oracle.ls_backward_error(A, X[:, c], Bh[:, c], omp=True) < 1e-15


def test_narrow_solve_is_repeatable():
    """The pipelines take their places from a ticket counter; the result does
    not depend on which workgroup got which place (bitwise, three runs)."""
    torch = _torch()
    from paper_0707_3548_amd import tqr, workloads
    m, n, b, ib, nrhs = 2500, 1200, 128, 16, 2
    _say("case narrow repeatability")
    A, Bh, _ = workloads.ls_problem(m, n, 1e3, seed=24, nrhs=nrhs)
    outs = []
    for _ in range(3):
        dA = tqr.fortran(torch.from_numpy(A).cuda())
        dB = tqr.fortran(torch.from_numpy(Bh).cuda())
        tqr.solve_ls(dA, dB, b, ib)
        torch.cuda.synchronize()
        outs.append(dB.cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
