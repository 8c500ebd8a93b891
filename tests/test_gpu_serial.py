"""Tile kernels in the reference order (one launch per task, Algorithm 1
order, no scheduler): R against the oracle, V and T tiles against the tiled
model.  GPU."""
import numpy as np
import pytest

import oracle
from oracle import tiled
from test_gpu_factor import run_factor, t_slots

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,n,b,ib", [(200, 150, 64, 16), (512, 512, 64, 16), (100, 70, 32, 16),
                                      (257, 129, 256, 32), (300, 300, 128, 32), (64, 64, 64, 64)])
def test_serial_factor_matches_oracle(m, n, b, ib):
    from paper_0707_3548_amd import tqr, workloads
    print(f"case serial m={m} n={n} b={b} ib={ib}", flush=True)
    A = workloads.gaussian(m, n, seed=m * 13 + n)
    dA, ws = run_factor(A, b, ib, mode=tqr.MODE_SERIAL)
    F = dA.cpu().numpy()
    _, R_or = oracle.qr(A)
    assert oracle.rel_fro(oracle.sign_normalize(np.triu(F[:n, :])), R_or) < 1e-10
    tiles, Tm = tiled.factor(A, b, ib)
    F_model = tiled.from_tiles(tiles, m, n)
    assert np.abs(F - F_model).max() < 1e-11 * max(1.0, np.abs(F_model).max()) * max(1, n // 64)
    Tg = t_slots(ws.T, m, n, b, ib)
    for k in range(min(Tg.shape[:2])):
        for i in range(k, Tg.shape[0]):
            assert np.abs(Tg[i, k] - Tm[i, k]).max() < 1e-11 * max(1, n // 64) * max(1.0, np.abs(Tm[i, k]).max())
