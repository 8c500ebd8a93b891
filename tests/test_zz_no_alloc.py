"""tqr_factor_noalloc (the factorisation whose workspace is the library's
fixed device scratch) against tqr_factor with a caller-provided workspace
(GPU).

Both run the same kernels over the same task graph, and every legal schedule
applies the same operations to every tile in the same order (Algorithm 1), so
R, the reflector tiles and T must agree bit for bit.  Three calls in a row on
one stream share the scratch: the largest problem that fits it first, then
smaller ones, so each later call runs on scratch that still holds the earlier
call's tiles and scheduler words.
"""
import numpy as np
import pytest

import oracle
from paper_0707_3548_amd import workloads

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _factor_both(torch, tqr, A, b, ib):
    m, n = A.shape
    src = tqr.fortran(torch.from_numpy(A).cuda())
    ref = src.clone()
    _, T_ref = tqr.factor_plain(ref, b, ib)
    out = src.clone()
    T = torch.full((tqr.t_elems(m, n, b, ib),), np.nan, dtype=torch.float64, device="cuda")
    tqr.factor_noalloc(out, T, b, ib)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), T_ref.cpu().numpy(), out.cpu().numpy(), T.cpu().numpy()


def test_noalloc_matches_the_workspace_call_on_consecutive_calls():
    torch = _torch()
    from paper_0707_3548_amd import tqr
    torch.cuda.set_device(0)
    # largest first (3840^2 at b = 256 needs 120.4 MiB of the 128 MiB), then smaller
    cases = [(3840, 3840, 256, 16, 0), (1500, 1100, 128, 16, 1), (300, 200, 64, 16, 2)]
    for m, n, b, ib, seed in cases:
        need = tqr.workspace_bytes(m, n, 0, b, ib)
        assert 0 < need <= tqr.NOALLOC_SCRATCH_BYTES
        print(f"noalloc: {m}x{n} b={b} ib={ib} seed={seed} (workspace {need} bytes)", flush=True)
        A = workloads.gaussian(m, n, seed=seed)
        ref, T_ref, out, T = _factor_both(torch, tqr, A, b, ib)
        assert np.array_equal(out, ref), f"{m}x{n}: A differs from tqr_factor's"
        # T slots with i >= k are written; compare those (the rest is unspecified)
        p, q = -(-m // b), -(-n // b)
        slot = ib * b
        for k in range(q):
            for i in range(k, p):
                s = (k * p + i) * slot
                assert np.array_equal(T[s:s + slot], T_ref[s:s + slot]), f"{m}x{n}: T slot ({i},{k}) differs"
        if m <= 1500:
            _, R_or = oracle.qr(A)
            err = oracle.rel_fro(oracle.sign_normalize(np.triu(out[:n, :])), R_or)
            assert err < 1e-10, err


def test_noalloc_rejects_a_problem_beyond_the_scratch():
    torch = _torch()
    from paper_0707_3548_amd import tqr
    A = torch.zeros((4096, 4096), dtype=torch.float64, device="cuda").t()  # column-major view
    T = torch.zeros(tqr.t_elems(4096, 4096, 256, 16), dtype=torch.float64, device="cuda")
    with pytest.raises(tqr.TqrError) as e:
        tqr.factor_noalloc(A, T, 256, 16)
    assert e.value.code == tqr.TQR_ESCRATCH
    assert "scratch" in str(e.value)
