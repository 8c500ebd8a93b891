"""FP32 precision tier (trailing updates on the FP32 matrix cores) and the
mixed-precision least-squares solver (FP32-update factor, then FP64 CGLS on
A R^{-1}).

Tolerances: the FP32-update factor is compared with the unblocked FP64 oracle
to FP32 accuracy (R to 1e-4 relative, ||A - QR|| / ||A|| to 50 sqrt(n) u32),
while Q stays orthogonal to FP64 accuracy (every reflector comes from the
FP64 panels and is applied in FP64).  The refined least-squares solution
must meet the FP64 bounds of the FP64 solver's own test: backward error
< 1e-14 and forward error < cond * 1e-13 against the oracle."""
import numpy as np
import pytest

import oracle

U32 = 2.0 ** -24


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_mixed_workspace_query():
    from paper_0707_3548_amd import tqr
    L = tqr.lib()
    assert L.tqr_ls_mixed_workspace_bytes(100, 50, 2, 64) > 0
    assert L.tqr_ls_mixed_workspace_bytes(100, 50, 2, 32) == -1
    assert L.tqr_ls_mixed_workspace_bytes(10, 50, 2, 64) == -1
    assert L.tqr_ls_mixed_workspace_bytes(100, 50, 0, 64) == -1


def test_mixed_argument_checks():
    import ctypes
    from paper_0707_3548_amd import tqr
    L = tqr.lib()
    a = ctypes.c_void_p(4096)
    args = [100, 50, 1, a, 100, a, 100, a, 50, 64, 3, a, a, 1 << 30, a, None, None, None]
    def rc(**kw):
        v = list(args)
        names = ["m", "n", "nrhs", "A", "lda", "B", "ldb", "X", "ldx", "tile_b", "iters", "T", "work", "wb", "info"]
        for k, x in kw.items():
            v[names.index(k)] = x
        return L.tqr_solve_ls_mixed(*v)
    assert rc(m=10) == -1
    assert rc(n=-1) == -2
    assert rc(nrhs=0) == -3
    assert rc(lda=99) == -5
    assert rc(ldb=10) == -7
    assert rc(ldx=10) == -9
    assert rc(tile_b=32) == -10
    assert rc(iters=201) == -11
    assert rc(iters=-1) == -11
    assert rc(wb=100) == -14
    assert rc(info=None) == -15


@pytest.mark.gpu
@pytest.mark.parametrize("m,n,b", [(512, 512, 64), (600, 400, 128), (1000, 300, 256), (257, 129, 64)])
def test_fp32_updates_factor(m, n, b):
    torch = _torch()
    from paper_0707_3548_amd import tqr, workloads
    print(f"case fp32-updates factor m={m} n={n} b={b}", flush=True)
    A = workloads.gaussian(m, n, seed=31)
    dA = tqr.fortran(torch.from_numpy(A).cuda())
    ws = tqr.Workspace(m, n, 0, b, 16)
    tqr.factor(dA, b, 16, ws, precision=tqr.PRECISION_FP32_UPDATES)
    torch.cuda.synchronize()
    F = dA.cpu().numpy()
    R = np.triu(F[:n, :])
    _, R_or = oracle.qr(A)
    assert oracle.rel_fro(oracle.sign_normalize(R), R_or) < 1e-4
    E = torch.zeros((n, m), dtype=torch.float64, device="cuda").t()
    E[torch.arange(n), torch.arange(n)] = 1.0
    tqr.apply_q(dA, ws.T, E, b, 16)
    torch.cuda.synchronize()
    Q = E.cpu().numpy()
    assert oracle.orth_error(Q) <= 10 * n * oracle.EPS
    assert oracle.fact_error(A, Q, R) <= 50 * np.sqrt(n) * U32
    # and it is not the FP64 factor: the tier really ran in FP32
    dB = tqr.fortran(torch.from_numpy(A).cuda())
    tqr.factor(dB, b, 16)
    torch.cuda.synchronize()
    assert not torch.equal(dA, dB)


@pytest.mark.gpu
@pytest.mark.parametrize("m,n,b,nrhs,cond", [(512, 256, 64, 1, 1e2), (600, 400, 64, 3, 1e5), (1000, 300, 128, 2, 1e3),
                                             (777, 500, 256, 1, 1e4), (900, 400, 128, 6, 1e6)])
def test_mixed_ls_reaches_fp64_accuracy(m, n, b, nrhs, cond):
    """The refined solution meets the FP64 solver's bounds: backward error
    < 1e-14 and forward error < cond * 1e-13 against the oracle; the device's
    stopping test reports convergence or stagnation (not the limit), and its
    estimate agrees with the oracle's backward error (same formula with the
    oracle's triangle of [A; mu I])."""
    torch = _torch()
    from paper_0707_3548_amd import tqr, workloads
    print(f"case mixed LS m={m} n={n} b={b} nrhs={nrhs} cond={cond}", flush=True)
    A, Bh, _ = workloads.ls_problem(m, n, cond, seed=32, nrhs=nrhs)
    dA = tqr.fortran(torch.from_numpy(A).cuda())
    dB = tqr.fortran(torch.from_numpy(Bh).cuda())
    A0, B0 = dA.clone(), dB.clone()
    X, _, info, stats = tqr.solve_ls_mixed(dA, dB, b, iterations=40)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    assert torch.equal(dA, A0) and torch.equal(dB, B0)
    Xh = X.cpu().numpy()
    Xo, _ = oracle.lstsq(A, Bh)
    assert np.linalg.norm(Xh - Xo) / np.linalg.norm(Xo) < cond * 1e-13
    st = tqr.refine_stats(stats)
    for c in range(nrhs):
        eta = oracle.ls_backward_error(A, Xh[:, c], Bh[:, c])
        print(f"  rhs {c}: {st[c]}, oracle eta {eta:.3e}", flush=True)
        assert eta < 1e-14
        assert st[c]["stop"] in (tqr.REFINE_CONVERGED, tqr.REFINE_STAGNATED)
        assert 0 < st[c]["iterations"] < 40
        assert st[c]["eta"] < 1e-14


@pytest.mark.gpu
def test_mixed_ls_with_fp64_factor_and_zero_iterations():
    """iterations = 0 returns x = 0; with an FP64 factor A R^{-1} is
    orthogonal to FP64 rounding and CGLS stops within three iterations."""
    torch = _torch()
    from paper_0707_3548_amd import tqr, workloads
    print("case mixed LS fp64 factor", flush=True)
    A, Bh, _ = workloads.ls_problem(300, 200, 1e2, seed=33, nrhs=1)
    dA = tqr.fortran(torch.from_numpy(A).cuda())
    dB = tqr.fortran(torch.from_numpy(Bh).cuda())
    X0, _, _, st0 = tqr.solve_ls_mixed(dA, dB, 64, iterations=0)
    torch.cuda.synchronize()
    assert float(X0.abs().max()) == 0.0
    assert tqr.refine_stats(st0)[0]["iterations"] == 0
    X, _, info, st = tqr.solve_ls_mixed(dA, dB, 64, iterations=20, precision=tqr.PRECISION_FP64)
    torch.cuda.synchronize()
    assert oracle.ls_backward_error(A, X.cpu().numpy()[:, 0], Bh[:, 0]) < 1e-14
    assert tqr.refine_stats(st)[0]["iterations"] <= 3


@pytest.mark.gpu
def test_mixed_ls_beyond_the_fp32_factor_reports_stagnation_honestly():
    """cond 1e8 exceeds 1 / u32: the FP32-update factor's R is no longer a
    useful preconditioner (cond * u32 ~ 6), CGLS stalls far above FP64
    accuracy, and the solver says so (stop = stagnated, its estimate within
    a factor 10 of the oracle's backward error, which is above 1e-14).  The
    same solver with the FP64 factor reaches FP64 accuracy."""
    torch = _torch()
    from paper_0707_3548_amd import tqr, workloads
    m, n, b, cond = 700, 350, 64, 1e8
    print(f"case mixed LS cond={cond:g} (beyond the FP32 factor)", flush=True)
    A, Bh, _ = workloads.ls_problem(m, n, cond, seed=34, nrhs=1)
    dA = tqr.fortran(torch.from_numpy(A).cuda())
    dB = tqr.fortran(torch.from_numpy(Bh).cuda())
    X, _, info, stats = tqr.solve_ls_mixed(dA, dB, b, iterations=60)
    torch.cuda.synchronize()
    st = tqr.refine_stats(stats)[0]
    eta = oracle.ls_backward_error(A, X.cpu().numpy()[:, 0], Bh[:, 0])
    print(f"  FP32 factor: {st}, oracle eta {eta:.3e}", flush=True)
    if eta < 1e-14:
        assert st["stop"] == tqr.REFINE_CONVERGED
    else:
        assert st["stop"] in (tqr.REFINE_STAGNATED, tqr.REFINE_MAX_ITERATIONS)
        assert st["eta"] > 1e-14 and 0.1 < st["eta"] / eta < 10
    X, _, info, stats = tqr.solve_ls_mixed(dA, dB, b, iterations=20, precision=tqr.PRECISION_FP64)
    torch.cuda.synchronize()
    st = tqr.refine_stats(stats)[0]
    Xh = X.cpu().numpy()
    eta = oracle.ls_backward_error(A, Xh[:, 0], Bh[:, 0])
    print(f"  FP64 factor: {st}, oracle eta {eta:.3e}", flush=True)
    assert eta < 1e-14 and st["stop"] == tqr.REFINE_CONVERGED
    Xo, _ = oracle.lstsq(A, Bh)
    assert np.linalg.norm(Xh - Xo) / np.linalg.norm(Xo) < cond * 1e-13


U_BF16 = 2.0 ** -8   # unit roundoff of BF16 (8 significand bits)


@pytest.mark.gpu
@pytest.mark.parametrize("m,n,b", [(512, 512, 64), (777, 500, 128), (1024, 1024, 256)])
def test_bf16_updates_factor(m, n, b):
    """BF16 tier: the trailing updates' products take BF16 operands, so R
    carries BF16 rounding (R within 5 u_bf16 of the oracle, ||A - QR|| within
    5 u_bf16 of ||A||), while Q, built from the FP64 panels, stays orthogonal
    to FP64 accuracy; and the tier really ran (its R differs from the FP32
    tier's by more than FP32 rounding)."""
    torch = _torch()
    from paper_0707_3548_amd import tqr, workloads
    print(f"case bf16-updates factor m={m} n={n} b={b}", flush=True)
    A = workloads.gaussian(m, n, seed=35)
    dA = tqr.fortran(torch.from_numpy(A).cuda())
    ws = tqr.Workspace(m, n, 0, b, 16)
    tqr.factor(dA, b, 16, ws, precision=tqr.PRECISION_BF16_UPDATES)
    torch.cuda.synchronize()
    R = np.triu(dA.cpu().numpy()[:n, :])
    _, R_or = oracle.qr(A)
    e_r = oracle.rel_fro(oracle.sign_normalize(R), R_or)
    E = torch.zeros((n, m), dtype=torch.float64, device="cuda").t()
    E[torch.arange(n), torch.arange(n)] = 1.0
    tqr.apply_q(dA, ws.T, E, b, 16)
    torch.cuda.synchronize()
    Q = E.cpu().numpy()
    e_f = oracle.fact_error(A, Q, R)
    print(f"  R error {e_r:.3e}, factorisation error {e_f:.3e}", flush=True)
    assert e_r < 5 * U_BF16 and e_f < 5 * U_BF16
    assert oracle.orth_error(Q) <= 10 * n * oracle.EPS
    dF = tqr.fortran(torch.from_numpy(A).cuda())
    tqr.factor(dF, b, 16, precision=tqr.PRECISION_FP32_UPDATES)
    torch.cuda.synchronize()
    R32 = np.triu(dF.cpu().numpy()[:n, :])
    assert oracle.rel_fro(R, R32) > 100 * U32


@pytest.mark.gpu
def test_mixed_ls_with_bf16_factor():
    """BF16-update factor + FP64 CGLS: at cond 1e2 (cond * u_bf16 < 1) the
    refinement reaches FP64 accuracy; at cond 1e4 the BF16 R is no usable
    preconditioner and the solver reports stagnation with an estimate that
    agrees with the oracle's backward error."""
    torch = _torch()
    from paper_0707_3548_amd import tqr, workloads
    for cond, expect_converge in ((1e2, True), (1e4, False)):
        print(f"case mixed LS bf16 factor cond={cond:g}", flush=True)
        A, Bh, _ = workloads.ls_problem(800, 400, cond, seed=36, nrhs=1)
        dA = tqr.fortran(torch.from_numpy(A).cuda())
        dB = tqr.fortran(torch.from_numpy(Bh).cuda())
        X, _, info, stats = tqr.solve_ls_mixed(dA, dB, 128, iterations=60, precision=tqr.PRECISION_BF16_UPDATES)
        torch.cuda.synchronize()
        st = tqr.refine_stats(stats)[0]
        eta = oracle.ls_backward_error(A, X.cpu().numpy()[:, 0], Bh[:, 0])
        print(f"  {st}, oracle eta {eta:.3e}", flush=True)
        assert int(info.item()) == 0
        if expect_converge:
            assert st["stop"] == tqr.REFINE_CONVERGED and eta < 1e-14
        elif eta >= 1e-14:
            assert st["stop"] in (tqr.REFINE_STAGNATED, tqr.REFINE_MAX_ITERATIONS)
            assert 0.1 < st["eta"] / eta < 10
