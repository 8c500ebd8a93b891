"""Parity at the sizes the benchmark measures, and on grids large enough for
every scheduler mechanism (GPU).

* The square 8192 x 8192 N(0,1) factorisation (tile_b 256, inner_ib 16)
  through the plain boundary call tqr_factor, and the tall-skinny
  65536 x 1024 U[-1,1] one: the sign-normalised R against the unblocked
  oracle (Sec. 2.1) to 1e-10 relative, and the backward error
  ||A - QR||_F / ||A||_F and the orthogonality of Q within 10 n eps, both
  estimated on a block of 16 random orthonormal directions through the
  library's own application of Q (the thin Q of an 8192^2 problem is too
  large to form for a test).
* Grids with TSQRT helper tasks, the pipelined R_kk chain of 6+ tile rows and
  the next-column SSRFB pipelines (1536^2 at b = 256, 1024^2 at b = 128) and a
  tall one (4096 x 512 at b = 128): R against the oracle, and the result
  bitwise the same with 1, 7 and all workgroups under all three priority
  policies (every legal schedule applies the same operations to every tile in
  the same order, Algorithm 1).

The oracle runs on its OpenMP build (bitwise the same as the serial one).
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

EPS = oracle.EPS


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)


def oracle_r(A):
    P, _ = oracle.geqr2(A, omp=True)
    n = A.shape[1]
    return oracle.sign_normalize(oracle.r_factor(P)[:n, :n])


def cond2_of_triangular(R, iters=60, seed=0):
    """kappa_2 of an upper-triangular R (= that of A) by power iteration on
    R^T R and inverse iteration through two triangular solves."""
    from scipy.linalg import solve_triangular
    g = np.random.default_rng(seed)
    x = g.standard_normal(R.shape[0])
    for _ in range(iters):
        x = R.T @ (R @ x)
        x /= np.linalg.norm(x)
    smax = np.sqrt(np.linalg.norm(R.T @ (R @ x)))
    y = g.standard_normal(R.shape[0])
    for _ in range(iters):
        y = solve_triangular(R, solve_triangular(R, y, trans="T"))
        y /= np.linalg.norm(y)
    z = solve_triangular(R, solve_triangular(R, y, trans="T"))
    smin = 1.0 / np.sqrt(np.linalg.norm(z))
    return smax / smin


def implicit_q_checks(torch, tqr, A, dA, T, b, ib, k=16, seed=7):
    """Estimates of ||A - QR||_F/||A||_F and ||Q^T Q - I||_F from a block X
    of k random orthonormal directions: ||(A - QR) X||_F^2 is about
    (k/n) ||A - QR||_F^2, so the estimate scales it by sqrt(n/k)."""
    m, n = A.shape
    g = np.random.default_rng(seed)
    X, _ = np.linalg.qr(g.standard_normal((n, k)))
    dX = torch.from_numpy(X).cuda()
    R = torch.triu(dA[:n, :])
    Y = torch.zeros((k, m), dtype=torch.float64, device="cuda").t()  # m x k column-major
    Y[:n] = R @ dX
    tqr.apply_q(dA, T, Y, b, ib)
    dAh = torch.from_numpy(np.asarray(A)).cuda()
    AX = dAh @ dX
    scale = np.sqrt(n / k)
    e_fact = float(torch.linalg.norm(AX - Y)) / float(torch.linalg.norm(dAh)) * scale
    # orthogonality: Q^T (Q [Z; 0]) = [Z; 0] for Z with orthonormal columns
    Z = torch.zeros((k, m), dtype=torch.float64, device="cuda").t()
    Z[:n] = dX
    W = Z.clone()
    tqr.apply_q(dA, T, W, b, ib)
    tqr.apply_qt(dA, T, W, b, ib)
    torch.cuda.synchronize()
    e_orth = float(torch.linalg.norm(W - Z)) * scale
    return e_fact, e_orth


@pytest.mark.parametrize("name,m,n,seed,dist", [("square 8192^2 N(0,1)", 8192, 8192, 0, "gaussian"),
                                                ("tall-skinny 65536x1024 U[-1,1]", 65536, 1024, 1, "uniform")])
def test_benchmark_sizes_match_oracle(name, m, n, seed, dist):
    torch = _torch()
    from paper_0707_3548_amd import tqr, workloads
    b, ib = 256, 16
    _say(f"case measured {name}: generating")
    A = workloads.gaussian(m, n, seed=seed) if dist == "gaussian" else workloads.uniform(m, n, seed=seed)
    dA = tqr.fortran(torch.from_numpy(A).cuda())
    ws = tqr.Workspace(m, n, 0, b, ib)
    _say(f"case measured {name}: tqr_factor (no options) b={b} ib={ib}")
    tqr.factor_plain(dA, b, ib, ws)
    torch.cuda.synchronize()
    R = oracle.sign_normalize(np.triu(dA[:n, :].cpu().numpy()))
    _say(f"case measured {name}: oracle on {oracle.num_threads(omp=True)} threads")
    R_or = oracle_r(A)
    err = oracle.rel_fro(R, R_or)
    kappa = cond2_of_triangular(R_or)
    _say(f"case measured {name}: e_R = {err:.3e}, kappa_2(A) = {kappa:.3e}")
    assert err < 1e-10
    e_fact, e_orth = implicit_q_checks(torch, tqr, A, dA, ws.T, b, ib)
    _say(f"case measured {name}: ||A-QR||/||A|| ~ {e_fact:.3e}, ||Q^TQ-I|| ~ {e_orth:.3e} (bound {10 * n * EPS:.3e})")
    assert e_fact <= 10 * n * EPS
    assert e_orth <= 10 * n * EPS


# grids where the helpers are on (b >= 128, p <= 2q), with 6+ tile rows, and a
# tall grid (helpers off, long pipelined chains)
GRIDS = [(1536, 1536, 256, 16), (1024, 1024, 128, 16), (4096, 512, 128, 16)]


@pytest.mark.parametrize("m,n,b,ib", GRIDS)
def test_large_grids_match_oracle_and_are_schedule_invariant(m, n, b, ib):
    torch = _torch()
    from paper_0707_3548_amd import tqr, workloads
    A = workloads.gaussian(m, n, seed=m + 7 * n + b)
    R_or = oracle_r(A)
    ref = None
    for wg in (0, 1, 7):
        for pol in (tqr.POLICY_COLUMN, tqr.POLICY_PAPER, tqr.POLICY_LOOKAHEAD):
            _say(f"case grid m={m} n={n} b={b} ib={ib} workgroups={wg} policy={pol}")
            dA = tqr.fortran(torch.from_numpy(A).cuda())
            ws = tqr.Workspace(m, n, 0, b, ib)
            status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
            tqr.factor(dA, b, ib, ws, workgroups=wg, policy=pol, status=status)
            torch.cuda.synchronize()
            assert int(status.item()) == 0
            out = (dA.cpu().numpy(), ws.T.cpu().numpy())
            if ref is None:
                ref = out
                R = oracle.sign_normalize(np.triu(out[0][:n, :]))
                assert oracle.rel_fro(R, R_or) < 1e-10
            else:
                assert np.array_equal(out[0], ref[0]), (wg, pol)
                assert np.array_equal(out[1], ref[1]), (wg, pol)


# Least squares at the size the benchmark's mixed-precision leg measures:
# 16384 x 4096, A = U diag(s) V^T with s log-spaced (cond in {1e2, 1e5, 1e8}),
# U and V from QR of Gaussians, b = A x + 1e-6 N(0,1).
@pytest.mark.parametrize("cond", [1e2, 1e5, 1e8])
def test_least_squares_16384x4096_fp64_and_mixed_match_oracle(cond):
    torch = _torch()
    from paper_0707_3548_amd import tqr, workloads
    m, n, b, ib = 16384, 4096, 256, 16
    _say(f"case LS {m}x{n} cond={cond:g}: generating")
    A, Bh, _ = workloads.ls_problem(m, n, cond, seed=41, nrhs=1)
    dA0 = tqr.fortran(torch.from_numpy(A).cuda())
    dB0 = tqr.fortran(torch.from_numpy(Bh).cuda())
    _say(f"case LS cond={cond:g}: FP64 tqr_solve_ls")
    dA, dB = dA0.clone(), dB0.clone()
    _, info = tqr.solve_ls(dA, dB, b, ib)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    x64 = dB[:n, 0].cpu().numpy()
    # beyond 1 / u32 the FP32-update factor is no usable preconditioner: the
    # mixed solver is run with the FP64 factor there (its FP32 attempt is
    # checked to report its stagnation honestly in tests/test_mixed.py)
    prec = tqr.PRECISION_FP32_UPDATES if cond < 1e7 else tqr.PRECISION_FP64
    _say(f"case LS cond={cond:g}: mixed (factor precision {prec} + FP64 CGLS)")
    X, _, info, stats = tqr.solve_ls_mixed(dA0, dB0, b, iterations=30, precision=prec)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    xmx = X[:, 0].cpu().numpy()
    st = tqr.refine_stats(stats)[0]
    _say(f"case LS cond={cond:g}: oracle lstsq and backward errors on {oracle.num_threads(omp=True)} threads")
    xo, _ = oracle.lstsq(A, Bh, omp=True)
    xo = xo[:, 0]
    f64 = np.linalg.norm(x64 - xo) / np.linalg.norm(xo)
    fmx = np.linalg.norm(xmx - xo) / np.linalg.norm(xo)
    e64 = oracle.ls_backward_error(A, x64, Bh[:, 0], omp=True)
    emx = oracle.ls_backward_error(A, xmx, Bh[:, 0], omp=True)
    _say(f"case LS cond={cond:g}: FP64 forward {f64:.3e} eta {e64:.3e}; mixed forward {fmx:.3e} eta {emx:.3e} "
         f"({st['iterations']} iterations, stop {st['stop']}, device eta {st['eta']:.3e})")
    assert f64 < cond * 1e-13 and e64 < 1e-14
    assert fmx < cond * 1e-13 and emx < 1e-14
    assert st["stop"] in (tqr.REFINE_CONVERGED, tqr.REFINE_STAGNATED)
