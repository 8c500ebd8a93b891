"""Pins of the FP64 oracle against facts that do not come from the oracle:
closed forms, textbook routines (Cholesky, LAPACK through numpy), invariants
of the QR factorisation, exact special cases and the least-squares backward
error of Waldén, Karlson and Sun.  CPU only."""
import numpy as np
import pytest

import oracle
from conftest import golden_blocks
from paper_0707_3548_amd import workloads

EPS = oracle.EPS


def test_closed_form_2x2_fixture():
    A, R_raw, R_hat, tau = golden_blocks("qr_2x2.txt", [2, 2, 2, 1])
    P, t = oracle.geqr2(A)
    R = oracle.r_factor(P)
    np.testing.assert_allclose(R, R_raw, rtol=0, atol=4 * EPS * 5)
    np.testing.assert_allclose(oracle.sign_normalize(R), R_hat, rtol=0, atol=4 * EPS * 5)
    np.testing.assert_allclose(t, tau[0], rtol=0, atol=4 * EPS)


@pytest.mark.parametrize("seed", range(20))
def test_closed_form_2x2_random(seed):
    g = np.random.default_rng(seed)
    a, b, c, d = g.standard_normal(4)
    r11 = np.hypot(a, c)
    exp = np.array([[r11, (a * b + c * d) / r11], [0.0, abs(a * d - b * c) / r11]])
    _, R = oracle.qr(np.array([[a, b], [c, d]]))
    np.testing.assert_allclose(R, exp, rtol=1e-13, atol=1e-13 * np.abs(exp).max())


def test_closed_form_3x3_fixture():
    A, R_hat = golden_blocks("qr_3x3.txt", [3, 3])
    Q, R = oracle.qr(A)
    assert oracle.rel_fro(R, R_hat) < 10 * EPS
    assert oracle.fact_error(A, Q, R) < 10 * EPS


@pytest.mark.parametrize("shape", [(4, 3), (6, 6), (9, 5), (12, 2)])
def test_cholesky_of_normal_matrix(shape):
    """R_hat is the upper Cholesky factor of A^T A (well-conditioned A)."""
    m, n = shape
    g = np.random.default_rng(m * 31 + n)
    Qr, _ = np.linalg.qr(g.standard_normal((m, n)))
    A = Qr @ np.diag(np.linspace(1.0, 3.0, n)) @ np.linalg.qr(g.standard_normal((n, n)))[0]  # cond 3
    L = np.linalg.cholesky(A.T @ A)
    _, R = oracle.qr(A)
    assert oracle.rel_fro(R[:n, :n], L.T) < 100 * EPS * 9


@pytest.mark.parametrize("shape", [(200, 120), (333, 333), (1000, 64), (50, 1), (1, 1)])
def test_matches_lapack_sign_normalised(shape):
    m, n = shape
    A = workloads.gaussian(m, n, seed=m + n)
    _, R_lapack = np.linalg.qr(A)
    _, R = oracle.qr(A)
    kappa = np.linalg.cond(A) if n > 1 else 1.0
    assert oracle.rel_fro(R, oracle.sign_normalize(R_lapack)) < 10 * kappa * n * EPS


@pytest.mark.parametrize("shape", [(64, 64), (300, 100), (513, 257), (1024, 16)])
def test_backward_and_orthogonality(shape):
    m, n = shape
    A = workloads.gaussian(m, n, seed=3)
    Q, R = oracle.qr(A)
    assert oracle.fact_error(A, Q, R) <= 10 * n * EPS
    assert oracle.orth_error(Q) <= 10 * n * EPS


def test_row_permutation_invariance():
    A = workloads.gaussian(80, 30, seed=5)
    perm = np.random.default_rng(1).permutation(80)
    _, R1 = oracle.qr(A)
    _, R2 = oracle.qr(A[perm])
    assert oracle.rel_fro(R2, R1) < 1e-13


def test_positive_column_scaling():
    A = workloads.gaussian(60, 20, seed=6)
    D = np.exp(np.random.default_rng(2).uniform(-2, 2, 20))
    _, R1 = oracle.qr(A)
    _, R2 = oracle.qr(A * D[None, :])
    assert oracle.rel_fro(R2, R1 * D[None, :]) < 1e-13


def test_orthogonal_input_gives_identity():
    Qin, _ = np.linalg.qr(workloads.gaussian(40, 40, seed=7))
    _, R = oracle.qr(Qin)
    assert np.abs(R - np.eye(40)).max() < 100 * EPS


def test_upper_triangular_input_is_returned_exactly():
    """sigma^2 == 0 at every step: tau = 0 and H = I, also for a negative
    diagonal entry, so the packed output equals the input bit for bit."""
    g = np.random.default_rng(8)
    U = np.triu(g.standard_normal((12, 9)))
    U[2, 2] = -abs(U[2, 2])
    P, tau = oracle.geqr2(U)
    assert np.array_equal(P, U)
    assert np.all(tau == 0)


def test_zero_and_rank_deficient_do_not_nan():
    P, tau = oracle.geqr2(np.zeros((7, 5)))
    assert np.all(P == 0) and np.all(tau == 0)
    A = workloads.gaussian(30, 10, seed=9)
    A[:, 4] = A[:, 1] + A[:, 2]
    P, tau = oracle.geqr2(A)
    assert np.all(np.isfinite(P)) and np.all(np.isfinite(tau))


def test_qt_applied_to_a_gives_r():
    A = workloads.gaussian(50, 20, seed=10)
    P, tau = oracle.geqr2(A)
    C = oracle.apply_qt(P, tau, A)
    assert np.abs(C[20:]).max() < 50 * EPS * np.abs(A).max()
    np.testing.assert_allclose(np.triu(C[:20]), oracle.r_factor(P), atol=50 * EPS * np.abs(A).max())


def test_apply_q_inverts_apply_qt():
    A = workloads.gaussian(40, 15, seed=11)
    P, tau = oracle.geqr2(A)
    B = workloads.gaussian(40, 3, seed=12)
    B2 = oracle.apply_q(P, tau, oracle.apply_qt(P, tau, B))
    assert oracle.rel_fro(B2, B) < 50 * EPS


def test_trsv_upper():
    g = np.random.default_rng(13)
    R = np.triu(g.standard_normal((25, 25))) + 5 * np.eye(25)
    x = g.standard_normal((25, 2))
    X, info = oracle.trsv_upper(R, R @ x)
    assert info == 0
    np.testing.assert_allclose(X, x, rtol=1e-12, atol=1e-12)
    R[7, 7] = 0.0
    X, info = oracle.trsv_upper(R, R @ x)
    assert info == 8


def test_openmp_build_is_bitwise_identical():
    A = workloads.gaussian(300, 200, seed=14)
    P1, t1 = oracle.geqr2(A)
    P2, t2 = oracle.geqr2(A, omp=True)
    assert np.array_equal(P1, P2) and np.array_equal(t1, t2)


def test_least_squares_consistent_recovers_x():
    A, _, x = workloads.ls_problem(120, 40, 1e3, seed=15)
    X, info = oracle.lstsq(A, A @ x)
    assert info == 0
    assert np.linalg.norm(X - x) / np.linalg.norm(x) < 1e3 * 40 * EPS


@pytest.mark.parametrize("cond", [1e2, 1e5, 1e8])
def test_least_squares_matches_lapack_and_is_backward_stable(cond):
    A, b, _ = workloads.ls_problem(90, 30, cond, seed=16)
    X, info = oracle.lstsq(A, b)
    xl = np.linalg.lstsq(A, b, rcond=None)[0]
    assert info == 0
    assert np.linalg.norm(X - xl) / np.linalg.norm(xl) < cond * 1e-12
    assert oracle.ls_backward_error(A, X[:, 0], b[:, 0]) < 1e-15


@pytest.mark.parametrize("cond", [1e2, 1e5, 1e8])
def test_backward_error_estimate_vs_exact(cond):
    """The Karlson--Walden estimate lies within a factor sqrt(2) of the exact
    backward error sigma_min([A, mu (I - r r^T / ||r||^2)])."""
    A, b, _ = workloads.ls_problem(40, 12, cond, seed=17)
    x = np.linalg.lstsq(A, b, rcond=None)[0][:, 0]
    x = x * (1 + 1e-7 * np.random.default_rng(3).standard_normal(12))  # a visibly perturbed solution
    est = oracle.ls_backward_error(A, x, b[:, 0])
    exact = oracle.ls_backward_error_exact(A, x, b[:, 0])
    assert exact > 0
    assert 1 / np.sqrt(2) - 1e-6 <= est / exact <= np.sqrt(2) + 1e-6


def test_flop_count():
    assert oracle.flops_standard(8192, 8192) == pytest.approx(7.330e11, rel=1e-3)
    assert oracle.flops_standard(512, 512) == pytest.approx(1.790e8, rel=1e-3)


@pytest.mark.parametrize("shape", [(6, 4), (50, 50), (200, 37)])
def test_packed_reflectors_match_lapack_raw(shape):
    """LAPACK's dgeqrf (numpy mode='raw') uses the same reflector convention
    (beta = -sgn(alpha) ||.||, tau = (beta - alpha)/beta, v = x/(alpha - beta)),
    so the whole packed output -- V below the diagonal, R above, tau -- agrees."""
    m, n = shape
    A = workloads.gaussian(m, n, seed=m)
    h, tau_l = np.linalg.qr(A, mode="raw")
    P, tau = oracle.geqr2(A)
    kappa = np.linalg.cond(A)
    assert np.abs(h.T - P).max() < 10 * kappa * n * EPS * np.abs(A).max()
    assert np.abs(tau_l - tau).max() < 10 * kappa * n * EPS
