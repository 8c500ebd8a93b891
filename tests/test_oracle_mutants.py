"""The oracle's pins must catch plausible mistakes.  Each case below plants
one mistake in a copy of the oracle's C source (on the CPU, in a temporary
directory), builds it and checks that at least one pin fails.  The pins used
here are the same kinds as in test_oracle.py: closed-form fixtures, LAPACK's
packed output, the factorisation/orthogonality invariants and the exact
upper-triangular case."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from conftest import golden_blocks
from paper_0707_3548_amd import workloads

SRC = os.path.join(os.path.dirname(oracle.__file__), "householder.c")

MUTANTS = {
    "tau_dropped_from_update": ("        w *= t;\n            colc[j] -= w;", "        colc[j] -= w;"),
    "beta_sign_flipped": ("(alpha >= 0.0) ? -norm : norm", "(alpha >= 0.0) ? norm : -norm"),
    "norm_includes_diagonal": ("for (int64_t i = j + 1; i < m; ++i)\n            sigma2", "for (int64_t i = j; i < m; ++i)\n            sigma2"),
    "dot_drops_leading_term": ("double w = colc[j];", "double w = 0.0;"),
    "tau_sign": ("double t = (beta - alpha) / beta;", "double t = (alpha - beta) / beta;"),
    "v_scaled_wrong_way": ("colj[i] = colj[i] / denom;", "colj[i] = colj[i] * denom;"),
    "apply_q_wrong_order": ("for (int64_t j = kmax - 1; j >= 0; --j)", "for (int64_t j = 0; j < kmax; ++j)"),
    "trsv_transposed_operand": ("s -= R[j * ldr + i] * x[j];", "s -= R[i * ldr + j] * x[j];"),
    "update_skips_last_row": ("for (int64_t i = j + 1; i < m; ++i)\n                colc[i] -= w * colj[i];", "for (int64_t i = j + 1; i < m - 1; ++i)\n                colc[i] -= w * colj[i];"),
}


def _load(path):
    lib = ctypes.CDLL(path)
    i64, dp = ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    lib.orc_geqr2.argtypes = [i64, i64, dp, i64, dp]
    lib.orc_form_q.argtypes = [i64, i64, dp, i64, dp, dp, i64]
    lib.orc_trsv_upper.argtypes = [i64, dp, i64, i64, dp, i64]
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _pins(lib):
    """Return the names of the pins that fail for this library."""
    failed = []
    eps = oracle.EPS

    def qr(A):
        F = np.array(A, dtype=np.float64, order="F")
        m, n = F.shape
        tau = np.zeros(min(m, n))
        lib.orc_geqr2(m, n, _p(F), m, _p(tau))
        Q = np.zeros((m, min(m, n)), order="F")
        lib.orc_form_q(m, n, _p(F), m, _p(tau), _p(Q), m)
        return F, tau, Q

    A, R_raw, _, tau2 = golden_blocks("qr_2x2.txt", [2, 2, 2, 1])
    P, t, _ = qr(A)
    if not (np.allclose(np.triu(P), R_raw, atol=1e-14) and np.allclose(t, tau2[0], atol=1e-14)):
        failed.append("fixture_2x2")
    A3, R3 = golden_blocks("qr_3x3.txt", [3, 3])
    P, t, _ = qr(A3)
    if oracle.rel_fro(oracle.sign_normalize(np.triu(P)), R3) > 1e-14:
        failed.append("fixture_3x3")
    A = workloads.gaussian(40, 25, seed=1)
    P, t, Q = qr(A)
    h, tl = np.linalg.qr(A, mode="raw")
    if np.abs(h.T - P).max() > 1e-11 or np.abs(tl - t).max() > 1e-11:
        failed.append("lapack_raw")
    R = np.triu(P[:25])
    if oracle.fact_error(A, Q, R) > 10 * 25 * eps or oracle.orth_error(Q) > 10 * 25 * eps:
        failed.append("invariants")
    U = np.triu(workloads.gaussian(9, 9, seed=2))
    P, t, _ = qr(U)
    if not (np.array_equal(P, U) and np.all(t == 0)):
        failed.append("upper_triangular_exact")
    Rm = np.asfortranarray(np.triu(workloads.gaussian(12, 12, seed=3)) + 4 * np.eye(12))
    x = workloads.gaussian(12, 1, seed=4)
    X = np.asfortranarray(Rm @ x)
    lib.orc_trsv_upper(12, _p(Rm), 12, 1, _p(X), 12)
    if np.abs(X - x).max() > 1e-12:
        failed.append("trsv")
    return failed


def test_unmutated_source_passes_every_pin(tmp_path):
    out = tmp_path / "lib.so"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", SRC, "-o", str(out), "-lm"])
    assert _pins(_load(str(out))) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    path = tmp_path / "mut.c"
    path.write_text(src.replace(old, new))
    out = tmp_path / "mut.so"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", str(path), "-o", str(out), "-lm"])
    assert _pins(_load(str(out))), f"no pin caught the planted mistake {name}"
