"""The oracle: a plain, slow, FP64 CPU reference for the tiled QR path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The product
library (``paper_0707_3548_amd``) never imports it and shares no code with it.

Contents
--------
* ``householder.c`` (loaded here through ctypes) -- unblocked Householder QR,
  Q formation, Q / Q^T application and back substitution, written from the
  problem statement of Sec. 2.1 of Buttari et al. (A = QR by min(m,n)
  Householder reflections; the level-2 column-at-a-time panel algorithm).
* this module -- thin numpy wrappers, sign normalisation, error metrics and
  the least-squares backward error used to judge results.
* ``tiled.py`` -- Algorithm 1 of Sec. 3.1 run sequentially with the four tile
  kernels (GEQRT/DGEQT2, LARFB/DLARFB, TSQRT/DTSQT2, SSRFB/DSSRFB) in numpy,
  the reference for the V and T tiles that the unblocked QR cannot see.
* ``dag.py`` -- the task list of Algorithm 1, a generic read/write hazard
  analysis, the task graph of Sec. 3.3 and its priority levels.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "householder.c")
LIB_SERIAL = os.path.join(_HERE, "liboracle.so")
LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")

EPS = float(np.finfo(np.float64).eps)  # 2**-52, the FP64 machine epsilon


def build(force: bool = True) -> None:
    """Compile the C oracle twice: single thread and OpenMP (fork-join)."""
    for out, extra in ((LIB_SERIAL, []), (LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
            cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11", *extra, _SRC, "-o", out + ".tmp", "-lm"]
            subprocess.check_call(cmd)
            os.replace(out + ".tmp", out)


_libs: dict[str, ctypes.CDLL] = {}


def _lib(omp: bool = False) -> ctypes.CDLL:
    path = LIB_OMP if omp else LIB_SERIAL
    if path not in _libs:
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build(force=False)
        lib = ctypes.CDLL(path)
        i64, dp, i32 = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_int
        lib.orc_geqr2.argtypes = [i64, i64, dp, i64, dp]
        lib.orc_apply_qt.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64]
        lib.orc_apply_q.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64]
        lib.orc_form_q.argtypes = [i64, i64, dp, i64, dp, dp, i64]
        lib.orc_trsv_upper.argtypes = [i64, dp, i64, i64, dp, i64]
        for f in ("orc_geqr2", "orc_apply_qt", "orc_apply_q", "orc_form_q", "orc_trsv_upper", "orc_num_threads"):
            getattr(lib, f).restype = i32
        _libs[path] = lib
    return _libs[path]


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fortran(a) -> np.ndarray:
    return np.array(a, dtype=np.float64, order="F", copy=True)


def num_threads(omp: bool = False) -> int:
    return int(_lib(omp).orc_num_threads())


def geqr2(A, omp: bool = False):
    """Householder QR (Sec. 2.1).  Returns (packed, tau): R in the upper
    triangle of ``packed``, reflector tails below it, ``tau`` the scalars."""
    F = _fortran(A)
    if F.ndim != 2:
        raise ValueError("A must be 2-D")
    m, n = F.shape
    tau = np.zeros(min(m, n))
    rc = _lib(omp).orc_geqr2(m, n, _ptr(F), max(1, m), _ptr(tau))
    if rc != 0:
        raise ValueError(f"orc_geqr2 rejected its arguments ({rc})")
    return F, tau


def r_factor(packed) -> np.ndarray:
    """Thin R (min(m,n) x n, upper trapezoidal) from the packed factor."""
    m, n = packed.shape
    k = min(m, n)
    return np.triu(np.asarray(packed)[:k, :])


def apply_qt(packed, tau, B) -> np.ndarray:
    P = np.asarray(packed, dtype=np.float64, order="F")
    Bf = _fortran(B)
    if Bf.ndim == 1:
        Bf = Bf.reshape(-1, 1, order="F")
    m, n = P.shape
    rc = _lib().orc_apply_qt(m, n, _ptr(P), max(1, m), _ptr(np.ascontiguousarray(tau)), Bf.shape[1], _ptr(Bf), max(1, m))
    if rc != 0:
        raise ValueError("orc_apply_qt rejected its arguments")
    return Bf


def apply_q(packed, tau, B) -> np.ndarray:
    P = np.asarray(packed, dtype=np.float64, order="F")
    Bf = _fortran(B)
    if Bf.ndim == 1:
        Bf = Bf.reshape(-1, 1, order="F")
    m, n = P.shape
    rc = _lib().orc_apply_q(m, n, _ptr(P), max(1, m), _ptr(np.ascontiguousarray(tau)), Bf.shape[1], _ptr(Bf), max(1, m))
    if rc != 0:
        raise ValueError("orc_apply_q rejected its arguments")
    return Bf


def form_q(packed, tau) -> np.ndarray:
    """Thin Q, m x min(m,n)."""
    P = np.asarray(packed, dtype=np.float64, order="F")
    m, n = P.shape
    k = min(m, n)
    Q = np.zeros((m, k), order="F")
    rc = _lib().orc_form_q(m, n, _ptr(P), max(1, m), _ptr(np.ascontiguousarray(tau)), _ptr(Q), max(1, m))
    if rc != 0:
        raise ValueError("orc_form_q rejected its arguments")
    return Q


def trsv_upper(R, X):
    """Back substitution X <- R^{-1} X with the leading n x n upper triangle of
    R.  Returns (X, info); info > 0 is the 1-based index of an exactly zero
    diagonal entry (then X is returned unchanged)."""
    Rf = np.asarray(R, dtype=np.float64, order="F")
    n = Rf.shape[1]
    Xf = _fortran(X)
    if Xf.ndim == 1:
        Xf = Xf.reshape(-1, 1, order="F")
    info = _lib().orc_trsv_upper(n, _ptr(Rf), max(1, Rf.shape[0]), Xf.shape[1], _ptr(Xf), max(1, Xf.shape[0]))
    if info < 0:
        raise ValueError("orc_trsv_upper rejected its arguments")
    return Xf, int(info)


# ---------------------------------------------------------------------------
# sign normalisation and metrics
# ---------------------------------------------------------------------------

def signs(R) -> np.ndarray:
    """d_i = sgn(R_ii), sgn(0) = +1."""
    d = np.sign(np.diag(np.asarray(R)))
    d[d == 0] = 1.0
    return d


def sign_normalize(R, Q=None):
    """R_hat = diag(d) R (and Q_hat = Q diag(d)) so that diag(R_hat) >= 0.
    For full column rank this R_hat is the unique QR factor, which is what
    every R parity check compares."""
    R = np.asarray(R, dtype=np.float64)
    d = signs(R)
    Rh = d[:, None] * R
    if Q is None:
        return Rh
    return Rh, np.asarray(Q) * d[None, :]


def qr(A, omp: bool = False):
    """Sign-normalised thin (Q_hat, R_hat)."""
    P, tau = geqr2(A, omp=omp)
    Q = form_q(P, tau)
    R = r_factor(P)
    Rh, Qh = sign_normalize(R, Q)
    return Qh, Rh


def rel_fro(X, Y) -> float:
    """||X - Y||_F / ||Y||_F."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    den = np.linalg.norm(Y)
    return float(np.linalg.norm(X - Y) / (den if den > 0 else 1.0))


def fact_error(A, Q, R) -> float:
    """||A - QR||_F / ||A||_F."""
    return rel_fro(np.asarray(Q) @ np.asarray(R), A)


def orth_error(Q) -> float:
    """||Q^T Q - I||_F."""
    Q = np.asarray(Q)
    return float(np.linalg.norm(Q.T @ Q - np.eye(Q.shape[1])))


def lstsq(A, B, omp: bool = False):
    """min ||A x - b|| for m >= n and full column rank, via the oracle's QR:
    x = R_hat^{-1} (Q_hat^T b)[0:n].  Returns (X, info) as trsv_upper.
    ``omp`` runs the factorisation on the OpenMP build (the same bits)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if m < n:
        raise ValueError("lstsq needs m >= n")
    P, tau = geqr2(A, omp=omp)
    C = apply_qt(P, tau, B)
    R = r_factor(P)
    return trsv_upper(R[:n, :n], C[:n])


def ls_backward_error(A, x, b, omp: bool = False) -> float:
    """Normwise least-squares backward error estimate (Karlson--Walden):
        eta(x) = ||(A^T A + mu^2 I)^{-1/2} A^T r|| / (||x|| ||A||_F),
        r = b - A x,  mu = ||r|| / ||x||.
    With Rt the R factor of [A; mu I] (= R factor of [R_A; mu I]),
    (A^T A + mu^2 I)^{-1/2} A^T r has the norm of Rt^{-T} A^T r.
    The R factor is taken from the oracle's own QR (``omp``: its OpenMP
    build, which gives the same bits)."""
    A = np.asarray(A, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    m, n = A.shape
    r = b - A @ x
    nx = np.linalg.norm(x)
    if nx == 0:
        return float(np.linalg.norm(A.T @ r))
    mu = np.linalg.norm(r) / nx
    P, _ = geqr2(A, omp=omp)
    RA = r_factor(P)[:n, :n]
    aug = np.vstack([RA, mu * np.eye(n)])
    P2, _ = geqr2(aug, omp=omp)
    Rt = r_factor(P2)[:n, :n]
    g = A.T @ r
    # solve Rt^T y = g by forward substitution (Rt^T is lower triangular)
    y = np.zeros(n)
    for i in range(n):
        y[i] = (g[i] - Rt[:i, i] @ y[:i]) / Rt[i, i]
    return float(np.linalg.norm(y) / (nx * np.linalg.norm(A)))


def ls_backward_error_exact(A, x, b) -> float:
    """Exact normwise backward error of a least-squares solution on a tiny
    problem (Walden--Karlson--Sun):  sigma_min([A, mu (I - r r^T/||r||^2)])
    with mu = ||r||/||x||, normalised by ||A||_F.  SVD-based; test use only."""
    A = np.asarray(A, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    m = A.shape[0]
    r = b - A @ x
    nr = np.linalg.norm(r)
    nx = np.linalg.norm(x)
    mu = nr / nx
    if nr == 0:
        return 0.0
    M = np.hstack([A, mu * (np.eye(m) - np.outer(r, r) / nr**2)])
    s = np.linalg.svd(M, compute_uv=False)  # m values: M is m x (n + m)
    return float(min(mu, s[-1]) / np.linalg.norm(A))


def flops_standard(m: int, n: int) -> float:
    """2 n^2 (m - n/3): the Householder QR operation count of Sec. 2.1."""
    return 2.0 * n * n * (m - n / 3.0)
