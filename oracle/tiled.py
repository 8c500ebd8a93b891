"""Algorithm 1 of Buttari et al. (Sec. 3.1), run sequentially in numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring): the reference for the
V and T tiles that the tiled method writes next to R, which the unblocked
oracle in ``householder.c`` cannot see.  It follows the four elementary
operations of Sec. 3.1 in the paper's order, with one refinement that the
paper leaves open: each kernel works on inner blocks of ``ib`` columns and
keeps one ib x ib upper-triangular T per inner block (``ib == b`` is exactly
the paper's b x b T).

Readings of the paper used here:
* The kernels are written as applying ``(I - V T V^T)``; with the forward,
  column-wise T of the compact WY representation (Schreiber and Van Loan,
  cited in Sec. 2.1), ``H_1 ... H_ib = I - V T V^T``, so the factorisation
  must apply its transpose, ``I - V T^T V^T``.  That is what is done below.
* Loop bounds of Algorithm 1: i = k+1, k+2, ..., p.
* Matrices whose sizes are not multiples of b are zero-padded to whole tiles.
  Zero padding rows give reflector entries that are exactly zero and zero
  padding columns give tau = 0, so R[0:n, 0:n] is unchanged.
* TSQRT only touches the upper triangle of the diagonal tile; its strictly
  lower part still holds V_kk.

Storage: ``tiles[i, j]`` is the b x b tile (i, j); ``T[i, k]`` the ib x b
slot for the reflectors of tile (i, k): inner block s occupies columns
s*ib .. s*ib+ib-1.  Indices are 0-based.
"""
from __future__ import annotations

import numpy as np


def householder(alpha: float, x: np.ndarray):
    """Reflector H = I - tau [1; v][1; v]^T with H [alpha; x] = [beta; 0].
    beta = -sgn(alpha) sqrt(alpha^2 + x^T x), sgn(0) = +1.  x^T x == 0 gives
    tau = 0 and H = I (alpha is kept, even if negative)."""
    sigma2 = float(x @ x)
    if sigma2 == 0.0:
        return alpha, 0.0, np.zeros_like(x)
    norm = np.sqrt(alpha * alpha + sigma2)
    beta = -norm if alpha >= 0.0 else norm
    tau = (beta - alpha) / beta
    return beta, tau, x / (alpha - beta)


def to_tiles(A: np.ndarray, b: int) -> np.ndarray:
    m, n = A.shape
    p, q = -(-m // b), -(-n // b)
    P = np.zeros((p * b, q * b))
    P[:m, :n] = A
    return P.reshape(p, b, q, b).transpose(0, 2, 1, 3).copy()


def from_tiles(tiles: np.ndarray, m: int, n: int) -> np.ndarray:
    p, q, b, _ = tiles.shape
    return tiles.transpose(0, 2, 1, 3).reshape(p * b, q * b)[:m, :n].copy()


def _unit_lower(Akk: np.ndarray, c0: int, ib: int) -> np.ndarray:
    """V of inner block s of a diagonal tile: rows c0..b-1, columns
    c0..c0+ib-1, unit diagonal, zeros above it."""
    V = np.tril(Akk[c0:, c0:c0 + ib], -1)
    V[np.arange(ib), np.arange(ib)] = 1.0
    return V


# --- the four elementary operations (Sec. 3.1) ------------------------------

def geqrt(Akk: np.ndarray, ib: int) -> np.ndarray:
    """DGEQT2: A_kk <- V_kk, R_kk;  returns T_kk (ib x b)."""
    b = Akk.shape[0]
    T = np.zeros((ib, b))
    for c0 in range(0, b, ib):
        for jj in range(ib):
            j = c0 + jj
            beta, tau, v = householder(Akk[j, j], Akk[j + 1:, j].copy())
            Akk[j, j] = beta
            Akk[j + 1:, j] = v
            for c in range(j + 1, c0 + ib):
                w = Akk[j, c] + v @ Akk[j + 1:, c]
                Akk[j, c] -= tau * w
                Akk[j + 1:, c] -= tau * w * v
            T[jj, j] = tau
            if jj > 0:
                V = _unit_lower(Akk, c0, ib)
                z = V[:, :jj].T @ V[:, jj]
                T[:jj, j] = -tau * (T[:jj, c0:c0 + jj] @ z)
        if c0 + ib < b:
            V = _unit_lower(Akk, c0, ib)
            Ts = T[:, c0:c0 + ib]
            C = Akk[c0:, c0 + ib:]
            W = Ts.T @ (V.T @ C)
            Akk[c0:, c0 + ib:] = C - V @ W
    return T


def larfb(Akj: np.ndarray, Akk: np.ndarray, T: np.ndarray, transpose: bool = True) -> None:
    """DLARFB: A_kj <- (I - V_kk T_kk^T V_kk^T) A_kj  (or with T when
    ``transpose`` is False, i.e. applying Q instead of Q^T)."""
    b = Akk.shape[0]
    ib = T.shape[0]
    blocks = range(0, b, ib) if transpose else range(b - ib, -1, -ib)
    for c0 in blocks:
        V = _unit_lower(Akk, c0, ib)
        Ts = T[:, c0:c0 + ib]
        C = Akj[c0:, :]
        W = (Ts.T if transpose else Ts) @ (V.T @ C)
        Akj[c0:, :] = C - V @ W


def tsqrt(Akk: np.ndarray, Aik: np.ndarray, ib: int) -> np.ndarray:
    """DTSQT2: QR of [R_kk; A_ik].  R_kk (upper triangle of A_kk) <- R~_kk,
    A_ik <- V_ik; returns T_ik (ib x b).  The identity block on top of V_ik
    is implicit; the strictly lower part of A_kk is not touched."""
    b = Akk.shape[0]
    T = np.zeros((ib, b))
    for c0 in range(0, b, ib):
        for jj in range(ib):
            j = c0 + jj
            beta, tau, v = householder(Akk[j, j], Aik[:, j].copy())
            Akk[j, j] = beta
            Aik[:, j] = v
            for c in range(j + 1, c0 + ib):
                w = Akk[j, c] + v @ Aik[:, c]
                Akk[j, c] -= tau * w
                Aik[:, c] -= tau * w * v
            T[jj, j] = tau
            if jj > 0:
                # the unit entries of [e_j; v_j] sit in distinct rows of R,
                # so only the V_ik parts contribute to V^T v
                z = Aik[:, c0:j].T @ v
                T[:jj, j] = -tau * (T[:jj, c0:c0 + jj] @ z)
        if c0 + ib < b:
            V = Aik[:, c0:c0 + ib]
            Ts = T[:, c0:c0 + ib]
            W = Ts.T @ (Akk[c0:c0 + ib, c0 + ib:] + V.T @ Aik[:, c0 + ib:])
            Akk[c0:c0 + ib, c0 + ib:] -= W
            Aik[:, c0 + ib:] -= V @ W
    return T


def ssrfb(Akj: np.ndarray, Aij: np.ndarray, Vik: np.ndarray, T: np.ndarray, transpose: bool = True) -> None:
    """DSSRFB: [A_kj; A_ij] <- (I - [I; V_ik] T_ik^T [I; V_ik]^T) [A_kj; A_ij]
    (with T instead of T^T when ``transpose`` is False)."""
    b = Vik.shape[0]
    ib = T.shape[0]
    blocks = range(0, b, ib) if transpose else range(b - ib, -1, -ib)
    for c0 in blocks:
        V = Vik[:, c0:c0 + ib]
        Ts = T[:, c0:c0 + ib]
        W = (Ts.T if transpose else Ts) @ (Akj[c0:c0 + ib, :] + V.T @ Aij)
        Akj[c0:c0 + ib, :] -= W
        Aij -= V @ W


# --- Algorithm 1 --------------------------------------------------------------

def factor(A: np.ndarray, b: int, ib: int):
    """Tiled QR of A (m x n, m >= n) in Algorithm 1 order.
    Returns (tiles, T) with T of shape (p, q, ib, b)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if b < 1 or ib < 1 or b % ib != 0:
        raise ValueError("need b >= 1 and ib dividing b")
    tiles = to_tiles(A, b)
    p, q = tiles.shape[:2]
    T = np.zeros((p, q, ib, b))
    for k in range(min(p, q)):
        T[k, k] = geqrt(tiles[k, k], ib)
        for j in range(k + 1, q):
            larfb(tiles[k, j], tiles[k, k], T[k, k])
        for i in range(k + 1, p):
            T[i, k] = tsqrt(tiles[k, k], tiles[i, k], ib)
            for j in range(k + 1, q):
                ssrfb(tiles[k, j], tiles[i, j], tiles[i, k], T[i, k])
    return tiles, T


def _b_tiles(B: np.ndarray, b: int, p: int) -> np.ndarray:
    B = np.asarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
    P = np.zeros((p * b, B.shape[1]))
    P[:B.shape[0]] = B
    return P.reshape(p, b, B.shape[1]).copy()


def apply_qt(tiles: np.ndarray, T: np.ndarray, B: np.ndarray) -> np.ndarray:
    """B <- Q^T B with the tiled factors (same transformations, same order)."""
    p, q, b, _ = tiles.shape
    m = B.shape[0]
    Bt = _b_tiles(B, b, p)
    for k in range(min(p, q)):
        larfb(Bt[k], tiles[k, k], T[k, k])
        for i in range(k + 1, p):
            ssrfb(Bt[k], Bt[i], tiles[i, k], T[i, k])
    return Bt.reshape(p * b, -1)[:m]


def apply_q(tiles: np.ndarray, T: np.ndarray, B: np.ndarray) -> np.ndarray:
    """B <- Q B: the transformations of apply_qt, transposed, in reverse."""
    p, q, b, _ = tiles.shape
    m = B.shape[0]
    Bt = _b_tiles(B, b, p)
    for k in reversed(range(min(p, q))):
        for i in reversed(range(k + 1, p)):
            ssrfb(Bt[k], Bt[i], tiles[i, k], T[i, k], transpose=False)
        larfb(Bt[k], tiles[k, k], T[k, k], transpose=False)
    return Bt.reshape(p * b, -1)[:m]


def r_factor(tiles: np.ndarray, m: int, n: int) -> np.ndarray:
    return np.triu(from_tiles(tiles, m, n)[:min(m, n), :])


def form_q(tiles: np.ndarray, T: np.ndarray, m: int, n: int) -> np.ndarray:
    k = min(m, n)
    E = np.zeros((m, k))
    E[np.arange(k), np.arange(k)] = 1.0
    return apply_q(tiles, T, E)
