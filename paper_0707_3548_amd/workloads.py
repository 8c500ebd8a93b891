"""Seeded synthetic inputs for the tiled QR workloads.

This module only draws numbers; it holds none of the factorisation's
arithmetic, and both the HIP path's tests and the CPU oracle take their
inputs from it.  Every generator uses numpy's PCG64 with a seed; separate
quantities (the matrix, the singular vectors, x_true, the noise) come from
independent child streams of one ``SeedSequence`` so that changing one size
does not shift the others.

The paper (Buttari et al.) states no input distribution; the workloads are:

* ``gaussian``      -- i.i.d. N(0, 1) entries (square and tall QR).
* ``uniform``       -- i.i.d. U[-1, 1] entries (tall-skinny QR).
* ``ls_problem``    -- A = U diag(s) V^T with prescribed condition number,
                       s log-spaced from 1 down to 1/cond, U the thin Q of an
                       m x n Gaussian, V the Q of an n x n Gaussian (host
                       LAPACK, used here for generation only), b = A x_true
                       + 1e-6 N(0, 1).
* ``batch_shapes``  -- many small problems: m log-uniform in [16, 512],
                       n uniform in [8, m].
* ``arrivals``      -- a Poisson request stream for the serving loop.
"""
from __future__ import annotations

import numpy as np


def _streams(seed: int, count: int):
    return [np.random.Generator(np.random.PCG64(s)) for s in np.random.SeedSequence(seed).spawn(count)]


def gaussian(m: int, n: int, seed: int = 0, dtype=np.float64) -> np.ndarray:
    """m x n, entries N(0,1), Fortran (column-major) order."""
    g = _streams(seed, 1)[0]
    return np.asfortranarray(g.standard_normal((n, m)).T.astype(dtype, copy=False))


def uniform(m: int, n: int, seed: int = 0, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    g = _streams(seed, 1)[0]
    return np.asfortranarray(g.uniform(lo, hi, size=(n, m)).T)


def singular_values(n: int, cond: float) -> np.ndarray:
    """s_i = cond^(-i/(n-1)), i = 0..n-1: sigma_max = 1, sigma_min = 1/cond."""
    if n == 1:
        return np.ones(1)
    return cond ** (-np.arange(n) / (n - 1.0))


def ls_problem(m: int, n: int, cond: float, seed: int = 0, nrhs: int = 1, noise: float = 1e-6):
    """(A, b, x_true) for min ||A x - b||, A = U diag(s) V^T."""
    gu, gv, gx, gn = _streams(seed, 4)
    U, _ = np.linalg.qr(gu.standard_normal((m, n)))
    V, _ = np.linalg.qr(gv.standard_normal((n, n)))
    s = singular_values(n, cond)
    A = np.asfortranarray((U * s[None, :]) @ V.T)
    x = gx.standard_normal((n, nrhs))
    b = np.asfortranarray(A @ x + noise * gn.standard_normal((m, nrhs)))
    return A, b, x


def batch_shapes(count: int, seed: int = 0, m_lo: int = 16, m_hi: int = 512, n_lo: int = 8):
    """``count`` (m, n) pairs: m = round(exp(U[ln m_lo, ln m_hi])), n uniform in [n_lo, m]."""
    g = _streams(seed, 1)[0]
    m = np.rint(np.exp(g.uniform(np.log(m_lo), np.log(m_hi), size=count))).astype(np.int64)
    m = np.clip(m, m_lo, m_hi)
    n = np.array([g.integers(min(n_lo, mm), mm + 1) for mm in m], dtype=np.int64)
    return list(zip(m.tolist(), n.tolist()))


def batch_matrices(shapes, seed: int = 0, dtype=np.float64):
    gs = _streams(seed, len(shapes))
    return [np.asfortranarray(g.standard_normal((n, m)).T.astype(dtype, copy=False)) for g, (m, n) in zip(gs, shapes)]


def arrivals(rate: float, count: int, seed: int = 0, m_lo: int = 256, m_hi: int = 8192,
             cond_lo: float = 1e1, cond_hi: float = 1e6, rhs_max: int = 4):
    """A Poisson stream of least-squares requests: exponential gaps of mean
    1/rate seconds; m log-uniform in [m_lo, m_hi]; n uniform in [ceil(m/8), m];
    1..rhs_max right-hand sides; cond log-uniform in [cond_lo, cond_hi].
    Returns a list of dicts with keys t, m, n, nrhs, cond, seed."""
    g = _streams(seed, 1)[0]
    gaps = g.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for r in range(count):
        m = int(np.clip(np.rint(np.exp(g.uniform(np.log(m_lo), np.log(m_hi)))), m_lo, m_hi))
        n = int(g.integers(-(-m // 8), m + 1))
        nrhs = int(g.integers(1, rhs_max + 1))
        cond = float(np.exp(g.uniform(np.log(cond_lo), np.log(cond_hi))))
        out.append({"t": float(t[r]), "m": m, "n": n, "nrhs": nrhs, "cond": cond, "seed": int(g.integers(1 << 31))})
    return out


def random_orthogonal_factor(m: int, k: int, g: np.random.Generator, reflectors: int = 4) -> np.ndarray:
    """An m x k matrix with orthonormal columns, built as a product of a few
    random Householder reflectors applied to [I; 0] -- O(m k) per reflector,
    cheap enough to build per request in a serving stream."""
    Q = np.zeros((m, k))
    Q[np.arange(k), np.arange(k)] = 1.0
    for _ in range(reflectors):
        u = g.standard_normal(m)
        u /= np.linalg.norm(u)
        Q -= 2.0 * np.outer(u, u @ Q)
    perm = g.permutation(m)
    return Q[perm]


def ls_request(m: int, n: int, nrhs: int, cond: float, seed: int, noise: float = 1e-6, reflectors: int = 4):
    """One serving request: A = U diag(s) V^T with exact singular values s,
    U = P H_r .. H_1 [I; 0] (the construction of random_orthogonal_factor)
    and V from a few reflectors as well; b = A x + noise.  The reflectors act
    directly on [diag(s) V^T; 0], so building A costs O(m n) per reflector."""
    gu, gv, gx, gn = _streams(seed, 4)
    V = random_orthogonal_factor(n, n, gv, reflectors)
    s = singular_values(n, cond)
    M = np.zeros((m, n))
    M[:n] = s[:, None] * V.T
    for _ in range(reflectors):
        u = gu.standard_normal(m)
        u /= np.linalg.norm(u)
        M -= 2.0 * np.outer(u, u @ M)
    A = np.asfortranarray(M[gu.permutation(m)])
    x = gx.standard_normal((n, nrhs))
    b = np.asfortranarray(A @ x + noise * gn.standard_normal((m, nrhs)))
    return A, b, x


def fill_normal_device(t, seed: int) -> None:
    """Fills a device tensor in place with N(0, 1) numbers from torch's
    seeded device generator (for batches too large to draw on the host)."""
    import torch
    g = torch.Generator(device=t.device)
    g.manual_seed(seed)
    t.normal_(generator=g)
