"""Operation counts for reporting rates (Buttari et al., Sec. 2.1 and 3.2).

* ``standard(m, n)``  -- 2 n^2 (m - n/3), the Householder QR count of Sec. 2.1
  (the paper's "relative performance" basis).
* ``tiled(m, n, b, ib)`` -- the flops the tiled method itself performs with
  inner blocks of ib columns: per task kind, the counts of Sec. 3.2 refined for
  inner blocking (SSRFB 4 b^3 + ib b^2, the paper's 5 b^3 at ib = b).
* ``bj_formula(m, n)`` -- (4 m n^2 - 4 n^3 / 3), twice the standard count.
"""
from __future__ import annotations


def standard(m: int, n: int) -> float:
    return 2.0 * n * n * (m - n / 3.0)


def bj_formula(m: int, n: int) -> float:
    return 4.0 * m * n * n - 4.0 * n ** 3 / 3.0


def kernel_flops(kind: str, b: int, ib: int) -> float:
    """Flops of one task at tile size b with inner block ib, exploiting the
    zero/unit structure of V and the triangular T."""
    nb = b // ib
    if kind == "SSRFB":
        return nb * (4.0 * ib * b * b + ib * ib * b)
    if kind == "LARFB":
        return sum(2 * (2.0 * (b - s * ib) * ib - ib * ib) * b + ib * ib * b for s in range(nb))
    if kind == "TSQRT":
        tot = 0.0
        for s in range(nb):
            rest = b - (s + 1) * ib
            tot += sum(4.0 * (b + 1) * (ib - 1 - j) + 3.0 * b for j in range(ib))
            tot += sum(2.0 * b * j + j * j for j in range(ib))
            tot += (4.0 * ib * b + ib * ib + 2 * ib) * rest
        return tot
    if kind == "GEQRT":
        tot = 0.0
        for s in range(nb):
            h = b - s * ib
            rest = b - (s + 1) * ib
            tot += sum(4.0 * (h - j) * (ib - 1 - j) + 3.0 * (h - j) for j in range(ib))
            tot += sum(2.0 * (h - j) * j + j * j for j in range(ib))
            tot += (2 * (2.0 * h * ib - ib * ib) + ib * ib) * rest
        return tot
    raise ValueError(kind)


def task_counts(p: int, q: int) -> dict:
    K = min(p, q)
    return {
        "GEQRT": K,
        "LARFB": sum(q - 1 - k for k in range(K)),
        "TSQRT": sum(p - 1 - k for k in range(K)),
        "SSRFB": sum((p - 1 - k) * (q - 1 - k) for k in range(K)),
    }


def tiled(m: int, n: int, b: int, ib: int) -> float:
    p, q = -(-m // b), -(-n // b)
    c = task_counts(p, q)
    return sum(kernel_flops(k, b, ib) * c[k] for k in c)
