"""Connected-determinant (CDet) comparison path -- TEST INFRASTRUCTURE ONLY.

For the SU(2) bipartite model (Alg. 1's quantity) the full sum over a labelled
vertex set T (each vertex absent, on A or on B; Methods, 3^n principal minors)
is a product of two principal minors,

    a(T) = det A_up[T] * det A_dn[T],

and the connected part follows the recursion of the Methods section,

    c(T) = a(T) - sum_{T' subset T, T' holds the lowest vertex of T, T' != T} c(T') a(T \\ T'),

(labels inherited from T); the result is the sum of c over the 2^n full
labellings.  Here every minor is an exact rational determinant of the
float64 inputs (fractions.Fraction, Bareiss elimination) and the recursion is
exact: this is the reference the floating-point CDet kernels are measured
against (Methods, numerical instabilities of CDet).

Codes: a labelled subset is a base-3 number, digit k = 0 (absent), 1 (A),
2 (B); rows / columns of A are 2k + s.
"""
from __future__ import annotations

from fractions import Fraction
from itertools import product

import numpy as np


def _det_exact(M):
    """Exact determinant of a square list-of-Fractions matrix (Bareiss)."""
    n = len(M)
    if n == 0:
        return Fraction(1)
    A = [row[:] for row in M]
    sign = 1
    prev = Fraction(1)
    for k in range(n - 1):
        if A[k][k] == 0:
            sw = next((r for r in range(k + 1, n) if A[r][k] != 0), None)
            if sw is None:
                return Fraction(0)
            A[k], A[sw] = A[sw], A[k]
            sign = -sign
        for i in range(k + 1, n):
            for j in range(k + 1, n):
                A[i][j] = (A[i][j] * A[k][k] - A[i][k] * A[k][j]) / prev
        prev = A[k][k]
    return sign * A[n - 1][n - 1]


def digits(code: int, n: int):
    out = []
    for _ in range(n):
        out.append(code % 3)
        code //= 3
    return out


def minors(A, n: int):
    """Exact principal minors det A[T] for all 3^n labelled subsets T."""
    F = [[Fraction(float(x)) for x in row] for row in np.asarray(A, dtype=np.float64)]
    out = []
    for code in range(3 ** n):
        d = digits(code, n)
        idx = [2 * k + (d[k] - 1) for k in range(n) if d[k]]
        out.append(_det_exact([[F[i][j] for j in idx] for i in idx]))
    return out


def connected(a, n: int):
    """c(T) for every code T from a(T) by the subset recursion."""
    p3 = [3 ** k for k in range(n + 1)]
    c = [Fraction(0)] * (3 ** n)
    for code in range(1, 3 ** n):
        d = digits(code, n)
        present = [k for k in range(n) if d[k]]
        low, rest = present[0], present[1:]
        s = a[code]
        # proper labelled subsets that keep the lowest vertex
        for keep in product((0, 1), repeat=len(rest)):
            if all(keep):
                continue
            sub = d[low] * p3[low] + sum(d[k] * p3[k] for k, kk in zip(rest, keep) if kk)
            s -= c[sub] * a[code - sub]
        c[code] = s
    return c


def cdet_alg1(A_up, A_dn) -> Fraction:
    """Sum over the 2^n full labellings of the connected part of det A_up det A_dn."""
    A_up = np.asarray(A_up, dtype=np.float64)
    n = A_up.shape[-1] // 2
    mu, md = minors(A_up, n), minors(A_dn, n)
    a = [x * y for x, y in zip(mu, md)]
    c = connected(a, n)
    p3 = [3 ** k for k in range(n)]
    return sum(c[sum((1 + s[k]) * p3[k] for k in range(n))] for s in product((0, 1), repeat=n))
