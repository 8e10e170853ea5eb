"""Diagram counts from the exponential formula -- TEST INFRASTRUCTURE ONLY.

With every propagator equal to 1, the full sum over all diagrams on n
vertices (2n points) with weight x per closed cycle is the rising factorial
x (x+1) ... (x+2n-1) (the cycle-index generating function of the symmetric
group).  Diagrams split uniquely into connected components on vertex
subsets and the weight factorises, so with A(z) = sum a_n z^n / n! and
C(z) = sum c_n z^n / n!, A = exp(C); c_n is read off C = log A.  Exact
integer arithmetic (Python ints / Fractions).
"""
from __future__ import annotations

from fractions import Fraction
from math import comb


def full_counts(nmax, x):
    """a_n = x (x+1) ... (x+2n-1) for n = 0..nmax (x integer)."""
    out = []
    for n in range(nmax + 1):
        a = 1
        for j in range(2 * n):
            a *= x + j
        out.append(a)
    return out


def connected_counts(nmax, x):
    """c_n for n = 1..nmax (index 0 unused = 0), via a_n = sum_k C(n-1,k-1) c_k a_{n-k}
    (split off the component that holds vertex 1)."""
    a = full_counts(nmax, x)
    c = [0] * (nmax + 1)
    for n in range(1, nmax + 1):
        s = a[n]
        for k in range(1, n):
            s -= comb(n - 1, k - 1) * c[k] * a[n - k]
        c[n] = s
    return c


def connected_counts_log(nmax, x):
    """The same sequence from C = log A by power-series logarithm (an
    independent route used to cross-check ``connected_counts``)."""
    from math import factorial
    a = [Fraction(v, factorial(i)) for i, v in enumerate(full_counts(nmax, x))]
    # log(1 + B) with B = A - 1: C' = A'/A  ->  n C_n = n a_n - sum_{k<n} k C_k a_{n-k}
    C = [Fraction(0)] * (nmax + 1)
    for n in range(1, nmax + 1):
        s = n * a[n]
        for k in range(1, n):
            s -= k * C[k] * a[n - k]
        C[n] = s / n
    return [int(C[n] * factorial(n)) if n else 0 for n in range(nmax + 1)]
