"""O2: determinant closed form plus the connected-part recursion -- TEST
INFRASTRUCTURE ONLY.

Full sum over all (connected or not) diagrams on a vertex set S, for cycle
weight -1.  A sum over permutations of the points of one flavour with a
factor -1 per cycle equals (-1)^size * det (the determinant as a sum over
cycle covers with sign (-1)^(size - #cycles), Results, "Theoretical
Constructions").  Points of the same vertex share a row of G, so a flavour
class that holds both points of a vertex has a repeated row and vanishes;
hence each vertex k carries either an unordered pair of distinct flavours
(two orderings, same determinant) or, with shifts, one flavour on one point
and a shift head of that flavour on the other (two choices, weight -sigma).
The signs cancel and

    a(S) = 2^|S| * sum_F  prod_{k: F_k = {l}} sigma_l  *  prod_l det G_l[S_l],

S_l = {k in S : l in F_k}; for two flavours without shifts this is the
two-flavour determinant product of the Methods section.  Connected parts
follow from the recursion of the Methods section,

    c(V) = a(V) - sum_{v0 in S, S strict subset of V} c(S) a(V \\ S),

with a(empty) = 1.  Everything runs in exact rational arithmetic
(``fractions.Fraction``; float64 inputs are exact rationals), so the result
is exact up to the final rounding.  Only practical for small n.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def det_exact(M):
    """Exact determinant of a square matrix of Fractions (Gaussian elimination)."""
    A = [list(r) for r in M]
    m = len(A)
    if m == 0:
        return Fraction(1)
    det = Fraction(1)
    for c in range(m):
        piv = next((r for r in range(c, m) if A[r][c] != 0), None)
        if piv is None:
            return Fraction(0)
        if piv != c:
            A[c], A[piv] = A[piv], A[c]
            det = -det
        p = A[c][c]
        det *= p
        for r in range(c + 1, m):
            if A[r][c] != 0:
                fac = A[r][c] / p
                for k in range(c, m):
                    A[r][k] -= fac * A[c][k]
    return det


def _as_fractions(G, nf, variant):
    G = np.asarray(G, dtype=np.float64)
    mats = [G] * nf if variant == 0 else [G[l] for l in range(nf)]
    return [[[Fraction(float(x)) for x in row] for row in M] for M in mats]


def full_sums(G, nf, variant=0, stub=None):
    """a(S) for every vertex subset S (dict bitmask -> Fraction), weight -1."""
    mats = _as_fractions(G, nf, variant)
    n = len(mats[0])
    if stub is None:
        sig = None
    else:
        s = np.asarray(stub, dtype=np.float64).reshape(-1)
        sig = [Fraction(float(s[0]))] * nf if variant == 0 else [Fraction(float(x)) for x in s]
    options = [("pair", (a, b)) for a in range(nf) for b in range(a + 1, nf)]
    if sig is not None:
        options += [("stub", (l,)) for l in range(nf)]
    out = {0: Fraction(1)}
    det_cache = {}

    def det_sub(l, idx):
        key = (l, idx)
        if key not in det_cache:
            det_cache[key] = det_exact([[mats[l][i][j] for j in idx] for i in idx])
        return det_cache[key]

    for bits in range(1, 1 << n):
        verts = [k for k in range(n) if (bits >> k) & 1]
        total = Fraction(0)
        for choice in itertools.product(options, repeat=len(verts)):
            weight = Fraction(1)
            classes = [[] for _ in range(nf)]
            for k, (kind, fl) in zip(verts, choice):
                for l in fl:
                    classes[l].append(k)
                if kind == "stub":
                    weight *= sig[fl[0]]
            if weight == 0:
                continue
            for l in range(nf):
                weight *= det_sub(l, tuple(classes[l]))
                if weight == 0:
                    break
            total += weight
        out[bits] = Fraction(2) ** len(verts) * total
    return out


def connected_sums(G, nf, variant=0, stub=None):
    """c(S) for every subset S containing vertex 0, from the recursion."""
    a = full_sums(G, nf, variant, stub)
    n = (np.asarray(G).shape[-1])
    c = {}
    for bits in sorted(range(1, 1 << n), key=lambda b: bin(b).count("1")):
        if not bits & 1:
            continue
        val = a[bits]
        sub = (bits - 1) & bits
        while sub:
            if sub & 1 and sub != bits:
                val -= c[sub] * a[bits & ~sub]
            sub = (sub - 1) & bits
        c[bits] = val
    return a, c


def closed_form(G, nf, variant=0, stub=None):
    """Connected sum over all n vertices (cycle weight -1), as a float."""
    n = np.asarray(G).shape[-1]
    _, c = connected_sums(G, nf, variant, stub)
    return float(c[(1 << n) - 1])
