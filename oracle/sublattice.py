"""Sublattice-summed connected sums (bipartite lattices) -- TEST INFRASTRUCTURE ONLY.

On a bipartite lattice every interaction vertex k also carries a sublattice
label s_k in {A, B} (both of its points sit on the same sublattice), and the
propagator between two points depends on both labels.  The method sums the
connected diagrams over every assignment of labels in one pass, with the
four-state interaction mask {0, (1,A), (1,B), 2} (Results, "Theoretical
Constructions", bipartite paragraph; Methods, Alg. 1 and Alg. 2; Methods,
strategy (i) for bipartite lattices: a_E(W) and c_E(W) as sums over sublattice
configurations).

Argument convention: ``A`` has shape (2n, 2n) (variant U) or (nf, 2n, 2n)
(variant F); row and column index 2k + s for vertex k on sublattice s
(0 = A, 1 = B).

  :func:`by_assignment`   the definition: sum over the 2^n label assignments
                          of the connected sum of the n x n matrix they pick
                          (oracle O3 per assignment)
  :func:`by_assignment_adjoint`  the same with the O3 reverse sweep: dS/dA
  :func:`brute_labeled`   independent enumeration of labelled permutations
                          (pure Python, n <= 3)
  :func:`alg1_brute`      the SU(2) form of Alg. 1 (up and down point per
                          vertex, cycles inside a block) by enumeration
  :func:`plan_counts`     breadth-first enumeration of the labelled DP states
"""
from __future__ import annotations

import itertools

import numpy as np


def pick(A: np.ndarray, s) -> np.ndarray:
    """The n x n (per flavour) matrix of one label assignment s:
    G[k][j] = A[2k + s_k][2j + s_j]."""
    A = np.asarray(A, dtype=np.float64)
    idx = 2 * np.arange(len(s)) + np.asarray(s, dtype=np.int64)
    return A[..., idx[:, None], idx[None, :]]


def by_assignment(A, nf: int, variant: int = 0, w: float = -1.0, precision: str = "ld") -> float:
    """Connected sum summed over all sublattice assignments (strategy (i) of
    the Methods section), with the vertex-level oracle O3 for each one."""
    import oracle
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[-1] // 2
    tot = 0.0
    for s in itertools.product((0, 1), repeat=n):
        tot += oracle.dp(pick(A, s), nf, variant, None, w, precision)
    return tot


def by_assignment_adjoint(A, nf: int, variant: int = 0, w: float = -1.0):
    """(S, dS/dA) of :func:`by_assignment`: for each label assignment the
    oracle O3 reverse sweep of the matrix it picks, added back into the
    entries it was picked from."""
    import oracle
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[-1] // 2
    tot = 0.0
    grad = np.zeros_like(A)
    for s in itertools.product((0, 1), repeat=n):
        idx = 2 * np.arange(n) + np.asarray(s, dtype=np.int64)
        S, g, _ = oracle.dp_adjoint(pick(A, s), nf, variant, None, w)
        tot += S
        grad[..., idx[:, None], idx[None, :]] += g
    return tot, grad


def brute_labeled(A, nf: int, variant: int = 0, w: float = -1.0) -> float:
    """Enumeration straight from the definition, for tiny n: every labelling
    s, every permutation pi of the 2n points (vertex of point p: p mod n),
    every flavour per cycle (variant F; variant U multiplies each cycle by
    nf), kept when the cycles connect all vertices.  A cycle contributes
    w * prod_p A_l[2 v(p) + s_v(p)][2 v(pi p) + s_v(pi p)]."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[-1] // 2
    P = 2 * n
    mats = [A] if variant == 0 else [A[l] for l in range(nf)]
    total = 0.0
    for s in itertools.product((0, 1), repeat=n):
        lab = [2 * (p % n) + s[p % n] for p in range(P)]
        for pi in itertools.permutations(range(P)):
            seen = [False] * P
            cycles = []
            for p0 in range(P):
                if seen[p0]:
                    continue
                cyc = []
                p = p0
                while not seen[p]:
                    seen[p] = True
                    cyc.append(p)
                    p = pi[p]
                cycles.append(cyc)
            # connectivity over vertices (union-find on the vertices of each cycle)
            parent = list(range(n))

            def find(x):
                while parent[x] != x:
                    parent[x] = parent[parent[x]]
                    x = parent[x]
                return x
            for cyc in cycles:
                r0 = find(cyc[0] % n)
                for p in cyc[1:]:
                    parent[find(p % n)] = r0
            if len({find(k) for k in range(n)}) != 1:
                continue
            term = 1.0
            for cyc in cycles:
                csum = 0.0
                for M in mats:
                    prod = 1.0
                    for p in cyc:
                        prod *= M[lab[p], lab[pi[p]]]
                    csum += prod
                term *= w * (nf * csum if variant == 0 else csum)
            total += term
    return total


def alg1_brute(A_up, A_dn, w: float = -1.0) -> float:
    """SU(2) bipartite sum as Alg. 1 states it, by enumeration (tiny n): the 2n
    points are the up point k and the down point k + n of each vertex k; a
    cycle stays inside one block (Blk: up points go to up points); labels s_k
    are summed; a cycle contributes w * prod A_block[2 v(p) + s][2 v(pi p) + t];
    only connected diagrams count."""
    A_up = np.asarray(A_up, dtype=np.float64)
    A_dn = np.asarray(A_dn, dtype=np.float64)
    n = A_up.shape[-1] // 2
    total = 0.0
    for s in itertools.product((0, 1), repeat=n):
        lab = [2 * k + s[k] for k in range(n)]
        for pu in itertools.permutations(range(n)):
            for pd in itertools.permutations(range(n)):
                parent = list(range(n))

                def find(x):
                    while parent[x] != x:
                        parent[x] = parent[parent[x]]
                        x = parent[x]
                    return x
                term = 1.0
                for perm, M in ((pu, A_up), (pd, A_dn)):
                    seen = [False] * n
                    for k0 in range(n):
                        if seen[k0]:
                            continue
                        prod = 1.0
                        k = k0
                        while not seen[k]:
                            seen[k] = True
                            prod *= M[lab[k], lab[perm[k]]]
                            parent[find(perm[k])] = find(k)
                            k = perm[k]
                        term *= w * prod
                if len({find(k) for k in range(n)}) == 1:
                    total += term
    return total


def plan_counts(n: int) -> dict:
    """States, extension transitions, closes, masks and rows of the labelled
    vertex DP, by breadth-first enumeration from the two start states (vertex 0
    on A or on B).  A state is (mask, head, head label, current, current label);
    a mask digit is 0, (1, A), (1, B) or 2; the next head opens on the lowest
    once-visited vertex."""
    start = [(tuple([1 + s] + [0] * (n - 1)), 0, s, 0, s) for s in (0, 1)]
    level = set(start)
    states = ext = 0
    masks, rows = set(), set()
    for _ in range(2 * n):
        nxt = set()
        for (m, u, su, v, sv) in level:
            states += 1
            masks.add(m)
            rows.add((m, u, su))
            for x in range(n):
                if m[x] == 3:
                    continue
                for sx in ((0, 1) if m[x] == 0 else (m[x] - 1,)):
                    mm = list(m)
                    mm[x] = 1 + sx if m[x] == 0 else 3
                    nxt.add((tuple(mm), u, su, x, sx))
                    ext += 1
            once = [k for k in range(n) if m[k] in (1, 2)]
            if once:
                h = once[0]
                mm = list(m)
                mm[h] = 3
                nxt.add((tuple(mm), h, m[h] - 1, h, m[h] - 1))
        level = nxt
    return {"states": states, "ext": ext, "closes": states, "masks": len(masks), "rows": len(rows)}
