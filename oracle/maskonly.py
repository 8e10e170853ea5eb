"""Mask-only connected sum (SU(2); non-physical clows kept) -- TEST INFRASTRUCTURE ONLY.

When a cycle carries no factor beyond its sign (SU(2): each spin block is its
own determinant), the DP may track only the interaction masks (Results,
"Theoretical Constructions", the variant without cycle factors; Methods,
Alg. 1): the state is (head point, current point, mask), a point is one end
of an interaction line, and

  * extend: from the current point v to any point w of v's spin block except
    the head, provided w's interaction has not been visited twice (so a point
    may be visited twice: such non-physical clows cancel among themselves);
  * close: multiply by w * a(v, head); the next cycle opens on the lowest
    interaction visited once, at either of its two ends except the current
    head (no head is repeated); with no such interaction the cycle cannot
    close, so only connected diagrams are generated;
  * the sum is over the states after 2n - 1 steps, closed once more.

The non-physical clows cancel through the sign of a cycle only, so the
method needs w = -1 (each spin block a determinant); ``w`` stays a parameter
so that tests can show that the clows are really kept.

Points: interaction k joins the up point k and the down point k + n; a spin
block holds the points of one spin.  With sublattice labels (bipartite
lattices) every point also carries a label: a point of an unvisited
interaction is reached with either label, a point of an interaction visited
once keeps the label recorded in the mask, and the label is forgotten once the
interaction is visited twice (four mask states 0, (1, A), (1, B), 2).

This is a separate algorithm from the vertex-level DP of ``oracle.dp``: it
works on points, keeps non-physical clows and does not canonicalise heads.

Argument convention: ``A_up``, ``A_dn`` are n x n (unlabelled) or 2n x 2n
with index 2k + s (labelled, s = 0 for A, 1 for B).
"""
from __future__ import annotations

import numpy as np

_TWICE = -1


def alg1(A_up, A_dn, labelled: bool = False, w: float = -1.0, count_states: bool = False):
    """The mask-only connected sum by the DP of Alg. 1 (pure Python, dict of
    states per level).  Returns the sum, or (sum, number of states) with
    ``count_states``."""
    blocks = (np.asarray(A_up, dtype=np.float64), np.asarray(A_dn, dtype=np.float64))
    side = blocks[0].shape[-1]
    n = side // 2 if labelled else side
    labels = (0, 1) if labelled else (0,)

    def a(v, sv, x, sx):
        """Propagator from point v (label sv) to point x (label sx), same block."""
        b, i, j = v // n, v % n, x % n
        if labelled:
            return blocks[b][2 * i + sv, 2 * j + sx]
        return blocks[b][i, j]

    def visit(mu, k, s):
        m = list(mu)
        m[k] = (1 + s) if m[k] == 0 else _TWICE
        return tuple(m)

    # start: the up point of interaction 0, each label
    V = {}
    for s in labels:
        V[((0, s), (0, s), visit((0,) * n, 0, s))] = 1.0
    nstates = len(V)
    for _ in range(2 * n - 1):
        nxt = {}
        for ((u, su), (v, sv), mu), om in V.items():
            blk = v // n
            # extend within v's block, never onto the head, never onto an
            # interaction visited twice
            for x in range(blk * n, blk * n + n):
                k = x % n
                if x == u or mu[k] == _TWICE:
                    continue
                for sx in (labels if mu[k] == 0 else (mu[k] - 1,)):
                    key = ((u, su), (x, sx), visit(mu, k, sx))
                    nxt[key] = nxt.get(key, 0.0) + om * a(v, sv, x, sx)
            # close, then open on the lowest interaction visited once
            once = [k for k in range(n) if mu[k] not in (0, _TWICE)]
            if once:
                k = once[0]
                sk = mu[k] - 1
                val = w * om * a(v, sv, u, su)
                for h in (k, k + n):
                    if h == u:
                        continue
                    key = ((h, sk), (h, sk), visit(mu, k, sk))
                    nxt[key] = nxt.get(key, 0.0) + val
        V = nxt
        nstates += len(V)
    total = 0.0
    for ((u, su), (v, sv), mu), om in V.items():
        total += om * w * a(v, sv, u, su)
    return (total, nstates) if count_states else total


def brute_unlabelled(A_up, A_dn, w: float = -1.0) -> float:
    """Definition for tiny n: every pair of permutations (up block, down
    block), w per cycle times the product of its propagators, kept when the
    cycles connect all interactions (interaction k holds up point k and down
    point k)."""
    import itertools
    A_up = np.asarray(A_up, dtype=np.float64)
    A_dn = np.asarray(A_dn, dtype=np.float64)
    n = A_up.shape[0]
    total = 0.0
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
                        prod *= M[k, perm[k]]
                        parent[find(perm[k])] = find(k)
                        k = perm[k]
                    term *= w * prod
            if len({find(k) for k in range(n)}) == 1:
                total += term
    return total


def plan_counts(n: int, labelled: bool = False) -> dict:
    """Reachable states of the DP of :func:`alg1`, by breadth-first search from
    its start states: number of states, extension transitions, and states
    that close a cycle (a once-visited interaction exists, or the mask is
    full)."""
    labels = (0, 1) if labelled else (0,)

    def visit(mu, k, s):
        m = list(mu)
        m[k] = (1 + s) if m[k] == 0 else _TWICE
        return tuple(m)

    level = {((0, s), (0, s), visit((0,) * n, 0, s)) for s in labels}
    states = ext = closes = 0
    for step in range(2 * n):
        nxt = set()
        for (u, su), (v, sv), mu in level:
            states += 1
            once = [k for k in range(n) if mu[k] not in (0, _TWICE)]
            if once or step == 2 * n - 1:
                closes += 1
            if step == 2 * n - 1:
                continue
            blk = v // n
            for x in range(blk * n, blk * n + n):
                k = x % n
                if x == u or mu[k] == _TWICE:
                    continue
                for sx in (labels if mu[k] == 0 else (mu[k] - 1,)):
                    nxt.add(((u, su), (x, sx), visit(mu, k, sx)))
                    ext += 1
            if once:
                k = once[0]
                sk = mu[k] - 1
                for h in (k, k + n):
                    if h != u:
                        nxt.add(((h, sk), (h, sk), visit(mu, k, sk)))
        level = nxt
    return {"states": states, "ext": ext, "closes": closes}
