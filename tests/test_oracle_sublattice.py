"""Pins of the sublattice-summed oracle (bipartite lattices): the sum over
label assignments (oracle) against an independent enumeration of labelled
permutations, a closed form for label-factorised propagators, the label-swap
symmetry, diagram counts, and the labelled state space."""
import itertools

import numpy as np
import pytest

from oracle import sublattice as SL


def _rand(rng, n, nmat):
    return rng.normal(size=(nmat, 2 * n, 2 * n)) * 0.7


@pytest.mark.parametrize("n", [1, 2, 3])
@pytest.mark.parametrize("nf,variant", [(2, 0), (3, 0), (2, 1)])
def test_assignment_sum_equals_labelled_enumeration(oracle_mod, n, nf, variant):
    rng = np.random.default_rng(100 * n + 10 * nf + variant)
    A = _rand(rng, n, 1 if variant == 0 else nf)
    A = A[0] if variant == 0 else A
    got = SL.by_assignment(A, nf, variant)
    ref = SL.brute_labeled(A, nf, variant)
    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (got, ref)


@pytest.mark.parametrize("n", [2, 4, 6])
def test_label_factorised_closed_form(oracle_mod, n):
    """A[(k,s),(j,t)] = x_s y_t G[k][j]: every vertex has two points, each with
    one outgoing and one incoming edge, so an assignment scales the sum by
    prod_k (x_{s_k} y_{s_k})^2 and the total is S(G) (sum_s (x_s y_s)^2)^n."""
    rng = np.random.default_rng(7 + n)
    G = rng.normal(size=(n, n)) * 0.6
    x, y = rng.normal(size=2), rng.normal(size=2)
    A = np.einsum("s,t,kj->ksjt", x, y, G).reshape(2 * n, 2 * n)
    got = SL.by_assignment(A, 3, 0)
    ref = oracle_mod.dp(G, 3, 0) * (np.sum((x * y) ** 2)) ** n
    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)) * 4 ** n


@pytest.mark.parametrize("n", [3, 5])
def test_label_swap_symmetry(oracle_mod, n):
    rng = np.random.default_rng(40 + n)
    A = _rand(rng, n, 2)
    perm = np.array([2 * k + 1 - s for k in range(n) for s in (0, 1)])
    a = SL.by_assignment(A, 2, 1)
    b = SL.by_assignment(A[:, perm][:, :, perm], 2, 1)
    assert abs(a - b) <= 1e-12 * max(1.0, abs(a))


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_counts(oracle_mod, n):
    """All propagators 1: every assignment gives the counting sequence c_n(w N)."""
    from oracle import counts
    got = SL.by_assignment(np.ones((2 * n, 2 * n)), 1, 0, 1.0)
    assert got == 2 ** n * counts.connected_counts(n, 1)[n]


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_state_space(n):
    c = SL.plan_counts(n)
    assert c["masks"] == 3 * 4 ** (n - 1)
    assert c["closes"] == c["states"]
    # each state of level l < 2n extends to one child per (open vertex, admissible label)
    assert c["ext"] > c["states"] or n == 1


@pytest.mark.parametrize("n", [1, 2, 3])
def test_alg1_is_two_flavour_sum_over_2n(oracle_mod, n):
    """Alg. 1 (SU(2), one up and one down point per vertex, cycles inside a
    block) equals the two-flavour sum divided by 2^n: in the flavour sum a
    vertex with both points in one flavour cancels (equal rows), and each
    vertex with one point per flavour appears twice (which point is up)."""
    rng = np.random.default_rng(900 + n)
    A = _rand(rng, n, 2)
    got = SL.alg1_brute(A[0], A[1])
    ref = SL.by_assignment(A, 2, 1) / 2 ** n
    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (got, ref)


@pytest.mark.parametrize("n,nf,variant", [(2, 2, 0), (3, 2, 1), (3, 3, 0)])
def test_assignment_adjoint_against_central_differences(oracle_mod, n, nf, variant):
    """dS/dA of the labelled sum: S is a polynomial of degree at most 2 in
    each entry (both points of a vertex can carry the same matrix entry), so a
    central difference is exact up to rounding."""
    rng = np.random.default_rng(90 + 10 * n + variant)
    A = rng.normal(size=(2 * n, 2 * n)) if variant == 0 else rng.normal(size=(nf, 2 * n, 2 * n))
    S, g = SL.by_assignment_adjoint(A, nf, variant)
    assert S == pytest.approx(SL.by_assignment(A, nf, variant), rel=1e-13, abs=1e-14)
    h = 1e-5
    for idx in np.ndindex(A.shape):
        P, M = A.copy(), A.copy()
        P[idx] += h
        M[idx] -= h
        fd = (SL.by_assignment(P, nf, variant) - SL.by_assignment(M, nf, variant)) / (2 * h)
        assert abs(g[idx] - fd) <= 1e-7 * max(1.0, abs(fd)), (idx, g[idx], fd)
