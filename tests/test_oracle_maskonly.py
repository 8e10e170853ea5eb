"""Pins of the mask-only oracle (Alg. 1's DP on points, non-physical clows
kept): enumeration of permutation pairs, the vertex-level DP of the two-flavour
sum (a different algorithm), the labelled Alg. 1 enumeration, the exact CDet
value, and a closed form that only holds if the non-physical clows cancel."""
from math import factorial

import numpy as np
import pytest

from oracle import cdet
from oracle import maskonly as MO
from oracle import sublattice as SL


def test_one_interaction():
    """n = 1: one cycle in each block, S = (w a_up)(w a_dn)."""
    assert MO.alg1([[0.7]], [[-1.3]]) == pytest.approx(0.7 * -1.3, rel=1e-15)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_unlabelled_equals_enumeration(n):
    rng = np.random.default_rng(40 + n)
    Au, Ad = rng.normal(size=(2, n, n))
    assert MO.alg1(Au, Ad) == pytest.approx(MO.brute_unlabelled(Au, Ad), rel=1e-12, abs=1e-13)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_non_physical_clows_are_kept(n):
    """The non-physical clows cancel only through the sign of a cycle (w = -1,
    each block a determinant).  With w = +1 (a permanent) they do not, so the
    DP must then differ from the enumeration of cycle covers: a DP that
    dropped them would agree for every w."""
    rng = np.random.default_rng(45 + n)
    Au, Ad = np.abs(rng.normal(size=(2, n, n))) + 0.1
    assert abs(MO.alg1(Au, Ad, w=1.0) - MO.brute_unlabelled(Au, Ad, 1.0)) > 1e-3 * MO.brute_unlabelled(Au, Ad, 1.0)


@pytest.mark.parametrize("n", [5, 6, 7])
def test_unlabelled_equals_vertex_dp(oracle_mod, n):
    """The vertex-level DP of the two-flavour sum counts every SU(2) diagram
    2^n times (which point of each vertex is up)."""
    rng = np.random.default_rng(50 + n)
    G = rng.normal(size=(2, n, n)) * 0.8
    ref = oracle_mod.dp(G, 2, 1, None, -1.0, "ld") / 2 ** n
    sabs = oracle_mod.dp(np.abs(G), 2, 1, None, 1.0, "ld") / 2 ** n
    assert abs(MO.alg1(G[0], G[1]) - ref) <= 1e-13 * sabs


@pytest.mark.parametrize("n", [1, 2, 3])
def test_labelled_equals_alg1_enumeration(n):
    rng = np.random.default_rng(60 + n)
    A = rng.normal(size=(2, 2 * n, 2 * n)) * 0.7
    assert MO.alg1(A[0], A[1], labelled=True) == pytest.approx(SL.alg1_brute(A[0], A[1]), rel=1e-12, abs=1e-13)


@pytest.mark.parametrize("n", [4, 5])
def test_labelled_equals_exact_cdet(n):
    rng = np.random.default_rng(70 + n)
    A = rng.normal(size=(2, 2 * n, 2 * n)) * 0.6
    ex = float(cdet.cdet_alg1(A[0], A[1]))
    sabs = SL.by_assignment(np.abs(A), 2, 1, 1.0) / 2 ** n
    assert abs(MO.alg1(A[0], A[1], labelled=True) - ex) <= 1e-13 * sabs


@pytest.mark.parametrize("n", [3, 4, 5, 6])
def test_diagonal_down_block_counts_hamiltonian_cycles(n):
    """Down block diagonal (d_k), up block all ones: the down points are
    self-loops, so the up block alone must connect every interaction with one
    n-cycle: S = (-d_1) ... (-d_n) * (-(n - 1)!).  The DP reaches this only after
    its non-physical clows (points visited twice) cancel."""
    d = np.linspace(0.5, 1.5, n)
    got = MO.alg1(np.ones((n, n)), np.diag(d))
    assert got == pytest.approx((-1) ** (n + 1) * np.prod(d) * factorial(n - 1), rel=1e-12)
