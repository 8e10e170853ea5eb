"""Pins of the exact CDet reference: one vertex in closed form, exact minors
against floating-point determinants, and the connected recursion against the
Alg. 1 enumeration and against the two-flavour labelled DP over 2^n."""
import numpy as np
import pytest

from oracle import cdet
from oracle import sublattice as SL


def test_one_vertex():
    rng = np.random.default_rng(1)
    A, B = rng.normal(size=(2, 2)), rng.normal(size=(2, 2))
    assert float(cdet.cdet_alg1(A, B)) == pytest.approx(A[0, 0] * B[0, 0] + A[1, 1] * B[1, 1], rel=1e-15)


def test_minors_against_float_determinants():
    rng = np.random.default_rng(2)
    n = 4
    A = rng.normal(size=(2 * n, 2 * n))
    m = cdet.minors(A, n)
    for code in range(3 ** n):
        d = cdet.digits(code, n)
        idx = [2 * k + d[k] - 1 for k in range(n) if d[k]]
        ref = np.linalg.det(A[np.ix_(idx, idx)]) if idx else 1.0
        assert abs(float(m[code]) - ref) <= 1e-12 * max(1.0, abs(ref))


@pytest.mark.parametrize("n", [1, 2, 3])
def test_equals_alg1_enumeration(n):
    rng = np.random.default_rng(10 + n)
    A = rng.normal(size=(2, 2 * n, 2 * n)) * 0.7
    assert float(cdet.cdet_alg1(A[0], A[1])) == pytest.approx(SL.alg1_brute(A[0], A[1]), rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("n", [4, 5])
def test_equals_labelled_dp(oracle_mod, n):
    rng = np.random.default_rng(20 + n)
    A = rng.normal(size=(2, 2 * n, 2 * n)) * 0.6
    got = float(cdet.cdet_alg1(A[0], A[1]))
    ref = SL.by_assignment(A, 2, 1) / 2 ** n
    sabs = SL.by_assignment(np.abs(A), 2, 1, 1.0) / 2 ** n
    assert abs(got - ref) <= 1e-13 * sabs, (got, ref)
