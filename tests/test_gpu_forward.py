"""GPU parity of the forward sum against the CPU oracle (through the C ABI).

Tolerance: the sum is a multilinear form of degree 2n in the entries of G;
with FP64 round-to-nearest every term passes through at most 2n steps, each an
inner product of length <= n, so |S_gpu - S_exact| <= 8 n (n + 2) eps S_abs,
S_abs being the same sum over absolute values.  The reference is the oracle's
vertex-level DP in long double (its own error is negligible at that scale).
Where that bound is tighter than 1e-10 relative, 1e-10 relative is required.
"""
import numpy as np
import pytest

from gpu_util import announce, gpu_forward, oracle_args, scale

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def _case(rng, n, nf, variant, stubs):
    nmat = 1 if variant == 0 else nf
    M = rng.normal(size=(nmat, n, n))
    st = rng.normal(size=(1 if variant == 0 else nf)) if stubs else None
    return M, st


@pytest.mark.parametrize("nf,variant,stubs", [(1, 0, False), (2, 0, False), (4, 0, False), (3, 0, True),
                                              (2, 1, False), (3, 1, False), (3, 1, True), (6, 1, True)])
def test_random_uneven_batch(oracle_mod, nf, variant, stubs):
    """One batch with every order 1..8 (uneven), random normal matrices."""
    announce("random batch nf=%d variant=%d stubs=%d" % (nf, variant, stubs))
    rng = np.random.default_rng(1000 + 10 * nf + 2 * variant + stubs)
    orders = [1, 2, 3, 4, 5, 6, 7, 8, 3, 5]
    if variant == 1 and nf >= 6:
        orders = [1, 2, 3, 4, 5, 6]
    cases = [_case(rng, n, nf, variant, stubs) for n in orders]
    mats = [c[0] for c in cases]
    sts = None if not stubs else np.stack([c[1] for c in cases])
    S = gpu_forward(mats, nf, variant, sts)
    for i, (M, st) in enumerate(cases):
        n = M.shape[-1]
        ref = oracle_mod.dp(oracle_args(M, variant), nf, variant, st)
        sa = scale(oracle_mod, M, nf, variant, st)
        assert abs(S[i] - ref) <= 8 * n * (n + 2) * EPS * sa, (i, n, S[i], ref)


def test_single_flavour_is_zero(oracle_mod):
    """N = 1 without shifts: Pauli zero at every order."""
    announce("pauli zero")
    rng = np.random.default_rng(7)
    mats = [rng.normal(size=(1, n, n)) for n in range(1, 9)]
    S = gpu_forward(mats, 1, 0)
    for i, M in enumerate(mats):
        n = M.shape[-1]
        assert abs(S[i]) <= 8 * n * (n + 2) * EPS * scale(oracle_mod, M, 1, 0, None)


def test_zero_shifts_equal_no_shifts():
    announce("zero shifts")
    rng = np.random.default_rng(8)
    mats = [rng.normal(size=(3, n, n)) for n in (2, 4, 6)]
    a = gpu_forward(mats, 3, 1, None)
    b = gpu_forward(mats, 3, 1, np.zeros((3, 3)))
    assert np.array_equal(a, b)


def test_uniform_equals_flavour_with_equal_matrices():
    announce("U == F with equal G")
    rng = np.random.default_rng(9)
    mats = [rng.normal(size=(1, n, n)) for n in (3, 5, 7)]
    a = gpu_forward(mats, 3, 0, None)
    b = gpu_forward([np.repeat(M, 3, axis=0) for M in mats], 3, 1, None)
    assert np.allclose(a, b, rtol=1e-13, atol=0)


@pytest.mark.parametrize("x,nf,w", [(1, 1, 1.0), (-2, 2, -1.0), (-4, 4, -1.0), (-6, 6, -1.0)])
def test_diagram_counts(x, nf, w):
    """Unit propagators: the connected sum counts diagrams weighted by (w N)^cycles;
    exact in FP64 while the counts stay below 2^53 (stored values: exponential
    formula, tests/golden/connected_counts.json)."""
    import json
    import os
    announce("counts x=%d" % x)
    seq = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "connected_counts.json")))
    seq = [int(v) for v in seq["sequences"][str(x)]]
    ns = [n for n in range(1, 13) if abs(seq[n - 1]) < 2 ** 53 and n <= 10]
    S = gpu_forward([np.ones((1, n, n)) for n in ns], nf, 0, None, w=w)
    for n, s in zip(ns, S):
        assert s == float(seq[n - 1]), (n, s, seq[n - 1])


def test_max_flavours_small_order(oracle_mod):
    """COS_FMAX = 16 flavours (16 waves per workgroup)."""
    announce("16 flavours")
    rng = np.random.default_rng(11)
    mats = [rng.normal(size=(16, n, n)) for n in (1, 2, 3)]
    st = rng.normal(size=(3, 16))
    S = gpu_forward(mats, 16, 1, st)
    for i, M in enumerate(mats):
        ref = oracle_mod.dp(M, 16, 1, st[i])
        n = M.shape[-1]
        assert abs(S[i] - ref) <= 8 * n * (n + 2) * EPS * scale(oracle_mod, M, 16, 1, st[i])


def test_max_order(oracle_mod):
    """n = COS_NMAX = 12, uniform SU(2), one configuration."""
    announce("n=12")
    rng = np.random.default_rng(12)
    M = rng.normal(size=(1, 12, 12)) * 0.5
    S = gpu_forward([M], 2, 0, None)
    ref = oracle_mod.dp(M[0], 2, 0)
    sa = scale(oracle_mod, M, 2, 0, None)
    assert abs(S[0] - ref) <= 8 * 12 * 14 * EPS * sa
