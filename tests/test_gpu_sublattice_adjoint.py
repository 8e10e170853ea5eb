"""Reverse sweep of the sublattice-summed sums on the GPU (COS_F_SUBLATTICE,
also in mask-only mode) against the oracle's gradient: for each label
assignment the vertex-level reverse sweep of the matrix it picks, added back
into the entries it came from.

Tolerance per entry: 8 n (n + 2) eps times the same gradient over absolute
values (|A|, |w|)."""
import numpy as np
import pytest

from gpu_util import announce

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def _run(mats, nflav, variant, mask_only=False, tune=False, w=-1.0):
    """mats: list of (nmat, 2n, 2n) -> (S forward, S adjoint, dS/dA list)."""
    import torch
    from paper_2507_12349_amd import _binding as B
    n = np.array([m.shape[-1] // 2 for m in mats], dtype=np.int32)
    sizes = np.array([m.size for m in mats], dtype=np.int64)
    off = np.zeros(len(mats), dtype=np.int64)
    off[1:] = np.cumsum(sizes[:-1])
    dev = torch.device("cuda:0")
    G = torch.as_tensor(np.concatenate([m.reshape(-1) for m in mats]), device=dev)
    Goff = torch.as_tensor(off, device=dev)
    b = B.Batch(n, nflav, variant, sublattice=True, mask_only=mask_only)
    try:
        out = torch.full((len(mats),), float("nan"), dtype=torch.float64, device=dev)
        ob = torch.ones(len(mats), dtype=torch.float64, device=dev)
        Gb = torch.full_like(G, float("nan"))
        if tune:
            b.autotune(G, Goff, None, w, out, ob, Gb, None)
        b.forward(G, Goff, None, w, out)
        torch.cuda.synchronize()
        S = out.cpu().numpy()
        out2 = torch.full_like(out, float("nan"))
        Gb.fill_(float("nan"))
        b.adjoint(G, Goff, None, w, ob, out2, Gb, None)
        torch.cuda.synchronize()
        gb = Gb.cpu().numpy()
        return S, out2.cpu().numpy(), [gb[off[i]:off[i] + mats[i].size].reshape(mats[i].shape)
                                       for i in range(len(mats))]
    finally:
        b.close()


def _check(Gb, A, nf, variant, scale=1.0):
    from oracle import sublattice as SL
    n = A.shape[-1] // 2
    M = A[0] if variant == 0 else A
    _, g = SL.by_assignment_adjoint(M, nf, variant)
    _, gabs = SL.by_assignment_adjoint(np.abs(M), nf, variant, 1.0)
    g, gabs = g * scale, gabs * scale
    got = Gb[0] if variant == 0 else Gb
    err = np.abs(got - g)
    assert np.all(err <= 8 * n * (n + 2) * EPS * gabs + 1e-300), np.max(err / np.maximum(gabs, 1e-300))


@pytest.mark.parametrize("nf,variant", [(2, 0), (3, 1)])
def test_random_batch(oracle_mod, nf, variant):
    """Orders 1..6 (matrices and the dS/dG accumulator both in LDS) plus a
    ragged group of 66 configurations of order 4."""
    announce("sublattice reverse sweep nf=%d variant=%d" % (nf, variant))
    rng = np.random.default_rng(700 + 10 * nf + variant)
    nmat = 1 if variant == 0 else nf
    orders = [1, 2, 3, 5, 6] + [4] * 66
    mats = [rng.normal(size=(nmat, 2 * k, 2 * k)) * 0.5 for k in orders]
    S, S2, Gb = _run(mats, nf, variant)
    assert np.array_equal(S, S2)
    for i in (0, 1, 2, 3, 4, 5, 37, 70):
        _check(Gb[i], mats[i], nf, variant)


@pytest.mark.parametrize("n", [7, 8])
def test_high_orders(oracle_mod, n):
    """Orders 7 and 8 (G read from global memory, accumulator in LDS), two
    flavour matrices, 65 configurations, autotuned; the ragged tail (and at
    n = 7 the first) checked: the oracle takes seconds per configuration."""
    announce("sublattice reverse sweep n=%d" % n)
    rng = np.random.default_rng(720 + n)
    mats = [rng.normal(size=(2, 2 * n, 2 * n)) * 0.4 for _ in range(65)]
    S, S2, Gb = _run(mats, 2, 1, tune=True)
    assert np.array_equal(S, S2)
    for i in ((0, 64) if n == 7 else (64,)):
        _check(Gb[i], mats[i], 2, 1)


@pytest.mark.parametrize("orders", [[1, 2, 3, 4, 5], [8, 8]])
def test_mask_only(oracle_mod, orders):
    """Alg. 1 with labels: the gradient is 2^-n times the two-flavour labelled
    gradient (the identity of the sums, pinned on the CPU)."""
    announce("mask-only labelled reverse sweep, orders %s" % orders)
    rng = np.random.default_rng(740 + len(orders))
    mats = [rng.normal(size=(2, 2 * k, 2 * k)) * 0.5 for k in orders]
    S, S2, Gb = _run(mats, 2, 1, mask_only=True)
    assert np.array_equal(S, S2)
    for i, k in enumerate(orders):
        if k < 8 or i == 0:
            _check(Gb[i], mats[i], 2, 1, scale=2.0 ** -k)


def test_mask_only_against_finite_differences_of_its_oracle():
    """n = 2 with labels: central differences of the mask-only oracle itself."""
    from oracle import maskonly as MO
    announce("mask-only labelled reverse sweep vs finite differences")
    rng = np.random.default_rng(750)
    A = rng.normal(size=(2, 4, 4))
    _, _, Gb = _run([A], 2, 1, mask_only=True)
    h = 1e-5
    for idx in np.ndindex(A.shape):
        P, M = A.copy(), A.copy()
        P[idx] += h
        M[idx] -= h
        fd = (MO.alg1(P[0], P[1], True) - MO.alg1(M[0], M[1], True)) / (2 * h)
        assert abs(Gb[0][idx] - fd) <= 1e-8 * max(1.0, abs(fd)), (idx, Gb[0][idx], fd)
