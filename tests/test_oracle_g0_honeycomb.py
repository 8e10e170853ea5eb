"""Pins of the honeycomb free propagator oracle: the atomic limit (t = 0) in
closed form, one unit cell (L = 1) by direct matrix exponentials, half filling
at mu = alpha and Delta = 0 (particle-hole symmetry: density 1/2 per site),
anti-periodicity in imaginary time, and the equal-time jump."""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle import g0_honeycomb as GH


def _scalar(xi, d, beta):
    if d > 0:
        return -np.exp(-xi * d) * (1.0 - 1.0 / (np.exp(beta * xi) + 1.0))
    return np.exp(-xi * d) / (np.exp(beta * xi) + 1.0)


def test_atomic_limit():
    beta, mu, alpha, delta = 3.0, 0.4, 0.1, 0.25
    cells = np.array([[0, 0], [0, 0], [2, 1]])
    tau = np.array([1.3, 0.2, 0.7])
    G = GH.build_g0(4, 0.0, beta, [mu], [alpha], [delta], cells, tau)[0]
    xi = {0: delta - (mu - alpha), 1: -delta - (mu - alpha)}
    for a in range(3):
        for b in range(3):
            for p in range(2):
                for q in range(2):
                    want = _scalar(xi[p], tau[a] - tau[b], beta) if (p == q and a in (0, 1) and b in (0, 1)) else 0.0
                    if a == b and p == q:
                        want = _scalar(xi[p], 0.0, beta)
                    assert abs(G[2 * a + p, 2 * b + q] - want) < 1e-14, (a, b, p, q)


@pytest.mark.parametrize("d", [0.7, 0.0, -1.1])
def test_single_cell_matrix_exponential(d):
    """L = 1: one k-point, eps = -3t; G(tau) = -expm(-H tau)(1 - nF(H)) or expm(-H tau) nF(H)."""
    t, beta, mu, alpha, delta = 1.0, 2.5, 0.3, -0.2, 0.15
    H = np.array([[delta - (mu - alpha), -3 * t], [-3 * t, -delta - (mu - alpha)]])
    nF = np.linalg.inv(np.eye(2) + expm(beta * H))
    want = -expm(-H * d) @ (np.eye(2) - nF) if d > 0 else expm(-H * d) @ nF
    G = GH.build_g0(1, t, beta, [mu], [alpha], [delta], np.array([[0, 0], [0, 0]]), np.array([d, 0.0]))[0]
    assert np.allclose(G[0:2, 2:4], want, rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("L", [3, 6])
def test_half_filling_density(L):
    G = GH.build_g0(L, 1.0, 4.0, [0.37], [0.37], [0.0], np.array([[1, 2]]), np.array([0.5]))[0]
    assert abs(G[0, 0] - 0.5) < 1e-13 and abs(G[1, 1] - 0.5) < 1e-13


def test_antiperiodic():
    L, t, beta = 4, 1.0, 3.0
    cells = np.array([[0, 0], [1, 3]])
    a = GH.build_g0(L, t, beta, [0.2], [0.0], [0.1], cells, np.array([2.1, 0.4]))[0]   # tau = 1.7
    b = GH.build_g0(L, t, beta, [0.2], [0.0], [0.1], cells, np.array([2.1 - beta, 0.4]))[0]   # tau = 1.7 - beta
    assert np.allclose(a[0:2, 2:4], -b[0:2, 2:4], rtol=1e-12, atol=1e-15)


def test_equal_time_jump():
    """G(0+) - G(0-) = -{c, c^+}: minus the identity between a site and
    itself, zero between different sites (same cell other sublattice, other
    cells)."""
    L, t, beta, h = 5, 1.0, 2.0, 1e-7
    cells = np.array([[2, 2], [2, 2], [3, 2], [2, 3], [1, 2], [3, 3]])
    tau0 = np.zeros(6)
    tauh = tau0.copy()
    tauh[0] = h
    Gm = GH.build_g0(L, t, beta, [0.0], [0.0], [0.0], cells, tau0)[0]
    Gp = GH.build_g0(L, t, beta, [0.0], [0.0], [0.0], cells, tauh)[0]
    jump = Gp[0:2, :] - Gm[0:2, :]   # row: vertex 0 at 0+ (or 0-)
    want = np.zeros((2, 12))
    want[:, 2:4] = -np.eye(2)        # vertex 1: same cell
    assert np.allclose(jump, want, atol=1e-6)


def test_derivative_against_central_differences():
    """dG/dxi = -dG/dmu: central differences of the propagator in mu
    (including the equal-time pairs and both signs of the time difference)."""
    rng = np.random.default_rng(31)
    n, L, beta = 4, 6, 3.0
    cells = rng.integers(0, L, size=(n, 2))
    tau = rng.uniform(0, beta, size=n)
    tau[2] = tau[1]
    mu, alpha, delta = np.array([0.3, -0.2]), np.array([0.1, 0.0]), np.array([0.25, -0.25])
    dG = GH.build_dg0(L, 1.0, beta, mu, alpha, delta, cells, tau)
    h = 1e-5
    Gp = GH.build_g0(L, 1.0, beta, mu + h, alpha, delta, cells, tau)
    Gm = GH.build_g0(L, 1.0, beta, mu - h, alpha, delta, cells, tau)
    fd = -(Gp - Gm) / (2 * h)
    assert np.max(np.abs(dG - fd)) <= 1e-8 * max(1.0, np.max(np.abs(fd))), np.max(np.abs(dG - fd))


def test_mu_gradient_of_labelled_sum_against_central_differences(oracle_mod):
    """The chain the GPU test compares with, -sum dS/dG * dG/dxi, against
    central differences of the labelled sum in mu_f (n = 3, two flavours)."""
    from oracle import sublattice as SL
    rng = np.random.default_rng(32)
    n, L, beta = 3, 5, 2.0
    cells = rng.integers(0, L, size=(n, 2))
    tau = rng.uniform(0, beta, size=n)
    mu, alpha, delta = np.array([0.3, -0.1]), np.array([0.05, -0.05]), np.array([0.2, -0.2])
    G = GH.build_g0(L, 1.0, beta, mu, alpha, delta, cells, tau)
    dG = GH.build_dg0(L, 1.0, beta, mu, alpha, delta, cells, tau)
    _, g = SL.by_assignment_adjoint(G, 2, 1)
    h = 1e-5
    for f in range(2):
        e = np.zeros(2)
        e[f] = h
        Sp = SL.by_assignment(GH.build_g0(L, 1.0, beta, mu + e, alpha, delta, cells, tau), 2, 1)
        Sm = SL.by_assignment(GH.build_g0(L, 1.0, beta, mu - e, alpha, delta, cells, tau), 2, 1)
        fd = (Sp - Sm) / (2 * h)
        assert abs(-np.sum(g[f] * dG[f]) - fd) <= 1e-7 * max(1.0, abs(fd)), (f, -np.sum(g[f] * dG[f]), fd)
