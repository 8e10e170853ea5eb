"""Pins of the series oracle: the counter-based generator against the
published splitmix64 sequence, the sampler's support, the ln Z coefficient
normalisation against first- and second-order perturbation theory of the
single-site SU(N) model (closed forms), and Pade approximants against closed
forms."""
from math import comb, factorial

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import g0, series


def test_splitmix64_published_sequence():
    # splitmix64 from state 0: the first three outputs of the reference generator
    assert [series.mix64(0, i) for i in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_sampler_support():
    sites, tau = series.sample(200, 5, 7, 3.5, 12345, first=10)
    assert np.all(sites[0::5] == 0) and np.all(tau[0::5] == 0.0)
    free = np.ones(1000, bool)
    free[0::5] = False
    assert sites.min() >= 0 and sites.max() < 7 and tau[free].min() >= 0.0 and tau[free].max() < 3.5
    # roughly uniform sites (chi-square with 48 degrees of freedom, generous bound)
    idx = sites[free, 0] + 7 * sites[free, 1]
    cnt = np.bincount(idx, minlength=49)
    e = idx.size / 49
    assert np.sum((cnt - e) ** 2 / e) < 120


@pytest.mark.parametrize("N", [2, 3, 4])
def test_first_order_is_minus_interaction_energy(oracle_mod, N):
    """f_1 per site and unit time = -<U sum_{s<s'} n_s n_s'>_0 = -U C(N,2) n^2
    (first-order perturbation theory of ln Z), with n the free density."""
    L, t, beta, mu, U = 3, 1.0, 2.0, 0.3, 1.7
    G, _ = g0.build_g0(L, t, beta, [mu], [0.0], np.zeros((1, 2), int), np.zeros(1))
    S = oracle_mod.dp(G[0], N, 0)
    dens = g0.density(L, t, beta, mu, 0.0)
    assert abs(series.prefactor(1, U, L, beta) * S - (-U * comb(N, 2) * dens ** 2)) < 1e-13


@pytest.mark.parametrize("N", [2, 3])
def test_second_order_single_site(oracle_mod, N):
    """One site (L = 1): ln Z(xi) = ln sum_k C(N,k) exp(-beta (e k + xi U k(k-1)/2)),
    so f_2 = (beta U)^2 / 2 Var(k(k-1)/2) under k ~ Binomial(N, nF(e)); per unit
    time it must equal prefactor(2) * E_tau[S(0, tau)] = (U^2/8) int_0^beta S dtau."""
    L, t, beta, mu, U = 1, 0.5, 1.5, 0.2, 1.0
    e = -4 * t - mu
    p = 1.0 / (np.exp(beta * e) + 1.0)
    k = np.arange(N + 1)
    w = np.array([comb(N, j) * p ** j * (1 - p) ** (N - j) for j in k])
    x = k * (k - 1) / 2
    exact = (beta * U) ** 2 / 2 * (np.sum(w * x * x) - np.sum(w * x) ** 2) / beta

    def S(tt):
        G, _ = g0.build_g0(L, t, beta, [mu], [0.0], np.zeros((2, 2), int), np.array([0.0, tt]))
        return oracle_mod.dp(G[0], N, 0)
    integral = quad(S, 0.0, beta, epsabs=1e-13, epsrel=1e-12, limit=200)[0]
    got = series.prefactor(2, U, L, beta) * integral / beta
    assert abs(got - exact) <= 1e-9 * abs(exact), (got, exact)


def test_pade_closed_forms():
    ex = [1.0 / factorial(i) for i in range(12)]
    assert abs(series.pade(ex, 1, 1, 1.0) - 3.0) < 1e-14            # (1 + x/2) / (1 - x/2)
    assert abs(series.pade(ex, 2, 2, 1.0) - 19.0 / 7.0) < 1e-13     # (1 + x/2 + x^2/12) / (1 - x/2 + x^2/12)
    # a rational function is reproduced by the approximant of its degrees
    xs = 0.7
    P, Q = np.array([1.0, 2.0, -0.5]), np.array([1.0, -0.4, 0.3])
    a = np.zeros(9)
    # Taylor coefficients of P/Q by long division
    for i in range(9):
        a[i] = (P[i] if i < 3 else 0.0) - sum(Q[j] * a[i - j] for j in range(1, 3) if i - j >= 0)
    assert abs(series.pade(a, 2, 2, xs) - np.polyval(P[::-1], xs) / np.polyval(Q[::-1], xs)) < 1e-12
    # [m/0] is the partial sum
    assert abs(series.pade(a, 4, 0, xs) - np.polyval(a[:5][::-1], xs)) < 1e-14


def test_pade_band_is_linear_in_errors():
    a = np.array([1.0, -0.8, 0.5, -0.35, 0.2, -0.1, 0.06])
    da = np.array([0.0, 1e-3, 2e-3, 3e-3, 5e-3, 8e-3, 1e-2])
    lo1, hi1, v1, d1 = series.band(a, da, [1, 2, 3])
    lo2, hi2, v2, d2 = series.band(a, 2 * da, [1, 2, 3])
    assert np.allclose(v1, v2) and np.allclose(2 * np.array(d1), d2, rtol=1e-6)
    assert lo1 <= min(v1) and hi1 >= max(v1)
