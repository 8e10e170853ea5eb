"""Monte Carlo driver on the GPU: the device sampler against the oracle's
generator (bit for bit), the moment sums, and the ln Z coefficients against
first-order perturbation theory, the single-site second-order closed form and
the oracle evaluated on the very same sampled configurations."""
from math import comb

import numpy as np
import pytest

from gpu_util import announce

pytestmark = pytest.mark.gpu


def test_sampler_matches_oracle():
    import torch
    from oracle import series
    from paper_2507_12349_amd import _binding as B
    announce("mc sampler vs oracle generator")
    nconf, n, L, beta, seed, first = 300, 6, 8, 4.0, 987654321, 12345
    sites = torch.empty((nconf * n, 2), dtype=torch.int32, device="cuda:0")
    tau = torch.empty(nconf * n, dtype=torch.float64, device="cuda:0")
    B.mc_sample(nconf, n, L, beta, seed, first, sites, tau)
    torch.cuda.synchronize()
    s_ref, t_ref = series.sample(nconf, n, L, beta, seed, first)
    assert np.array_equal(sites.cpu().numpy(), s_ref)
    assert np.array_equal(tau.cpu().numpy(), t_ref)


def test_moments():
    import torch
    from paper_2507_12349_amd import _binding as B
    announce("moment sums")
    x = np.random.default_rng(3).normal(size=5000)
    acc = torch.zeros(2, dtype=torch.float64, device="cuda:0")
    xd = torch.as_tensor(x, device="cuda:0")
    B.accumulate_moments(x.size, xd, acc)
    B.accumulate_moments(x.size, xd, acc)
    torch.cuda.synchronize()
    a = acc.cpu().numpy()
    assert abs(a[0] - 2 * x.sum()) < 1e-11 and abs(a[1] - 2 * (x * x).sum()) < 1e-10


def test_first_order_coefficient():
    from oracle import g0
    from paper_2507_12349_amd import mc
    announce("mc: first order = -U C(N,2) n^2")
    L, t, beta, mu, U, N = 8, 1.0, 4.0, -0.5, 2.0, 4
    c = mc.lnz_coefficient(1, L=L, t=t, beta=beta, mu=[mu], alpha=[0.0], nflav=N, variant=0, U=U, nconf=64,
                           nbatches=2, seed=1)
    exact = -U * comb(N, 2) * g0.density(L, t, beta, mu, 0.0) ** 2
    assert abs(c.value - exact) < 1e-13 and c.error < 1e-15


def test_second_order_single_site():
    """L = 1: the exact second-order coefficient of the single-site model.  On
    one site S(0, tau) does not depend on tau (G(tau) G(-tau) = -n(1-n)), so
    every sample equals the integral and the estimate is exact to rounding."""
    from paper_2507_12349_amd import mc
    announce("mc: second order, single site")
    L, t, beta, mu, U, N = 1, 0.5, 1.5, 0.2, 1.0, 3
    c = mc.lnz_coefficient(2, L=L, t=t, beta=beta, mu=[mu], alpha=[0.0], nflav=N, variant=0, U=U, nconf=8192,
                           nbatches=8, seed=7)
    e = -4 * t - mu
    p = 1.0 / (np.exp(beta * e) + 1.0)
    k = np.arange(N + 1)
    w = np.array([comb(N, j) * p ** j * (1 - p) ** (N - j) for j in k])
    x = k * (k - 1) / 2
    exact = (beta * U) ** 2 / 2 * (np.sum(w * x * x) - np.sum(w * x) ** 2) / beta
    assert abs(c.value - exact) <= 1e-12 * abs(exact) + 5 * c.error, (c.value, exact, c.error)
    assert c.error <= 1e-12 * abs(exact)


def test_third_order_equals_oracle_on_same_samples(oracle_mod):
    """The driver's estimate equals the oracle's connected sums and propagators
    evaluated on the configurations the oracle's generator draws (same seed)."""
    from oracle import g0, series
    from paper_2507_12349_amd import mc
    announce("mc: third order vs oracle on the same samples")
    L, t, beta, mu, U, N, nconf, nb, seed = 3, 1.0, 2.0, 0.1, 1.5, 2, 40, 2, 99
    c = mc.lnz_coefficient(3, L=L, t=t, beta=beta, mu=[mu], alpha=[0.0], nflav=N, variant=0, U=U, nconf=nconf,
                           nbatches=nb, seed=seed)
    sites, tau = series.sample(nconf * nb, 3, L, beta, seed, 0)
    S = []
    Sabs = []
    for i in range(nconf * nb):
        G, _ = g0.build_g0(L, t, beta, [mu], [0.0], sites[3 * i:3 * i + 3], tau[3 * i:3 * i + 3])
        S.append(oracle_mod.dp(G[0], N, 0))
        Sabs.append(oracle_mod.dp(np.abs(G[0]), N, 0, None, 1.0))
    ref = series.prefactor(3, U, L, beta) * np.mean(S)
    tol = abs(series.prefactor(3, U, L, beta)) * np.mean(Sabs) * 1e-12
    assert abs(c.value - ref) <= tol, (c.value, ref)


def test_statistical_error_scaling():
    """Two independent seeds at n = 2 on a 4 x 4 lattice agree within their
    combined errors, and the error shrinks like 1/sqrt(samples)."""
    from paper_2507_12349_amd import mc
    announce("mc: error bars, n=2 on 4x4")
    kw = dict(L=4, t=1.0, beta=2.0, mu=[0.3], alpha=[0.0], nflav=2, variant=0, U=1.0, nbatches=8)
    a = mc.lnz_coefficient(2, nconf=2048, seed=11, **kw)
    b = mc.lnz_coefficient(2, nconf=2048, seed=12, **kw)
    c = mc.lnz_coefficient(2, nconf=8192, seed=13, **kw)
    assert a.error > 0 and b.error > 0
    assert abs(a.value - b.value) <= 5 * np.hypot(a.error, b.error), (a, b)
    assert 0.25 < c.error / (0.5 * (a.error + b.error)) < 0.8
