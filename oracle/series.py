"""Series coefficients by Monte Carlo and Pade re-summation -- TEST INFRASTRUCTURE ONLY.

The coefficient of xi^n in ln Z (Methods, shifted action: the interaction
carries xi (U/2) sum_{s,s'} n_s n_s' per site and time) is

    f_n = ((-U/2)^n / n!) * sum_{sites} int_0^beta dtau ... S(X_1, ..., X_n),

S the connected sum of the library (w = -1 per closed loop, no prefactors).
Per site and unit imaginary time, with vertex 0 fixed at (site 0, tau 0) by
translation invariance:

    f_n / (L^2 beta) = ((-U/2)^n / n!) (L^2 beta)^(n-1) E[S],

E over the other n-1 vertices drawn uniformly.  Pade re-summation follows the
Results section: symmetric approximants [m/m] of sum_i a_i xi^i at xi = 1,
each with the linear error delta^2 = sum_i (d Pade / d a_i)^2 delta_a_i^2, and
the band = min and max of value -/+ delta over the approximants.

  :func:`mix64`, :func:`sample`     the counter-based generator (splitmix64
                                    output function) and the vertex sampler
  :func:`prefactor`                 ((-U/2)^n / n!) (L^2 beta)^(n-1)
  :func:`pade`, :func:`pade_grad`   [m/k] by the defining linear system;
                                    gradient by central differences
  :func:`band`                      the re-summation band
"""
from __future__ import annotations

from math import factorial

import numpy as np

_M64 = (1 << 64) - 1


def mix64(seed: int, counter: int) -> int:
    """splitmix64 output function (Steele, Lea, Flood 2014) of
    seed + 0x9E3779B97F4A7C15 * (counter + 1), 64-bit arithmetic."""
    z = (seed + 0x9E3779B97F4A7C15 * (counter + 1)) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def sample(nconf: int, n: int, L: int, beta: float, seed: int, first: int = 0):
    """(sites (nconf*n, 2), tau (nconf*n,)): vertex 0 at site (0, 0), time 0;
    vertex k >= 1 of configuration c uses counters ((first + c) n + k) 2 + q,
    site = ((z >> 32) L^2) >> 32 as (x, y) = (site mod L, site div L), time =
    beta (z >> 11) 2^-53."""
    sites = np.zeros((nconf * n, 2), dtype=np.int32)
    tau = np.zeros(nconf * n)
    L2 = L * L
    for c in range(nconf):
        for k in range(1, n):
            ctr = ((first + c) * n + k) * 2
            zs, zt = mix64(seed, ctr), mix64(seed, ctr + 1)
            site = ((zs >> 32) * L2) >> 32
            sites[c * n + k] = (site % L, site // L)
            tau[c * n + k] = beta * ((zt >> 11) * 2.0 ** -53)
    return sites, tau


def prefactor(n: int, U: float, L: int, beta: float) -> float:
    return (-U / 2.0) ** n / factorial(n) * float(L * L * beta) ** (n - 1)


def pade(a, m: int, k: int, x: float) -> float:
    """[m/k] approximant P/Q of sum_i a_i x^i at x: Q(x) f(x) - P(x) = O(x^(m+k+1)),
    q_0 = 1 (numpy linear solve)."""
    a = np.asarray(a, dtype=np.float64)
    if k > 0:
        A = np.array([[a[m + 1 + r - j] if m + 1 + r - j >= 0 else 0.0 for j in range(1, k + 1)] for r in range(k)])
        q = np.concatenate([[1.0], np.linalg.solve(A, -a[m + 1:m + k + 1])])
    else:
        q = np.array([1.0])
    p = np.array([sum(q[j] * a[i - j] for j in range(min(i, k) + 1)) for i in range(m + 1)])
    return float(np.polyval(p[::-1], x) / np.polyval(q[::-1], x))


def pade_grad(a, m: int, k: int, x: float, h: float = 1e-6) -> np.ndarray:
    a = np.asarray(a, dtype=np.float64)
    g = np.zeros(m + k + 1)
    for i in range(m + k + 1):
        step = h * max(1.0, abs(a[i]))
        ap, am = a.copy(), a.copy()
        ap[i] += step
        am[i] -= step
        g[i] = (pade(ap, m, k, x) - pade(am, m, k, x)) / (2 * step)
    return g


def band(a, da, degrees, x: float = 1.0):
    """(low, high, values, deltas) over the symmetric approximants [m/m], m in degrees."""
    vals, dels = [], []
    for m in degrees:
        v = pade(a, m, m, x)
        g = pade_grad(a, m, m, x)
        d = float(np.sqrt(np.sum((g * np.asarray(da[:2 * m + 1])) ** 2)))
        vals.append(v)
        dels.append(d)
    lo = min(v - d for v, d in zip(vals, dels))
    hi = max(v + d for v, d in zip(vals, dels))
    return lo, hi, vals, dels
