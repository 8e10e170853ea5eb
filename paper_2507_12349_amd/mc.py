"""Monte Carlo series of ln Z and Pade re-summation around the batched kernel.

The coefficient of xi^n in ln Z per site and unit imaginary time (Methods,
shifted action with xi (U/2) sum_{s,s'} n_s n_s'; the connected sum S carries
no prefactors) is

    a_n = ((-U/2)^n / n!) (L^2 beta)^(n-1) E[S],

with vertex 0 fixed at the origin (translation invariance) and the other n-1
vertices uniform over sites and [0, beta).  Every step runs on the device
through the library: sampling (counter-based generator), propagators, the
batched connected sum and the moment sums; the host only loops over batches
and divides.  Errors are the spread of independent batch means.  Pade
re-summation follows the Results section: symmetric approximants [m/m] at
xi = 1 with the linear error propagation of the coefficient errors, the band
being the extremes of value -/+ error over the approximants.
"""
from __future__ import annotations

from dataclasses import dataclass
from math import factorial

import numpy as np

from . import _binding as B


@dataclass
class Coefficient:
    n: int
    value: float          # a_n
    error: float          # standard error from the batch means
    samples: int
    batch_means: np.ndarray


def prefactor(n: int, U: float, L: int, beta: float) -> float:
    return (-U / 2.0) ** n / factorial(n) * float(L * L * beta) ** (n - 1)


def lnz_coefficient(n: int, *, L: int, t: float, beta: float, mu, alpha, nflav: int, variant: int, U: float,
                    nconf: int, nbatches: int, seed: int, stream=None) -> Coefficient:
    """Estimate a_n on the square lattice (device sampling, G0, connected sum)."""
    import torch
    if nbatches < 2:
        raise ValueError("need at least two batches for an error estimate")
    dev = torch.device("cuda")
    nmat = nflav if variant == B.FLAVOUR else 1
    mu = np.asarray(mu, dtype=np.float64).reshape(-1)[:nmat]
    alpha = np.asarray(alpha, dtype=np.float64).reshape(-1)[:nmat]
    sites = torch.empty((nconf * n, 2), dtype=torch.int32, device=dev)
    tau = torch.empty(nconf * n, dtype=torch.float64, device=dev)
    nvec = torch.full((nconf,), n, dtype=torch.int32, device=dev)
    voff = torch.arange(nconf, dtype=torch.int64, device=dev) * n
    Goff = torch.arange(nconf, dtype=torch.int64, device=dev) * (nmat * n * n)
    G = torch.empty(nconf * nmat * n * n, dtype=torch.float64, device=dev)
    S = torch.empty(nconf, dtype=torch.float64, device=dev)
    acc = torch.zeros((nbatches, 2), dtype=torch.float64, device=dev)
    b = B.Batch([n] * nconf, nflav, variant)
    try:
        for k in range(nbatches):
            B.mc_sample(nconf, n, L, beta, seed, k * nconf, sites, tau, stream)
            B.build_g0(nconf, nvec, voff, sites, tau, L, t, beta, mu, alpha, Goff, G, None, stream)
            b.forward(G, Goff, None, -1.0, S, stream)
            B.accumulate_moments(nconf, S, acc[k], stream)
        torch.cuda.synchronize()
    finally:
        b.close()
    m = acc.cpu().numpy()
    means = m[:, 0] / nconf
    pf = prefactor(n, U, L, beta)
    val = pf * float(np.mean(means))
    err = abs(pf) * float(np.std(means, ddof=1)) / np.sqrt(nbatches)
    return Coefficient(n, val, err, nconf * nbatches, pf * means)


def pade_band(a, da, degrees, x: float = 1.0):
    """(low, high, values, errors) over the symmetric approximants [m/m]."""
    a = np.asarray(a, dtype=np.float64)
    da = np.asarray(da, dtype=np.float64)
    vals, errs = [], []
    for m in degrees:
        v, g = B.pade(a[:2 * m + 1], m, m, x)
        vals.append(v)
        errs.append(float(np.sqrt(np.sum((g * da[:2 * m + 1]) ** 2))))
    lo = min(v - e for v, e in zip(vals, errs))
    hi = max(v + e for v, e in zip(vals, errs))
    return lo, hi, vals, errs
