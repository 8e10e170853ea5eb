"""Free propagator of the square-lattice SU(N) model -- TEST INFRASTRUCTURE ONLY.

Methods, square-lattice dispersion: xi_s(k) = -2 t [cos kx + cos ky] - mu_s + alpha_s
on the momentum grid k = 2 pi (mx, my) / L.  Imaginary-time propagator (the
convention G0 = -<T c c^+> used throughout):

    0 < tau < beta :  G(k, tau) = -exp(-xi tau) (1 - nF(xi))
    -beta < tau <= 0 : G(k, tau) =  exp(-xi tau) nF(xi)

so an equal-time pair (tau = 0, read as 0^-) gives the density nF.  The
real-space matrix between vertices (r_k, tau_k) and (r_l, tau_l) is

    G_s[k, l] = (1/L^2) sum_k cos(k . (r_k - r_l)) G(k, tau_k - tau_l).

``dG_dxi`` is the derivative of that matrix when xi_s(k) moves by the same
amount at every k (d/dmu_s = -d/dxi, d/dalpha_s = +d/dxi).  Plain numpy,
float64, direct formulas (1 - nF evaluated as 1/(1 + exp(-beta xi)) so that
no cancellation occurs for xi < 0).
"""
from __future__ import annotations

import numpy as np


def dispersion(L, t, mu, alpha):
    m = np.arange(L)
    kx, ky = np.meshgrid(2 * np.pi * m / L, 2 * np.pi * m / L, indexing="ij")
    return -2.0 * t * (np.cos(kx) + np.cos(ky)) - mu + alpha, kx, ky


def build_g0(L, t, beta, mu, alpha, sites, tau):
    """Returns (G, dG_dxi), each of shape (nflav, n, n).

    sites: int array (n, 2) of lattice coordinates; tau: float array (n,);
    mu, alpha: per-flavour arrays (nflav,)."""
    mu = np.atleast_1d(np.asarray(mu, dtype=np.float64))
    alpha = np.atleast_1d(np.asarray(alpha, dtype=np.float64))
    nf = mu.size
    sites = np.asarray(sites)
    tau = np.asarray(tau, dtype=np.float64)
    n = tau.size
    G = np.zeros((nf, n, n))
    dG = np.zeros((nf, n, n))
    for s in range(nf):
        xi, kx, ky = dispersion(L, t, mu[s], alpha[s])
        nF = 1.0 / (np.exp(beta * xi) + 1.0)           # occupation
        hF = 1.0 / (1.0 + np.exp(-beta * xi))          # 1 - nF, written without cancellation
        for a in range(n):
            for b in range(n):
                dx = sites[a, 0] - sites[b, 0]
                dy = sites[a, 1] - sites[b, 1]
                d = tau[a] - tau[b]
                ph = np.cos(kx * dx + ky * dy)
                if d > 0:
                    gk = -np.exp(-xi * d) * hF
                    dgk = gk * (beta * nF - d)
                else:
                    gk = np.exp(-xi * d) * nF
                    dgk = gk * (beta * nF - beta - d)
                G[s, a, b] = np.sum(ph * gk) / (L * L)
                dG[s, a, b] = np.sum(ph * dgk) / (L * L)
    return G, dG


def density(L, t, beta, mu, alpha):
    """(1/L^2) sum_k nF(xi_k): the equal-time local propagator."""
    xi, _, _ = dispersion(L, t, mu, alpha)
    return float(np.mean(1.0 / (np.exp(beta * xi) + 1.0)))
