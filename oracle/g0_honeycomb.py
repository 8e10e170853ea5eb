"""Free propagator of the honeycomb-lattice model -- TEST INFRASTRUCTURE ONLY.

Methods, honeycomb lattice: per flavour s the Bloch Hamiltonian on an L x L
grid of unit cells is the 2 x 2 matrix

    H_s(k) = [[ Delta_s - (mu_s - alpha_s),  eps(k)                      ],
              [ conj(eps(k)),                -Delta_s - (mu_s - alpha_s)  ]]

with eps(k) = -t (1 + exp(i k.b1) + exp(i k.b2)), k.b_i = 2 pi m_i / L
(sublattice A of cell R hops to sublattice B of cells R, R + b1, R + b2).
Convention G0 = -<T c c^+>, as for the square lattice:

    0 < tau < beta :  G(k, tau) = -exp(-H tau) (1 - nF(H))
    -beta < tau <= 0 : G(k, tau) =  exp(-H tau) nF(H)          (tau = 0 read as 0^-)

(matrix functions of H(k)), and in real space, between vertex a (cell R_a,
sublattice p) and vertex b (cell R_b, sublattice q):

    G[2a + p, 2b + q] = (1/L^2) sum_k exp(i k.(R_a - R_b)) G_pq(k, tau_a - tau_b).

Plain numpy: eigen-decomposition of each H(k) (``numpy.linalg.eigh``), the
Fermi factors written without cancellation, a direct sum over k.
"""
from __future__ import annotations

import numpy as np


def _fermi_parts(E, beta):
    """(nF(E), 1 - nF(E)) without overflow or cancellation."""
    nF = np.where(E >= 0, np.exp(-beta * np.abs(E)) / (1.0 + np.exp(-beta * np.abs(E))),
                  1.0 / (1.0 + np.exp(-beta * np.abs(E))))
    hF = np.where(E >= 0, 1.0 / (1.0 + np.exp(-beta * np.abs(E))),
                  np.exp(-beta * np.abs(E)) / (1.0 + np.exp(-beta * np.abs(E))))
    return nF, hF


def _branch(E, d, beta):
    """Scalar factor of one eigenvalue for a time difference d."""
    nF, hF = _fermi_parts(E, beta)
    if d > 0:
        # -exp(-E d)(1 - nF): for E < 0 use exp(E (beta - d)) nF(-E)-style form
        return -np.where(E >= 0, np.exp(-E * d) * hF, np.exp(E * (beta - d)) / (1.0 + np.exp(beta * E)))
    s = -d
    return np.where(E <= 0, np.exp(E * s) * nF, np.exp(-E * (beta - s)) / (1.0 + np.exp(-beta * E)))


def bloch(L, t, mu, alpha, delta):
    """H(k) for every k of the L x L grid: array (L, L, 2, 2) complex."""
    m = np.arange(L)
    k1, k2 = np.meshgrid(2 * np.pi * m / L, 2 * np.pi * m / L, indexing="ij")
    eps = -t * (1.0 + np.exp(1j * k1) + np.exp(1j * k2))
    H = np.zeros((L, L, 2, 2), dtype=np.complex128)
    H[..., 0, 0] = delta - (mu - alpha)
    H[..., 1, 1] = -delta - (mu - alpha)
    H[..., 0, 1] = eps
    H[..., 1, 0] = np.conj(eps)
    return H, k1, k2


def build_g0(L, t, beta, mu, alpha, delta, cells, tau):
    """Returns G of shape (nflav, 2n, 2n), index 2k + s (s = 0 for A, 1 for B).

    cells: int array (n, 2) of unit-cell coordinates; tau: (n,); mu, alpha,
    delta: per-flavour arrays."""
    mu = np.atleast_1d(np.asarray(mu, dtype=np.float64))
    alpha = np.atleast_1d(np.asarray(alpha, dtype=np.float64))
    delta = np.atleast_1d(np.asarray(delta, dtype=np.float64))
    cells = np.asarray(cells)
    tau = np.asarray(tau, dtype=np.float64)
    n = tau.size
    G = np.zeros((mu.size, 2 * n, 2 * n))
    for f in range(mu.size):
        H, k1, k2 = bloch(L, t, mu[f], alpha[f], delta[f])
        E, V = np.linalg.eigh(H)                      # (L, L, 2), (L, L, 2, 2)
        for a in range(n):
            for b in range(n):
                d = tau[a] - tau[b]
                r1 = cells[a, 0] - cells[b, 0]
                r2 = cells[a, 1] - cells[b, 1]
                fE = _branch(E, d, beta)              # (L, L, 2)
                Gk = np.einsum("xyim,xym,xyjm->xyij", V, fE, np.conj(V))
                ph = np.exp(1j * (k1 * r1 + k2 * r2))
                g = np.einsum("xy,xyij->ij", ph, Gk) / (L * L)
                assert np.max(np.abs(g.imag)) < 1e-12 * max(1.0, np.max(np.abs(g.real)))
                G[f, 2 * a:2 * a + 2, 2 * b:2 * b + 2] = g.real
    return G


def build_dg0(L, t, beta, mu, alpha, delta, cells, tau):
    """dG/dxi for a uniform move H -> H + xi of every H(k) (xi = -(mu -
    alpha)), same shape as :func:`build_g0`.  The eigenvectors do not move, so
    each eigenvalue's factor f(E) is replaced by its derivative: for a time
    difference d > 0, f(E) = -exp(-E d)(1 - nF(E)) and f'(E) = f(E)(beta
    nF(E) - d); for d <= 0, f(E) = exp(-E d) nF(E) and f'(E) = f(E)(beta nF(E)
    - beta - d)."""
    mu = np.atleast_1d(np.asarray(mu, dtype=np.float64))
    alpha = np.atleast_1d(np.asarray(alpha, dtype=np.float64))
    delta = np.atleast_1d(np.asarray(delta, dtype=np.float64))
    cells = np.asarray(cells)
    tau = np.asarray(tau, dtype=np.float64)
    n = tau.size
    dG = np.zeros((mu.size, 2 * n, 2 * n))
    for f in range(mu.size):
        H, k1, k2 = bloch(L, t, mu[f], alpha[f], delta[f])
        E, V = np.linalg.eigh(H)
        nF, _ = _fermi_parts(E, beta)
        for a in range(n):
            for b in range(n):
                d = tau[a] - tau[b]
                fE = _branch(E, d, beta)
                dfE = fE * (beta * nF - d) if d > 0 else fE * (beta * nF - beta - d)
                Gk = np.einsum("xyim,xym,xyjm->xyij", V, dfE, np.conj(V))
                ph = np.exp(1j * ((cells[a, 0] - cells[b, 0]) * k1 + (cells[a, 1] - cells[b, 1]) * k2))
                g = np.einsum("xy,xyij->ij", ph, Gk) / (L * L)
                dG[f, 2 * a:2 * a + 2, 2 * b:2 * b + 2] = g.real
    return dG
