"""Seeded synthetic vertex configurations (inputs only, no method arithmetic).

Stand-ins for the Monte Carlo samples of the paper's 32x32-lattice runs
(Results, honeycomb SU(2) and square-lattice SU(3) studies): vertex sites are
drawn uniformly over the L x L periodic lattice (with replacement) and
imaginary times uniformly in [0, beta) (honeycomb: a site is a unit cell,
its sublattice is summed over by the method).  The workloads below are the
shapes the library is tested and measured on.  Both the GPU path and the CPU
oracle take their inputs from here; neither builds propagators here.

RNG: ``numpy.random.Generator(PCG64(seed))``; draw order: (shift workload
only) the per-flavour shifts once, then per configuration (uneven workload
only) n, then n site indices in [0, L^2), then n times.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

UNIFORM, FLAVOUR = 0, 1


@dataclass(frozen=True)
class Workload:
    name: str
    L: int
    t: float
    beta: float
    nflav: int
    variant: int                 # UNIFORM (one G, cycle factor -N) or FLAVOUR (G per flavour)
    mu: tuple                    # per flavour chemical potential
    n: int                       # order (number of vertices); 0 = drawn per config
    nconf: int
    seed: int
    stubs: bool = False          # SB-CoS shift heads present
    n_range: tuple = ()          # (lo, hi) inclusive when n is drawn
    shift_range: tuple = ()      # (lo, hi) for per-flavour shifts delta
    U: float = 1.0               # interaction strength: stub weight = delta / U
    note: str = field(default="", compare=False)
    lattice: str = "square"      # "honeycomb": sites are unit cells, the sublattice is summed
    stagger: tuple = ()          # honeycomb: per-flavour staggered field Delta


WORKLOADS = {
    "plain_single": Workload("plain_single", L=4, t=1.0, beta=2.0, nflav=2, variant=UNIFORM,
                             mu=(0.0, 0.0), n=4, nconf=1, seed=1,
                             note="4x4 lattice, beta=2, mu=0, SU(2) uniform, n=4, one config"),
    "plain_batch": Workload("plain_batch", L=8, t=1.0, beta=4.0, nflav=4, variant=UNIFORM,
                            mu=(-0.5,) * 4, n=8, nconf=4096, seed=2,
                            note="8x8, beta=4, mu=-0.5, SU(4) uniform, n=8, 4096 configs"),
    "sym_broken": Workload("sym_broken", L=8, t=1.0, beta=4.0, nflav=3, variant=FLAVOUR,
                           mu=(-0.3, 0.0, 0.4), n=10, nconf=1024, seed=3,
                           note="8x8, beta=4, SU(3), mu_s=(-0.3,0,0.4), n=10, 1024 configs"),
    "uneven": Workload("uneven", L=16, t=1.0, beta=5.0, nflav=6, variant=FLAVOUR,
                       mu=(0.0,) * 6, n=0, nconf=8192, seed=4, stubs=True,
                       n_range=(6, 12), shift_range=(-0.2, 0.2), U=1.0,
                       note="16x16, beta=5, SU(6), shifts U[-0.2,0.2], n~U{6..12}, 8192 configs"),
    "honeycomb": Workload("honeycomb", L=16, t=1.0, beta=5.0, nflav=2, variant=FLAVOUR,
                          mu=(0.3, 0.3), n=8, nconf=1024, seed=6, lattice="honeycomb", stagger=(0.3, -0.3),
                          note="16x16 honeycomb cells, beta=5, SU(2) with staggered field +-0.3 per spin, "
                               "mu=0.3, n=8, 1024 configs, sublattice labels summed"),
    "adjoint": Workload("adjoint", L=8, t=1.0, beta=4.0, nflav=4, variant=UNIFORM,
                        mu=(-0.5,) * 4, n=10, nconf=2048, seed=5, stubs=True,
                        note="8x8, beta=4, SU(4) uniform, mu=-0.5, n=10, 2048 configs, "
                             "shift derivative at delta=0"),
}


@dataclass
class Draw:
    workload: Workload
    n: np.ndarray          # int32 [nconf]
    voff: np.ndarray       # int64 [nconf] offset of each config's first vertex
    sites: np.ndarray      # int32 [sum n, 2] lattice coordinates (x, y)
    tau: np.ndarray        # float64 [sum n]
    delta: np.ndarray      # float64 [nflav] per-flavour shift (zeros if none)

    def config(self, c):
        """(sites, tau) of configuration c."""
        a, b = int(self.voff[c]), int(self.voff[c]) + int(self.n[c])
        return self.sites[a:b], self.tau[a:b]

    def prefix(self, orders):
        """A draw of len(orders) configurations: configuration c keeps the
        first orders[c] vertices of this draw's configuration c (small orders
        on the same lattice and distribution, for references that grow fast
        with n)."""
        parts = [self.config(c) for c in range(len(orders))]
        n = np.asarray(orders, dtype=np.int32)
        voff = np.zeros(n.size, dtype=np.int64)
        voff[1:] = np.cumsum(n[:-1])
        sites = np.concatenate([p[0][:k] for p, k in zip(parts, orders)]).astype(np.int32)
        tau = np.concatenate([p[1][:k] for p, k in zip(parts, orders)])
        return Draw(self.workload, n, voff, sites, tau, self.delta)


def draw(name: str, nconf: int | None = None) -> Draw:
    """Draw the first ``nconf`` configurations of a workload (all by default).
    A prefix of the draw is identical to the full draw's first configs."""
    w = WORKLOADS[name]
    nconf = w.nconf if nconf is None else int(nconf)
    rng = np.random.Generator(np.random.PCG64(w.seed))
    if w.shift_range:
        delta = rng.uniform(w.shift_range[0], w.shift_range[1], size=w.nflav)
    else:
        delta = np.zeros(w.nflav)
    ns, sites, taus = [], [], []
    for _ in range(nconf):
        n = int(rng.integers(w.n_range[0], w.n_range[1] + 1)) if w.n == 0 else w.n
        idx = rng.integers(0, w.L * w.L, size=n)
        tau = rng.uniform(0.0, w.beta, size=n)
        ns.append(n)
        sites.append(np.stack([idx % w.L, idx // w.L], axis=1))
        taus.append(tau)
    n_arr = np.asarray(ns, dtype=np.int32)
    voff = np.zeros(nconf, dtype=np.int64)
    if nconf > 1:
        voff[1:] = np.cumsum(n_arr[:-1], dtype=np.int64)
    return Draw(w, n_arr, voff, np.concatenate(sites).astype(np.int32),
                np.concatenate(taus).astype(np.float64), delta)


def random_matrices(seed: int, n: int, ng: int, scale: float = 1.0) -> np.ndarray:
    """Generic test matrices (standard normal * scale), shape (ng, n, n)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(size=(ng, n, n)) * scale
