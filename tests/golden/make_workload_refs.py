"""Writes the reference sums of the synthetic workloads (tests/golden/refs_*.npz)
by calling only the oracle package and the seeded input generator (which holds
no arithmetic of the method), never the GPU library.

The method is exact (Results, "Theoretical Constructions": the clow / cycle
cover DP reaches the sum of all connected diagrams), so every configuration
has one answer.  For each selected configuration c of a workload:

  G_c, dG_c   the oracle's propagators (oracle.g0, float64) and dG/dxi
  ghash       64-bit BLAKE2b digest of the bytes of G_c, so that a test can
              tell that it rebuilt exactly these inputs before comparing
  S           oracle.dp in long double (the DP with the rules of Alg. 2/3,
              shift heads as in Alg. 3), rounded to float64
  S_abs       the same DP on |G|, |w| and |sigma| (the scale of the rounding
              error; kappa = S_abs / |S| measures the cancellation)

and for the adjoint workload (uniform SU(4), shift derivative at delta = 0)
also the reverse sweep oracle.dp_adjoint (long double): dS/dG, dS/dsigma, and
the chain rule with the oracle's dG/dxi (Methods: xi = eps - mu + alpha,
sigma = alpha / U): mu_bar = -sum dS/dG * dG/dxi, alpha_bar = +sum dS/dG *
dG/dxi + dS/dsigma / U.

Selections: every configuration of plain_single, plain_batch, sym_broken and
adjoint; for the uneven workload the first 512 configurations (every order
6..12, including the six-flavour order-12 shift path) plus every configuration
of order <= 9 among the rest.

Run (CPU, about half an hour on 8 cores):
    python tests/golden/make_workload_refs.py [--jobs 8] [--only NAME ...]
"""
from __future__ import annotations

import argparse
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

from oracle_inputs import ghash, params, propagators, selection  # noqa: E402

NAMES = ("plain_single", "plain_batch", "sym_broken", "adjoint", "uneven", "order12_flavour")


ORDER12 = dict(mu=(0.0, 0.0), alpha=(0.1, -0.15), U=1.0)


def order12_config():
    """The first order-12 configuration of the uneven workload's draw (16 x 16
    lattice, beta = 5) as a two-flavour problem: mu = 0, shifts alpha =
    (0.1, -0.15) in xi and as shift weights sigma = alpha / U."""
    from paper_2507_12349_amd.workloads import draw
    from oracle import g0
    d = draw("uneven", nconf=512)
    c = int(np.nonzero(d.n == 12)[0][0])
    w = d.workload
    sites, tau = d.config(c)
    al = np.array(ORDER12["alpha"])
    G, _ = g0.build_g0(w.L, w.t, w.beta, np.array(ORDER12["mu"]), al, sites, tau)
    return c, G, al / ORDER12["U"]


def order12_flavour():
    """One order-12 configuration of the flavour variant with two different
    flavour matrices and shift weights (order12_config): S, S_abs, dS/dG and
    dS/dsigma of the oracle in long double."""
    import oracle
    t0 = time.time()
    c, M, st = order12_config()
    S, Gb, sb = oracle.dp_adjoint(M, 2, 1, st, -1.0, precision="ld")
    Sa = oracle.dp(np.abs(M), 2, 1, -np.abs(st), 1.0, precision="ld")
    path = os.path.join(HERE, "refs_order12_flavour.npz")
    np.savez_compressed(path, config=np.array(c), S=np.array(S), S_abs=np.array(Sa), Gbar=Gb, sbar=sb,
                        ghash=np.array(ghash(M), dtype=np.uint64),
                        meta=np.array("uneven workload configuration %d, two flavours, mu = %s, alpha = %s, U = %g; "
                                      "oracle.dp_adjoint in long double; written by "
                                      "tests/golden/make_workload_refs.py"
                                      % (c, ORDER12["mu"], ORDER12["alpha"], ORDER12["U"])))
    print("order12_flavour -> %s (%.0f s), kappa %.1e" % (os.path.relpath(path, ROOT), time.time() - t0,
                                                           Sa / abs(S)), flush=True)


def _one(args):
    name, c = args
    import oracle
    d, _ = selection(name)
    w = d.workload
    _, _, _, stub = params(d)
    G, dG = propagators(name, c)
    Ga = G[0] if w.variant == 0 else G
    out = {"c": c, "n": int(d.n[c]), "ghash": ghash(G)}
    if name == "adjoint":
        S, Gb, sb = oracle.dp_adjoint(Ga, w.nflav, w.variant, stub, -1.0, precision="ld")
        xb = float(np.sum(Gb * dG[0]))
        out.update(Gbar=Gb.reshape(-1), sbar=float(sb[0]), mubar=-xb, alphabar=xb + float(sb[0]) / w.U)
    else:
        S = oracle.dp(Ga, w.nflav, w.variant, stub, -1.0, precision="ld")
    out["S"] = S
    out["S_abs"] = oracle.dp(np.abs(Ga), w.nflav, w.variant, None if stub is None else -np.abs(stub), 1.0,
                             precision="ld")
    return out


def make(name, jobs):
    d, idx = selection(name)
    # largest orders first, so that the long order-12 references start early
    todo = sorted(idx.tolist(), key=lambda c: -int(d.n[c]))
    t0 = time.time()
    res = {}
    with mp.get_context("fork").Pool(jobs) as pool:
        for k, r in enumerate(pool.imap_unordered(_one, [(name, c) for c in todo], chunksize=1)):
            res[r["c"]] = r
            if (k + 1) % max(1, len(todo) // 20) == 0 or k + 1 == len(todo):
                print("  %s: %d / %d configurations, %.0f s" % (name, k + 1, len(todo), time.time() - t0),
                      flush=True)
    rows = [res[c] for c in idx.tolist()]
    arrays = dict(idx=idx.astype(np.int32), n=np.array([r["n"] for r in rows], dtype=np.int32),
                  S=np.array([r["S"] for r in rows]), S_abs=np.array([r["S_abs"] for r in rows]),
                  ghash=np.array([r["ghash"] for r in rows], dtype=np.uint64))
    if name == "adjoint":
        arrays.update(Gbar=np.stack([r["Gbar"] for r in rows]), sbar=np.array([r["sbar"] for r in rows]),
                      mubar=np.array([r["mubar"] for r in rows]), alphabar=np.array([r["alphabar"] for r in rows]))
    arrays["meta"] = np.array("workload %s; oracle.dp%s in long double on oracle.g0 propagators; "
                              "written by tests/golden/make_workload_refs.py"
                              % (name, "_adjoint" if name == "adjoint" else ""))
    path = os.path.join(HERE, "refs_%s.npz" % name)
    np.savez_compressed(path, **arrays)
    kappa = arrays["S_abs"] / np.abs(arrays["S"])
    print("%s: %d configurations -> %s (%.0f s); kappa median %.1e, max %.1e, above 1e5: %d"
          % (name, idx.size, os.path.relpath(path, ROOT), time.time() - t0, np.median(kappa), kappa.max(),
             int((kappa > 1e5).sum())), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", nargs="*", default=list(NAMES))
    args = ap.parse_args()
    import oracle
    oracle.build(force=False)
    for name in args.only:
        if name == "order12_flavour":
            order12_flavour()
        else:
            make(name, args.jobs)


if __name__ == "__main__":
    main()
