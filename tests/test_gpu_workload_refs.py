"""Oracle-referenced parity over whole workloads (the method is exact: every
configuration has one connected sum; Results, "Theoretical Constructions";
Methods, Alg. 2/3 with the SB-CoS shift heads).

The references in tests/golden/refs_*.npz were written on the CPU by
tests/golden/make_workload_refs.py from the oracle alone (long double DP on the
oracle's propagators).  Here the oracle's propagators of the same
configurations are rebuilt (tests/golden/oracle_inputs.py, a child process;
each configuration's bytes must match the digest stored with the references)
and fed to the batched GPU kernels in the launch configuration bench.py times
(the whole batch, autotuned launch shapes); the GPU's own propagator kernel is
compared with them entry by entry.

Gate: |S - S_ref| <= 1e-10 |S_ref| for every configuration, except the ones
named in EXCEPTIONS: configurations whose cancellation kappa = S_abs / |S_ref|
is so large (above 1e9) that FP64 rounding alone can exceed 1e-10 relative;
each must still meet the FP64 bound 8 n (n + 2) eps S_abs.  The printed
summary gives the largest relative error per order, separately for kappa
above and below 1e5.  Gradients (adjoint workload, every configuration): dS/dG
within 1e-10 of the configuration's largest |dS/dG| entry by entry, dS/dsigma,
mu_bar and alpha_bar within 1e-10 relative to their scales.

Covered: every configuration of plain_single (1), plain_batch (4096 x n=8),
sym_broken (1024 x n=10, three flavour matrices) and adjoint (2048 x n=10, forward
and reverse sweep, chain rule); of the uneven workload (8192 configurations,
orders 6..12, six flavour matrices with shift heads) the first 512 (every
order, including 66 of order 12) and all 4392 others of order <= 9."""
import os
import subprocess
import sys
import tempfile

import numpy as np
import pytest

from gpu_util import announce

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")
KAPPA_GATE = 1e5
# (workload, configuration): kappa 2.8e9, measured relative error 1.4e-10 (FP64 bound: 6e-4)
EXCEPTIONS = {("sym_broken", 96)}


def _refs(name):
    path = os.path.join(GOLDEN, "refs_%s.npz" % name)
    if not os.path.exists(path):
        pytest.fail("missing %s: run tests/golden/make_workload_refs.py" % path)
    return dict(np.load(path))


def _oracle_inputs(name):
    """The oracle's propagators of the referenced configurations, built in a
    child process (a pool of at most 16 workers, the machine's CPU share)."""
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    jobs = max(1, min(16, ncpu))
    with tempfile.TemporaryDirectory() as tmp:
        out = os.path.join(tmp, "g.npz")
        subprocess.run([sys.executable, os.path.join(GOLDEN, "oracle_inputs.py"), name, out, "--jobs", str(jobs)],
                       check=True, timeout=900)
        return dict(np.load(out))


def _run(name, adjoint=False, deterministic=False):
    """Whole workload on the GPU: propagator kernel, then the batched forward
    (and reverse sweep + chain rule) on the oracle's propagators for the
    referenced configurations (the GPU kernel's own for the others)."""
    import torch
    from paper_2507_12349_amd import _binding as B
    from paper_2507_12349_amd.autograd import Geometry
    from paper_2507_12349_amd.workloads import draw
    sys.path.insert(0, GOLDEN)
    from oracle_inputs import params

    ref = _refs(name)
    ora = _oracle_inputs(name)
    assert np.array_equal(ora["idx"], ref["idx"])
    bad = np.nonzero(ora["ghash"] != ref["ghash"])[0]
    assert bad.size == 0, ("the oracle's propagators differ from those the references were computed on "
                           "(configurations %s)" % ref["idx"][bad[:10]].tolist())
    d = draw(name)
    w = d.workload
    nmat, mu, alpha, stub = params(d)
    geo = Geometry(d, nmat)
    dev = geo.device
    G = torch.empty(geo.total, dtype=torch.float64, device=dev)
    dG = torch.empty_like(G)
    B.build_g0(geo.nconf, geo.n, geo.voff, geo.sites, geo.tau, geo.L, geo.t, geo.beta, mu, alpha, geo.Goff, G, dG)
    torch.cuda.synchronize()
    Gk, dGk = G.cpu().numpy(), dG.cpu().numpy()
    # scatter the oracle's matrices into the batch layout
    goff = geo.Goff_host
    sel = ref["idx"].astype(np.int64)
    sizes = nmat * d.n[sel].astype(np.int64) ** 2
    pos = goff[sel]
    take = np.concatenate([np.arange(p, p + s) for p, s in zip(pos, sizes)])
    src = np.concatenate([np.arange(o, o + s) for o, s in zip(ora["off"], sizes)])
    gdiff = np.abs(Gk[take] - ora["G"][src]).max()
    ddiff = np.abs(dGk[take] - ora["dG"][src]).max() / max(1.0, np.abs(ora["dG"]).max())
    print("  %s: G0 kernel vs oracle propagators over %d configurations: max |dG| %.2e, dG/dxi rel %.2e"
          % (name, sel.size, gdiff, ddiff), flush=True)
    # the kernel sums L^2 terms of magnitude <= 1 (then divides by L^2)
    assert gdiff <= 2 * w.L * w.L * EPS, gdiff
    assert ddiff <= 2 * w.L * w.L * w.beta * EPS, ddiff
    Gk[take] = ora["G"][src]
    dGk[take] = ora["dG"][src]
    G.copy_(torch.as_tensor(Gk, device=dev))
    dG.copy_(torch.as_tensor(dGk, device=dev))
    st = None if stub is None else torch.as_tensor(np.tile(stub, (geo.nconf, 1)), device=dev)
    b = B.Batch(d.n, w.nflav, w.variant, stubs=st is not None, deterministic=deterministic)
    out = torch.full((geo.nconf,), float("nan"), dtype=torch.float64, device=dev)
    ob = torch.ones(geo.nconf, dtype=torch.float64, device=dev)
    res = {"ref": ref, "sel": sel, "d": d}
    if adjoint:
        Gb = torch.full_like(G, float("nan"))
        sb = None if st is None else torch.full_like(st, float("nan"))
        b.autotune(G, geo.Goff, st, -1.0, out, ob, Gb, sb)
        out.fill_(float("nan"))
        Gb.fill_(float("nan"))
        b.adjoint(G, geo.Goff, st, -1.0, ob, out, Gb, sb)
        mub = torch.empty(geo.nconf * nmat, dtype=torch.float64, device=dev)
        alb = torch.empty_like(mub)
        B.chain_mu_shift(geo.nconf, geo.n, nmat, geo.Goff, Gb, dG, sb, 1 if st is None else st.shape[1], w.U,
                         mub, alb)
        torch.cuda.synchronize()
        res.update(Gb=Gb.cpu().numpy(), sb=None if sb is None else sb.cpu().numpy(), mub=mub.cpu().numpy(),
                   alb=alb.cpu().numpy(), goff=goff, Gabs=np.abs(Gk), dGabs=np.abs(dGk))
    else:
        b.autotune(G, geo.Goff, st, -1.0, out)
        out.fill_(float("nan"))
        b.forward(G, geo.Goff, st, -1.0, out)
        torch.cuda.synchronize()
    res["S"] = out.cpu().numpy()
    b.close()
    assert np.all(np.isfinite(res["S"]))
    return res


def _check_sums(name, res):
    ref, sel = res["ref"], res["sel"]
    S = res["S"][sel]
    n = ref["n"].astype(np.float64)
    err = np.abs(S - ref["S"])
    rel = err / np.abs(ref["S"])
    kappa = ref["S_abs"] / np.abs(ref["S"])
    bound = 8 * n * (n + 2) * EPS * ref["S_abs"]
    gate = kappa <= KAPPA_GATE
    high = np.nonzero(~gate)[0]
    for order in np.unique(ref["n"]):
        m = (ref["n"] == order) & gate
        if m.any():
            print("  %s n=%d: %d configurations, max rel err %.2e (kappa max %.1e)"
                  % (name, order, m.sum(), rel[m].max(), kappa[m].max()), flush=True)
    if high.size:
        print("  %s: %d configurations above kappa %.0e: max rel err %.2e (kappa max %.1e)"
              % (name, high.size, KAPPA_GATE, rel[high].max(), kappa[high].max()), flush=True)
    exc = np.array([(name, int(c)) in EXCEPTIONS for c in sel])
    for i in np.nonzero(exc | (rel > 1e-10))[0]:
        print("  %s config %d (n=%d): kappa %.2e, rel err %.2e, err / FP64 bound %.2e%s"
              % (name, sel[i], ref["n"][i], kappa[i], rel[i], err[i] / bound[i],
                 " (named exception)" if exc[i] else ""), flush=True)
    bad = np.nonzero(~exc & (rel > 1e-10))[0]
    assert bad.size == 0, (name, sel[bad].tolist(), rel[bad].tolist())
    assert np.all(err[exc] <= bound[exc]), (name, sel[exc].tolist())
    return float(rel[~exc].max())


def test_refs_plain_single():
    announce("oracle references: plain_single")
    _check_sums("plain_single", _run("plain_single"))


def test_refs_plain_batch():
    announce("oracle references: plain_batch, all 4096 configurations")
    _check_sums("plain_batch", _run("plain_batch"))


def test_refs_sym_broken():
    announce("oracle references: sym_broken, all 1024 configurations")
    _check_sums("sym_broken", _run("sym_broken"))


def test_refs_uneven():
    announce("oracle references: uneven, 8192-configuration batch, 4904 configurations checked")
    res = _run("uneven")
    _check_sums("uneven", res)
    assert set(np.unique(res["ref"]["n"])) == set(range(6, 13))
    assert (res["ref"]["n"] == 12).sum() >= 60


def _check_adjoint(res, tag):
    ref, sel, d = res["ref"], res["sel"], res["d"]
    worst_g = 0.0
    for i, c in enumerate(sel):
        n = int(d.n[c])
        a = int(res["goff"][c])
        gb = res["Gb"][a:a + n * n]
        gr = ref["Gbar"][i]
        e = np.abs(gb - gr).max() / np.abs(gr).max()
        worst_g = max(worst_g, e)
        assert e <= 1e-10, (int(c), e)
    sb = res["sb"][:, 0]
    e_sb = np.abs(sb - ref["sbar"]) / np.maximum(np.abs(ref["sbar"]), 1e-300)
    # chain rule: mu_bar = -sum Gbar dG, the scale is sum |Gbar dG|
    scale = np.array([np.sum(np.abs(ref["Gbar"][i]) * res["dGabs"][int(res["goff"][c]):int(res["goff"][c])
                                                                   + int(d.n[c]) ** 2])
                      for i, c in enumerate(sel)])
    e_mu = np.abs(res["mub"] - ref["mubar"]) / scale
    e_al = np.abs(res["alb"] - ref["alphabar"]) / (scale + np.abs(ref["sbar"]))
    print("  %s: dS/dG max err / max|dS/dG| %.2e; dS/dsigma rel %.2e; mu_bar %.2e; alpha_bar %.2e"
          % (tag, worst_g, e_sb.max(), e_mu.max(), e_al.max()), flush=True)
    assert e_sb.max() <= 1e-10
    assert e_mu.max() <= 1e-10 and e_al.max() <= 1e-10


def test_refs_adjoint():
    """Forward sums, dS/dG, dS/dsigma and the chain rule of all 2048
    configurations of the adjoint workload against the oracle's reverse sweep."""
    announce("oracle references: adjoint, all 2048 configurations, forward + reverse sweep + chain rule")
    res = _run("adjoint", adjoint=True)
    _check_sums("adjoint", res)
    _check_adjoint(res, "adjoint")


def test_refs_adjoint_deterministic():
    """The same with deterministic gradients (COS_F_DETERMINISTIC)."""
    announce("oracle references: adjoint, deterministic reverse sweep, all 2048 configurations")
    res = _run("adjoint", adjoint=True, deterministic=True)
    _check_sums("adjoint", res)
    _check_adjoint(res, "adjoint, deterministic")
