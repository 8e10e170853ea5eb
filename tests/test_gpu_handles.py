"""cos_release and batch handles.  Every handle of an order points into the
same cached state tables, so cos_release refuses (COS_EINVAL) while a handle is
alive and that handle keeps computing the same sums; once no handle is left
the tables are freed and the next call rebuilds them."""
import os
import subprocess
import sys

import numpy as np
import pytest

from gpu_util import announce, gpu_forward

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_release_refused_while_a_handle_is_alive():
    import torch
    from paper_2507_12349_amd import _binding as B
    announce("cos_release with a live handle")
    rng = np.random.default_rng(5)
    G = torch.as_tensor(rng.normal(size=70 * 36) * 0.5, device="cuda:0")
    out = torch.full((70,), float("nan"), dtype=torch.float64, device="cuda:0")
    b = B.Batch([6] * 70, 4, B.UNIFORM)
    try:
        b.forward(G, None, None, -1.0, out)
        torch.cuda.synchronize()
        S0 = out.cpu().numpy()
        assert np.all(np.isfinite(S0))
        assert B.lib.cos_release() == -1   # COS_EINVAL
        assert b"alive" in B.lib.cos_last_error()
        out.fill_(float("nan"))
        b.forward(G, None, None, -1.0, out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), S0)
    finally:
        b.close()
    # a fresh handle of the same order still agrees bitwise
    S1 = gpu_forward([G.cpu().numpy()[36 * i:36 * (i + 1)].reshape(1, 6, 6) for i in range(70)], 4, 0)
    assert np.array_equal(S1, S0)


_FRESH = r"""
import numpy as np
from paper_2507_12349_amd import _binding as B
G = np.random.default_rng(7).normal(size=(2, 7, 7)) * 0.5
a = B.connected_sum_host(G, 2, B.FLAVOUR)          # plans, runs and destroys its own handle
assert B.lib.cos_release() == 0, B.lib.cos_last_error()
b = B.connected_sum_host(G, 2, B.FLAVOUR)          # tables rebuilt
assert a == b and np.isfinite(a), (a, b)
assert B.lib.cos_release() == 0
print("release-ok", a)
"""


def test_release_frees_and_rebuilds_the_tables():
    """In a process of its own, so that no handle of another test is alive."""
    announce("cos_release after every handle is destroyed (child process)")
    env = dict(os.environ, PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    r = subprocess.run([sys.executable, "-c", _FRESH], capture_output=True, text=True, timeout=120, cwd=ROOT,
                       env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "release-ok" in r.stdout


def test_binding_rejects_bad_buffers():
    """The binding checks every device buffer of a call before the library
    launches anything: a host array, another dtype, a strided view, a buffer
    shorter than the call needs, offsets of another type.  A correct call on
    the same handle then still works."""
    import torch
    from paper_2507_12349_amd import _binding as B
    announce("binding buffer checks")
    dev = torch.device("cuda:0")
    b = B.Batch([5] * 3, 2, B.FLAVOUR, stubs=True)
    try:
        G = torch.zeros(3 * 2 * 25, dtype=torch.float64, device=dev)
        st = torch.zeros(3 * 2, dtype=torch.float64, device=dev)
        out = torch.zeros(3, dtype=torch.float64, device=dev)
        bad = [
            dict(G=G.cpu()),                                         # host memory
            dict(G=G.float()),                                       # float32
            dict(G=G[:-1]),                                          # one element short
            dict(G=torch.zeros(2 * G.numel(), dtype=torch.float64, device=dev)[::2]),   # strided
            dict(out=out[:2]),
            dict(stub=st[:5]),
            dict(Goff=torch.zeros(3, dtype=torch.int32, device=dev)),
            dict(Goff=torch.zeros(2, dtype=torch.int64, device=dev)),
        ]
        for kw in bad:
            a = dict(G=G, Goff=None, stub=st, out=out)
            a.update(kw)
            with pytest.raises((TypeError, ValueError)):
                b.forward(a["G"], a["Goff"], a["stub"], -1.0, a["out"])
        ob = torch.ones(3, dtype=torch.float64, device=dev)
        with pytest.raises(ValueError):
            b.adjoint(G, None, st, -1.0, ob, out, torch.zeros(G.numel() - 1, dtype=torch.float64, device=dev), st.clone())
        with pytest.raises(ValueError):
            b.adjoint(G, None, st, -1.0, ob[:1], out, torch.zeros_like(G), st.clone())
        with pytest.raises(ValueError):
            b.adjoint(G, None, st, -1.0, ob, out, torch.zeros_like(G), st[:1].clone())
        out.fill_(float("nan"))
        b.forward(G, None, st, -1.0, out)
        torch.cuda.synchronize()
        assert np.all(out.cpu().numpy() == 0.0)   # zero propagators: S = 0 exactly
    finally:
        b.close()


def test_binding_rejects_bad_buffers_of_the_other_entry_points():
    """Propagator builders, chain rule, sampler, moments and CDet: a host
    array, another dtype or a buffer shorter than the call needs is rejected
    before the library is called."""
    import torch
    from paper_2507_12349_amd import _binding as B
    announce("binding buffer checks: builders, chain rule, sampler, moments, CDet")
    dev = torch.device("cuda:0")
    nconf, n = 4, 3
    nvec = torch.full((nconf,), n, dtype=torch.int32, device=dev)
    voff = torch.arange(nconf, dtype=torch.int64, device=dev) * n
    sites = torch.zeros((nconf * n, 2), dtype=torch.int32, device=dev)
    tau = torch.zeros(nconf * n, dtype=torch.float64, device=dev)
    Goff = torch.arange(nconf, dtype=torch.int64, device=dev) * (n * n)
    G = torch.zeros(nconf * n * n, dtype=torch.float64, device=dev)
    args = dict(n=nvec, voff=voff, sites=sites, tau=tau, Goff=Goff, G=G)
    for key, bad in (("n", nvec.long()), ("voff", voff[:2]), ("sites", sites.long()), ("tau", tau.float()),
                     ("Goff", Goff.cpu()), ("G", G.float())):
        a = dict(args)
        a[key] = bad
        with pytest.raises((TypeError, ValueError)):
            B.build_g0(nconf, a["n"], a["voff"], a["sites"], a["tau"], 4, 1.0, 2.0, [0.0], [0.0], a["Goff"], a["G"])
    with pytest.raises(ValueError):
        B.build_g0(nconf, nvec, voff, sites, tau, 4, 1.0, 2.0, [0.0], [0.0], Goff, G, G[:-1].clone())
    with pytest.raises(ValueError):
        B.mc_sample(nconf, n, 4, 2.0, 1, 0, sites, tau[:-1])
    with pytest.raises(ValueError):
        B.accumulate_moments(nconf, tau[:nconf], torch.zeros(1, dtype=torch.float64, device=dev))
    mub = torch.zeros(nconf, dtype=torch.float64, device=dev)
    with pytest.raises(ValueError):
        B.chain_mu_shift(nconf, nvec, 1, Goff, G, G.clone(), None, 1, 1.0, mub[:3], mub.clone())
    with pytest.raises(ValueError):
        B.cdet_su2(torch.zeros(2 * 4 * 4, dtype=torch.float64, device=dev), 2, 0, torch.zeros(2, dtype=torch.float64, device=dev))
    # the same buffers, well formed, go through
    B.build_g0(nconf, nvec, voff, sites, tau, 4, 1.0, 2.0, [0.0], [0.0], Goff, G, torch.empty_like(G))
    B.mc_sample(nconf, n, 4, 2.0, 1, 0, sites, tau)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(G.cpu().numpy()))
