"""Gradients on the honeycomb lattice: the propagator derivative dG/dxi
(cos_build_g0_honeycomb) against the oracle, and dS/dmu, dS/dalpha of the
sublattice-summed sum through propagators -> reverse sweep -> chain rule, all
on the GPU, against the oracle's chain of the same steps."""
import numpy as np
import pytest

from gpu_util import announce

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def _device_problem(cells_list, tau_list, L, t, beta, mu, alpha, delta):
    import torch
    from paper_2507_12349_amd import _binding as B
    dev = torch.device("cuda:0")
    n = np.array([len(x) for x in tau_list], dtype=np.int32)
    nmat = len(mu)
    voff = np.zeros(n.size, dtype=np.int64)
    voff[1:] = np.cumsum(n[:-1])
    sizes = nmat * (2 * n.astype(np.int64)) ** 2
    off = np.zeros(n.size, dtype=np.int64)
    off[1:] = np.cumsum(sizes[:-1])
    G = torch.full((int(sizes.sum()),), float("nan"), dtype=torch.float64, device=dev)
    dG = torch.full_like(G, float("nan"))
    Goff = torch.as_tensor(off, device=dev)
    B.build_g0_honeycomb(n.size, torch.as_tensor(n, device=dev), torch.as_tensor(voff, device=dev),
                         torch.as_tensor(np.concatenate(cells_list).astype(np.int32), device=dev),
                         torch.as_tensor(np.concatenate(tau_list), device=dev), L, t, beta, np.array(mu),
                         np.array(alpha), np.array(delta), Goff, G, dG=dG)
    return n, off, sizes, G, dG, Goff


def test_dg0_against_oracle():
    from oracle import g0_honeycomb as GH
    from paper_2507_12349_amd.workloads import draw
    announce("honeycomb dG/dxi vs oracle")
    d = draw("honeycomb", nconf=3)
    w = d.workload
    cells = [d.config(c)[0] for c in range(3)]
    taus = [d.config(c)[1] for c in range(3)]
    alpha = np.array([0.05, -0.05])
    n, off, sizes, G, dG, _ = _device_problem(cells, taus, w.L, w.t, w.beta, w.mu, alpha, w.stagger)
    Gh, dGh = G.cpu().numpy(), dG.cpu().numpy()
    for c in range(3):
        Go = GH.build_g0(w.L, w.t, w.beta, np.array(w.mu), alpha, np.array(w.stagger), cells[c], taus[c])
        dGo = GH.build_dg0(w.L, w.t, w.beta, np.array(w.mu), alpha, np.array(w.stagger), cells[c], taus[c])
        assert np.allclose(Gh[off[c]:off[c] + sizes[c]].reshape(Go.shape), Go, rtol=1e-12, atol=1e-14), c
        got = dGh[off[c]:off[c] + sizes[c]].reshape(dGo.shape)
        assert np.allclose(got, dGo, rtol=1e-11, atol=1e-13 * np.max(np.abs(dGo))), (c, np.max(np.abs(got - dGo)))


def test_mu_and_shift_gradients(oracle_mod):
    """Orders 2..5 on the honeycomb workload's lattice (first vertices of its
    configurations), two flavours with a staggered field: dS/dmu_f and
    dS/dalpha_f per configuration."""
    import torch
    from oracle import g0_honeycomb as GH
    from oracle import sublattice as SL
    from paper_2507_12349_amd import _binding as B
    from paper_2507_12349_amd.workloads import draw
    announce("honeycomb dS/dmu, dS/dalpha end to end")
    d = draw("honeycomb", nconf=4)
    w = d.workload
    orders = [2, 3, 4, 5]
    cells = [d.config(c)[0][:k] for c, k in enumerate(orders)]
    taus = [d.config(c)[1][:k] for c, k in enumerate(orders)]
    mu, alpha, delta = np.array(w.mu), np.array([0.05, -0.05]), np.array(w.stagger)
    n, off, sizes, G, dG, Goff = _device_problem(cells, taus, w.L, w.t, w.beta, mu, alpha, delta)
    dev = G.device
    b = B.Batch(n, 2, B.FLAVOUR, sublattice=True)
    S = torch.empty(n.size, dtype=torch.float64, device=dev)
    Gb = torch.full_like(G, float("nan"))
    b.adjoint(G, Goff, None, -1.0, torch.ones(n.size, dtype=torch.float64, device=dev), S, Gb, None)
    mub = torch.full((n.size * 2,), float("nan"), dtype=torch.float64, device=dev)
    alb = torch.full_like(mub, float("nan"))
    side = torch.as_tensor(2 * n, device=dev)   # the chain rule takes the matrix side
    B.chain_mu_shift(n.size, side, 2, Goff, Gb, dG, None, 1, 1.0, mub, alb)
    torch.cuda.synchronize()
    b.close()
    mub, alb = mub.cpu().numpy().reshape(-1, 2), alb.cpu().numpy().reshape(-1, 2)
    for c, k in enumerate(orders):
        Go = GH.build_g0(w.L, w.t, w.beta, mu, alpha, delta, cells[c], taus[c])
        dGo = GH.build_dg0(w.L, w.t, w.beta, mu, alpha, delta, cells[c], taus[c])
        _, g = SL.by_assignment_adjoint(Go, 2, 1)
        _, gabs = SL.by_assignment_adjoint(np.abs(Go), 2, 1, 1.0)
        for f in range(2):
            ref = -np.sum(g[f] * dGo[f])
            tol = 8 * k * (k + 2) * EPS * np.sum(gabs[f] * np.abs(dGo[f])) + 1e-14 * abs(ref)
            assert abs(mub[c, f] - ref) <= tol, (c, f, mub[c, f], ref, tol)
            assert alb[c, f] == -mub[c, f]
