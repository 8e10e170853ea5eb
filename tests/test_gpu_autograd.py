"""The torch.autograd path end to end: (mu, alpha) -> propagators ->
connected sums -> scalar loss, backward through the reverse sweep and the
chain-rule kernels, on the square lattice (G0Propagator) and the honeycomb
lattice with sublattice labels (HoneycombPropagator), against the oracle's
chain of the same steps."""
import numpy as np
import pytest

from gpu_util import announce

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def test_square_lattice_mu_alpha_gradient(oracle_mod):
    import torch
    from oracle import g0
    from paper_2507_12349_amd import _binding as B
    from paper_2507_12349_amd.autograd import ConnectedSum, G0Propagator, Geometry
    from paper_2507_12349_amd.workloads import draw
    announce("autograd: square lattice, three flavours, orders 4..6")
    d = draw("sym_broken", nconf=3).prefix([4, 5, 6])
    w = d.workload
    geo = Geometry(d, w.nflav)
    mu = torch.tensor(w.mu, dtype=torch.float64, requires_grad=True)
    alpha = torch.tensor([0.02, -0.01, 0.03], dtype=torch.float64, requires_grad=True)
    b = B.Batch(d.n, w.nflav, B.FLAVOUR)
    G = G0Propagator.apply(mu, alpha, geo)
    S = ConnectedSum.apply(G, None, b, geo.Goff, -1.0)
    weights = torch.tensor([1.0, -0.5, 0.25], dtype=torch.float64, device=S.device)
    (S * weights).sum().backward()
    b.close()
    ref_mu, scale = np.zeros(3), np.zeros(3)
    for c in range(3):
        sites, tau = d.config(c)
        Go, dGo = g0.build_g0(w.L, w.t, w.beta, np.array(w.mu), alpha.detach().numpy(), sites, tau)
        _, g, _ = oracle_mod.dp_adjoint(Go, w.nflav, 1, None, -1.0)
        _, gabs, _ = oracle_mod.dp_adjoint(np.abs(Go), w.nflav, 1, None, 1.0)
        ref_mu += weights[c].item() * -np.sum(g * dGo, axis=(1, 2))
        k = int(d.n[c])
        scale += abs(weights[c].item()) * 8 * k * (k + 2) * EPS * np.sum(gabs * np.abs(dGo), axis=(1, 2))
    assert np.all(np.abs(mu.grad.numpy() - ref_mu) <= scale + 1e-14), (mu.grad.numpy(), ref_mu, scale)
    assert np.array_equal(alpha.grad.numpy(), -mu.grad.numpy())


def test_honeycomb_mu_alpha_gradient(oracle_mod):
    import torch
    from oracle import g0_honeycomb as GH
    from oracle import sublattice as SL
    from paper_2507_12349_amd import _binding as B
    from paper_2507_12349_amd.autograd import ConnectedSum, Geometry, HoneycombPropagator
    from paper_2507_12349_amd.workloads import draw
    announce("autograd: honeycomb, two flavours, sublattice labels, orders 3..5")
    d = draw("honeycomb", nconf=3).prefix([3, 4, 5])
    w = d.workload
    geo = Geometry(d, w.nflav, sublattice=True)
    mu = torch.tensor(w.mu, dtype=torch.float64, requires_grad=True)
    alpha = torch.tensor([0.05, -0.05], dtype=torch.float64, requires_grad=True)
    b = B.Batch(d.n, w.nflav, B.FLAVOUR, sublattice=True)
    G = HoneycombPropagator.apply(mu, alpha, w.stagger, geo)
    S = ConnectedSum.apply(G, None, b, geo.Goff, -1.0)
    S.sum().backward()
    b.close()
    ref_mu, scale = np.zeros(2), np.zeros(2)
    for c in range(3):
        cells, tau = d.config(c)
        args = (w.L, w.t, w.beta, np.array(w.mu), alpha.detach().numpy(), np.array(w.stagger), cells, tau)
        Go, dGo = GH.build_g0(*args), GH.build_dg0(*args)
        _, g = SL.by_assignment_adjoint(Go, 2, 1)
        _, gabs = SL.by_assignment_adjoint(np.abs(Go), 2, 1, 1.0)
        ref_mu += -np.sum(g * dGo, axis=(1, 2))
        k = int(d.n[c])
        scale += 8 * k * (k + 2) * EPS * np.sum(gabs * np.abs(dGo), axis=(1, 2))
    assert np.all(np.abs(mu.grad.numpy() - ref_mu) <= scale + 1e-14), (mu.grad.numpy(), ref_mu, scale)
    assert np.array_equal(alpha.grad.numpy(), -mu.grad.numpy())
