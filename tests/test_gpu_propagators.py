"""Propagator kernels (cos_build_g0, cos_build_g0_honeycomb) against the
oracle's builders in the regimes their closed forms separate: both signs of
xi and xi = 0 exactly (mu = -4t puts xi(k = 0) at zero on the square lattice),
forward, equal-time (read as 0^-) and backward time differences, tau = 0 and
tau just below beta, large beta |xi| (exponents down to about -480), odd and
even L down to L = 1 (the phase index (k . dr) mod L over negative and
wrapped site differences), and orders up to 12 (144 entries: more than one
pass of a workgroup's threads).  Methods, square-lattice dispersion and the
honeycomb Bloch Hamiltonian."""
import numpy as np
import pytest

from gpu_util import announce

pytestmark = pytest.mark.gpu


def _configs(L, beta, orders, seed):
    rng = np.random.default_rng(seed)
    out = []
    for n in orders:
        sites = rng.integers(0, L, size=(n, 2)).astype(np.int32)
        tau = rng.uniform(0.0, beta, size=n)
        if n >= 3:
            tau[1] = tau[0] = 0.0                   # an equal-time pair at tau = 0
            tau[2] = np.nextafter(beta, 0.0)        # d just below +-beta against them
        if n >= 5:
            tau[4] = tau[3]                         # an equal-time pair inside (0, beta)
            sites[4] = sites[3]                     # on one site: the local density
        out.append((sites, tau))
    return out


def _offsets(orders, per_config):
    n = np.asarray(orders, dtype=np.int32)
    voff = np.zeros(n.size, dtype=np.int64)
    voff[1:] = np.cumsum(n[:-1])
    sizes = per_config(n.astype(np.int64))
    off = np.zeros(n.size, dtype=np.int64)
    off[1:] = np.cumsum(sizes[:-1])
    return n, voff, sizes, off


def _close(got, ref, what):
    # entry by entry within 1e-12 relative, or 1e-13 of the matrix's largest
    # entry where the momentum sum cancels (a sum of L^2 terms of that size)
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(got - ref))
    print("  %s: max |ref| %.3e, max abs err %.2e" % (what, scale, err), flush=True)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-13 * scale), (what, err, scale)


@pytest.mark.parametrize("L,beta", [(1, 3.0), (2, 7.5), (5, 60.0), (8, 4.0), (9, 25.0)])
def test_square_lattice_propagators(L, beta):
    import torch
    from oracle import g0
    from paper_2507_12349_amd import _binding as B
    announce("square-lattice propagators L=%d beta=%g" % (L, beta))
    t = 1.0
    mu = np.array([-4.0 * t, 1.5, -0.3])    # xi >= 0 with xi(0) = 0; both signs; both signs
    alpha = np.array([0.0, 0.0, 0.2])
    orders = [1, 3, 6, 12, 5]
    cf = _configs(L, beta, orders, seed=L)
    nmat = mu.size
    n, voff, sizes, off = _offsets(orders, lambda k: nmat * k * k)
    dev = torch.device("cuda:0")
    G = torch.full((int(sizes.sum()),), float("nan"), dtype=torch.float64, device=dev)
    dG = torch.full_like(G, float("nan"))
    B.build_g0(n.size, torch.as_tensor(n, device=dev), torch.as_tensor(voff, device=dev),
               torch.as_tensor(np.concatenate([s for s, _ in cf]).reshape(-1), device=dev),
               torch.as_tensor(np.concatenate([tau for _, tau in cf]), device=dev), L, t, beta, mu, alpha,
               torch.as_tensor(off, device=dev), G, dG)
    torch.cuda.synchronize()
    Gh, dGh = G.cpu().numpy(), dG.cpu().numpy()
    for c, (sites, tau) in enumerate(cf):
        Go, dGo = g0.build_g0(L, t, beta, mu, alpha, sites, tau)
        k = orders[c]
        _close(Gh[off[c]:off[c] + sizes[c]].reshape(nmat, k, k), Go, "G n=%d" % k)
        _close(dGh[off[c]:off[c] + sizes[c]].reshape(nmat, k, k), dGo, "dG/dxi n=%d" % k)


@pytest.mark.parametrize("L,beta", [(1, 2.0), (3, 30.0), (4, 5.0)])
def test_honeycomb_propagators(L, beta):
    import torch
    from oracle import g0_honeycomb as GH
    from paper_2507_12349_amd import _binding as B
    announce("honeycomb propagators L=%d beta=%g" % (L, beta))
    t = 1.0
    mu = np.array([0.3, -1.2])
    alpha = np.array([0.1, 0.0])
    delta = np.array([0.4, 0.0])           # a staggered field; none (L = 3 holds the Dirac points, r near 0)
    orders = [1, 4, 9, 12]
    cf = _configs(L, beta, orders, seed=10 + L)
    nmat = mu.size
    n, voff, sizes, off = _offsets(orders, lambda k: nmat * (2 * k) ** 2)
    dev = torch.device("cuda:0")
    G = torch.full((int(sizes.sum()),), float("nan"), dtype=torch.float64, device=dev)
    dG = torch.full_like(G, float("nan"))
    B.build_g0_honeycomb(n.size, torch.as_tensor(n, device=dev), torch.as_tensor(voff, device=dev),
                         torch.as_tensor(np.concatenate([s for s, _ in cf]).reshape(-1), device=dev),
                         torch.as_tensor(np.concatenate([tau for _, tau in cf]), device=dev), L, t, beta, mu,
                         alpha, delta, torch.as_tensor(off, device=dev), G, dG=dG)
    torch.cuda.synchronize()
    Gh, dGh = G.cpu().numpy(), dG.cpu().numpy()
    for c, (cells, tau) in enumerate(cf):
        k = orders[c]
        Go = GH.build_g0(L, t, beta, mu, alpha, delta, cells, tau)
        dGo = GH.build_dg0(L, t, beta, mu, alpha, delta, cells, tau)
        _close(Gh[off[c]:off[c] + sizes[c]].reshape(nmat, 2 * k, 2 * k), Go, "G n=%d" % k)
        _close(dGh[off[c]:off[c] + sizes[c]].reshape(nmat, 2 * k, 2 * k), dGo, "dG/dxi n=%d" % k)
