"""Deterministic gradients (COS_F_DETERMINISTIC): dS/dG and dS/dsigma bit for
bit equal across runs, forward launch shapes, chunkings of the groups and
two-segment sweeps, and within the FP64 bound of the default reverse sweep
and of the oracle."""
import numpy as np
import pytest

from gpu_util import announce

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def _adjoint(B, torch, G, st, n, nflav, variant, det, w=-1.0, shape=None, limit=0, mask=False, sub=False):
    nmat = nflav if variant else 1
    side = 2 * n if sub else n
    nconf = G.numel() // (nmat * side * side)
    B.set_workspace_limit(limit)
    b = B.Batch(np.full(nconf, n, dtype=np.int32), nflav, variant, stubs=st is not None, deterministic=det,
                mask_only=mask, sublattice=sub)
    B.set_workspace_limit(0)
    if shape:
        b.set_launch_shape(n, *shape)
    out = torch.empty(nconf, dtype=torch.float64, device=G.device)
    Gb = torch.empty_like(G)
    sb = None if st is None else torch.empty_like(st)
    ob = torch.linspace(-1.0, 2.0, nconf, dtype=torch.float64, device=G.device)
    b.adjoint(G, None, st, w, ob, out, Gb, sb)
    torch.cuda.synchronize()
    b.close()
    return out.cpu().numpy(), Gb.cpu().numpy(), None if sb is None else sb.cpu().numpy()


@pytest.mark.parametrize("n,nflav,variant,stubs,mask,nconf", [
    (5, 2, 0, True, False, 130), (8, 4, 0, True, False, 150), (9, 3, 1, True, False, 70),
    (8, 2, 1, False, True, 100), (10, 4, 0, False, False, 64)])
def test_deterministic_gradients(oracle_mod, n, nflav, variant, stubs, mask, nconf):
    import torch
    from paper_2507_12349_amd import _binding as B
    announce("deterministic reverse: n=%d nflav=%d variant=%d stubs=%s mask_only=%s nconf=%d"
             % (n, nflav, variant, stubs, mask, nconf))
    rng = np.random.default_rng(900 + n)
    nmat = nflav if variant else 1
    G = torch.as_tensor(rng.normal(size=nconf * nmat * n * n) * 0.3, device="cuda:0")
    st = torch.as_tensor(rng.normal(size=(nconf, nmat)) * 0.2, device="cuda:0") if stubs else None
    runs = [_adjoint(B, torch, G, st, n, nflav, variant, True, mask=mask),
            _adjoint(B, torch, G, st, n, nflav, variant, True, mask=mask),
            _adjoint(B, torch, G, st, n, nflav, variant, True, shape=(4, 1, 2), mask=mask),
            _adjoint(B, torch, G, st, n, nflav, variant, True, limit=1, mask=mask)]   # one group per chunk
    S0, g0, s0 = runs[0]
    for S, g, s in runs[1:]:
        assert np.array_equal(S, S0)
        assert np.array_equal(g, g0)
        if stubs:
            assert np.array_equal(s, s0)
    # the default (atomic) reverse, and the scale of the rounding from |G|
    S1, g1, s1 = _adjoint(B, torch, G, st, n, nflav, variant, False, mask=mask)
    assert np.array_equal(S1, S0)
    if mask:
        # the mask-only variant takes w = -1 only: no absolute-value run; compare to the largest entry
        bound = 1e-10 * np.abs(g1).max() + np.zeros_like(g1)
    else:
        _, ga, sa = _adjoint(B, torch, G.abs(), None if st is None else -st.abs(), n, nflav, variant, False,
                             w=1.0)
        bound = 2 * 8 * n * (n + 2) * EPS * np.abs(ga) + 1e-300
    print("  max |det - default| / FP64 bound: %.2e" % (np.abs(g0 - g1) / bound).max(), flush=True)
    assert np.all(np.abs(g0 - g1) <= bound)
    if stubs:
        assert np.all(np.abs(s0 - s1) <= 2 * 8 * n * (n + 2) * EPS * np.abs(sa) + 1e-300)
    # two configurations against the oracle's reverse sweep
    if not mask and n <= 9:
        ob = np.linspace(-1.0, 2.0, nconf)
        Gh = G.cpu().numpy().reshape(nconf, nmat, n, n)
        for c in (0, nconf - 1):
            Ga = Gh[c, 0] if variant == 0 else Gh[c]
            sc = None if st is None else st.cpu().numpy()[c]
            _, gref, _ = oracle_mod.dp_adjoint(Ga, nflav, variant, sc, -1.0)
            gd = g0[c * nmat * n * n:(c + 1) * nmat * n * n].reshape(Ga.shape)
            assert np.allclose(gd, ob[c] * gref, rtol=0, atol=1e-10 * np.abs(ob[c] * gref).max())
