"""Failure handling, forced from the host (cos_inject_failures): a device
allocation that fails surfaces as COS_ENOMEM, or for the level workspaces
as a retry with halved chunks whose results are unchanged; a kernel launch
that fails surfaces as COS_EDEVICE; the library works normally afterwards.
No kernel faults: an injected failure is decided on the host before the
allocation or launch."""
import numpy as np
import pytest

from gpu_util import announce

pytestmark = pytest.mark.gpu


def _setup(nconf=150, n=6, nflav=2, seed=77):
    import torch
    rng = np.random.default_rng(seed)
    G = torch.as_tensor(rng.normal(size=nconf * n * n) * 0.4, device="cuda:0")
    out = torch.empty(nconf, dtype=torch.float64, device="cuda:0")
    return G, out


def _reference(B, G, out, nconf, n, nflav):
    b = B.Batch(np.full(nconf, n, dtype=np.int32), nflav, B.UNIFORM)
    b.forward(G, None, None, -1.0, out)
    import torch
    torch.cuda.synchronize()
    b.close()
    return out.clone()


def test_allocation_failures():
    import torch
    from paper_2507_12349_amd import _binding as B
    announce("injected device allocation failures")
    nconf, n = 150, 6
    G, out = _setup(nconf, n)
    ref = _reference(B, G, out, nconf, n, 2)   # also caches the order's state tables
    try:
        # the first allocation of the plan fails: COS_ENOMEM, nothing left behind
        B.inject_failures(0, 0, 1)
        with pytest.raises(B.CosError) as e:
            B.Batch(np.full(nconf, n, dtype=np.int32), 2, B.UNIFORM)
        assert e.value.status == -3
        # the level windows fail once: retried with halved chunks (3 groups -> 2 per chunk)
        B.inject_failures(0, 4, 1)
        b = B.Batch(np.full(nconf, n, dtype=np.int32), 2, B.UNIFORM)
        out.fill_(float("nan"))
        b.forward(G, None, None, -1.0, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        b.close()
        # the level windows fail at every size: COS_ENOMEM once one group per chunk fails too
        B.inject_failures(0, 4, 1000)
        with pytest.raises(B.CosError) as e:
            B.Batch(np.full(nconf, n, dtype=np.int32), 2, B.UNIFORM)
        assert e.value.status == -3 and "one group per chunk" in str(e.value)
        # the reverse sweep's first call: its gradient accumulators fail
        B.inject_failures(0, 0, 0)
        b = B.Batch(np.full(nconf, n, dtype=np.int32), 2, B.UNIFORM)
        Gb = torch.empty_like(G)
        ob = torch.ones(nconf, dtype=torch.float64, device=G.device)
        B.inject_failures(0, 0, 1)
        with pytest.raises(B.CosError) as e:
            b.adjoint(G, None, None, -1.0, ob, out, Gb, None)
        assert e.value.status == -3
        # and the next call succeeds
        out.fill_(float("nan"))
        b.adjoint(G, None, None, -1.0, ob, out, Gb, None)
        torch.cuda.synchronize()
        assert torch.equal(out, ref) and bool(torch.isfinite(Gb).all())
        b.close()
    finally:
        B.inject_failures(0, 0, 0)


def test_launch_failure():
    import torch
    from paper_2507_12349_amd import _binding as B
    announce("injected kernel launch failure")
    nconf, n = 150, 6
    G, out = _setup(nconf, n, seed=78)
    ref = _reference(B, G, out, nconf, n, 2)
    b = B.Batch(np.full(nconf, n, dtype=np.int32), 2, B.UNIFORM)
    try:
        B.inject_failures(1, 3, 1)   # the pack and two level launches proceed, the third level fails
        with pytest.raises(B.CosError) as e:
            b.forward(G, None, None, -1.0, out)
        assert e.value.status == -4 and "injected" in str(e.value)
        torch.cuda.synchronize()
        out.fill_(float("nan"))
        b.forward(G, None, None, -1.0, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
    finally:
        B.inject_failures(1, 0, 0)
        b.close()


@pytest.mark.parametrize("skip", [2, 40])
def test_launch_failure_side_stream(skip):
    """A batch of three orders runs the two smaller ones on its side stream.
    A failed launch there (skip = 2: the side stream's pack and first level
    proceed) or on the caller's stream (skip = 40: past the side orders'
    launches) surfaces as COS_EDEVICE, the call still joins the side stream
    back (the caller's stream drains), and the next call gives the sums of a
    fresh batch."""
    import torch
    from gpu_util import pack
    from paper_2507_12349_amd import _binding as B
    announce("injected launch failure with a side stream (skip %d)" % skip)
    rng = np.random.default_rng(79 + skip)
    orders = [8, 6, 5] * 30
    flat, off, n = pack([rng.normal(size=(2, k, k)) * 0.5 for k in orders])
    G, Goff = torch.as_tensor(flat, device="cuda:0"), torch.as_tensor(off, device="cuda:0")
    out = torch.empty(len(orders), dtype=torch.float64, device="cuda:0")
    ref = torch.empty_like(out)
    r = B.Batch(n, 2, B.FLAVOUR)
    r.forward(G, Goff, None, -1.0, ref)
    torch.cuda.synchronize()
    r.close()
    b = B.Batch(n, 2, B.FLAVOUR)
    try:
        B.inject_failures(1, skip, 1)
        with pytest.raises(B.CosError) as e:
            b.forward(G, Goff, None, -1.0, out)
        assert e.value.status == -4 and "injected" in str(e.value)
        B.inject_failures(1, 0, 0)
        torch.cuda.synchronize()
        out.fill_(float("nan"))
        b.forward(G, Goff, None, -1.0, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
    finally:
        B.inject_failures(1, 0, 0)
        b.close()
