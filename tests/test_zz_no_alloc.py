"""The forward entry point that allocates no device memory
(cos_connected_sum_static), called through the C ABI, against the batched
forward (cos_connected_sum_batched) on the same inputs: the same kernels
compute both, and a configuration's sum does not depend on the launch shape or
on how the groups are chunked, so the sums must agree bit for bit.  Two calls
in a row, the second with a smaller input (the static workspace keeps the last
call's contents); a call replayed from a graph; sizes beyond the static
workspace rejected before any launch; and a few sums against the oracle."""
import numpy as np
import pytest

from gpu_util import announce

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def _inputs(seed, nconf, n, nmat, stubs):
    rng = np.random.default_rng(seed)
    G = rng.normal(size=(nconf, nmat, n, n)) * 0.3
    st = rng.normal(size=(nconf, nmat)) * 0.2 if stubs else None
    return G, st


def _batched(B, torch, G, st, n, nflav, variant):
    dev = torch.device("cuda:0")
    nconf = G.shape[0]
    b = B.Batch(np.full(nconf, n, dtype=np.int32), nflav, variant, stubs=st is not None)
    out = torch.full((nconf,), float("nan"), dtype=torch.float64, device=dev)
    b.forward(torch.as_tensor(G.reshape(-1), device=dev), None,
              None if st is None else torch.as_tensor(st, device=dev), -1.0, out)
    torch.cuda.synchronize()
    b.close()
    return out.cpu().numpy()


def _static(B, torch, G, st, n, nflav, variant):
    dev = torch.device("cuda:0")
    nconf = G.shape[0]
    out = torch.full((nconf,), float("nan"), dtype=torch.float64, device=dev)
    B.connected_sum_static(torch.as_tensor(G.reshape(-1), device=dev), n, nflav, variant,
                           None if st is None else torch.as_tensor(st, device=dev), -1.0, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_static_equals_batched_two_calls(oracle_mod):
    import torch
    from paper_2507_12349_amd import _binding as B
    # first call: order 8, SU(4) uniform, 300 configurations = 5 groups of 64,
    # more than the level windows of one chunk hold (4 groups at order 8), so
    # the call runs two chunks; second call: smaller, order 6 with three
    # flavour matrices and shift weights
    cases = [(8, 4, B.UNIFORM, 300, False, 11), (6, 3, B.FLAVOUR, 70, True, 12)]
    for n, nflav, variant, nconf, stubs, seed in cases:
        announce("static forward n=%d nflav=%d variant=%d nconf=%d stubs=%s" % (n, nflav, variant, nconf, stubs))
        nmat = nflav if variant == B.FLAVOUR else 1
        G, st = _inputs(seed, nconf, n, nmat, stubs)
        s_static = _static(B, torch, G, st, n, nflav, variant)
        s_batched = _batched(B, torch, G, st, n, nflav, variant)
        assert np.all(np.isfinite(s_static))
        assert np.array_equal(s_static, s_batched), np.abs(s_static - s_batched).max()
        for c in (0, nconf // 2, nconf - 1):
            Ga = G[c, 0] if variant == B.UNIFORM else G[c]
            sc = None if st is None else st[c]
            ref = oracle_mod.dp(Ga, nflav, variant, sc)
            sa = oracle_mod.dp(np.abs(Ga), nflav, variant, None if sc is None else -np.abs(sc), 1.0)
            assert abs(s_static[c] - ref) <= max(1e-10 * abs(ref), 8 * n * (n + 2) * EPS * sa), (c, s_static[c], ref)


def test_static_graph_replay():
    import torch
    from paper_2507_12349_amd import _binding as B
    announce("static forward captured in a graph, replayed 3 times")
    dev = torch.device("cuda:0")
    n, nflav, nconf = 7, 2, 130
    G, st = _inputs(13, nconf, n, 2, True)
    Gd = torch.as_tensor(G.reshape(-1), device=dev)
    sd = torch.as_tensor(st, device=dev)
    ref = _batched(B, torch, G, st, n, nflav, B.FLAVOUR)
    out = torch.full((nconf,), float("nan"), dtype=torch.float64, device=dev)
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cs):
        B.connected_sum_static(Gd, n, nflav, B.FLAVOUR, sd, -1.0, out, cs)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=cs):
        B.connected_sum_static(Gd, n, nflav, B.FLAVOUR, sd, -1.0, out, cs)
    for _ in range(3):
        out.fill_(float("nan"))
        # other work on the static workspace between replays
        _static(B, torch, *_inputs(14, 40, 5, 1, False), 5, 2, B.UNIFORM)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref)


def test_static_rejects_oversized_calls():
    import torch
    from paper_2507_12349_amd import _binding as B
    announce("static forward: argument and size checks")
    dev = torch.device("cuda:0")
    out = torch.empty(4, dtype=torch.float64, device=dev)
    G = torch.zeros(4 * 16 * 8 * 8, dtype=torch.float64, device=dev)
    # order beyond the static state tables
    with pytest.raises(B.CosError) as e:
        B.connected_sum_static(torch.zeros(4 * 81, dtype=torch.float64, device=dev), 9, 2, B.UNIFORM, None, -1.0,
                               out)
    assert e.value.status == -2
    # order 8 with 16 flavour slots: one group's level windows alone exceed the scratch
    with pytest.raises(B.CosError) as e:
        B.connected_sum_static(G, 8, 16, B.FLAVOUR, None, -1.0, out)
    assert e.value.status == -2 and "static scratch" in str(e.value)
    # flags other than the shift weights
    assert B.lib.cos_connected_sum_static(4, 8, 2, B.FLAVOUR, B.F_SUBLATTICE, B._ptr(G), None, -1.0, B._ptr(out),
                                          None) == -1
