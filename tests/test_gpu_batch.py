"""Batching: the plain one-configuration-per-launch form and the batched
persistent form agree bit for bit; an uneven batch equals its per-order
pieces; a captured HIP graph replays with new inputs like eager calls."""
import numpy as np
import pytest

from gpu_util import announce, pack

pytestmark = pytest.mark.gpu


def _dev(x):
    import torch
    return torch.as_tensor(x, device="cuda:0")


def test_plain_equals_batched():
    import torch
    from paper_2507_12349_amd import _binding as B
    from paper_2507_12349_amd.workloads import draw
    from gpu_util import gpu_workload
    announce("plain vs batched, 64 configs of the adjoint workload")
    d = draw("adjoint", nconf=64)
    res = gpu_workload(d)
    G = _dev(res["G"])
    out = torch.full((64,), float("nan"), dtype=torch.float64, device="cuda:0")
    one = B.Batch([10], 4, 0)
    for c in range(64):
        a = int(res["Goff"][c])
        one.forward(G[a:a + 100], None, None, -1.0, out[c:c + 1])
    torch.cuda.synchronize()
    one.close()
    assert np.array_equal(out.cpu().numpy(), res["S"])


def test_uneven_equals_per_order():
    import torch
    from paper_2507_12349_amd import _binding as B
    announce("uneven batch vs per-order batches")
    rng = np.random.default_rng(3)
    orders = [5, 9, 3, 9, 7, 5, 11, 3]
    mats = [rng.normal(size=(2, n, n)) * 0.6 for n in orders]
    sts = rng.normal(size=(len(orders), 2)) * 0.1
    flat, off, n = pack(mats)
    b = B.Batch(n, 2, 1, stubs=True)
    out = torch.full((len(orders),), float("nan"), dtype=torch.float64, device="cuda:0")
    b.forward(_dev(flat), _dev(off), _dev(sts), -1.0, out)
    whole = out.cpu().numpy()
    for k in sorted(set(orders)):
        sel = [i for i, x in enumerate(orders) if x == k]
        f2, o2, n2 = pack([mats[i] for i in sel])
        b2 = B.Batch(n2, 2, 1, stubs=True)
        o = torch.full((len(sel),), float("nan"), dtype=torch.float64, device="cuda:0")
        b2.forward(_dev(f2), _dev(o2), _dev(np.ascontiguousarray(sts[sel])), -1.0, o)
        assert np.array_equal(o.cpu().numpy(), whole[sel]), k
        b2.close()
    b.close()


def test_graph_replay_with_new_inputs():
    """Capture the batched call on a stream; replay it three times, writing new
    matrices into the captured input buffer between replays (eager work and a
    synchronisation between replays), and compare each replay with an eager
    call on the same inputs."""
    import torch
    from paper_2507_12349_amd import _binding as B
    announce("graph capture / replay")
    rng = np.random.default_rng(4)
    nconf, n = 96, 8
    b = B.Batch([n] * nconf, 4, 0)
    G = torch.empty(nconf * n * n, dtype=torch.float64, device="cuda:0")
    out = torch.zeros(nconf, dtype=torch.float64, device="cuda:0")
    G.copy_(_dev(rng.normal(size=nconf * n * n) * 0.4))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.forward(G, None, None, -1.0, out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.forward(G, None, None, -1.0, out)
    ref_out = torch.zeros_like(out)
    for k in range(3):
        G.copy_(_dev(rng.normal(size=nconf * n * n) * 0.4))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = out.clone()
        b.forward(G, None, None, -1.0, ref_out)
        torch.cuda.synchronize()
        assert torch.equal(got, ref_out), k
    b.close()


def test_graph_replay_forward_uneven_side_stream():
    """An uneven batch of five orders runs the four after the largest on the
    batch's side stream (a fork from the caller's stream and a join back).
    Capture the batched forward in a graph, replay it three times with new
    matrices (eager work and a synchronisation between replays), and compare
    every replay with an eager call and with one batch per order, bitwise."""
    import torch
    from paper_2507_12349_amd import _binding as B
    announce("graph capture / replay of an uneven forward with a side stream (5 orders)")
    rng = np.random.default_rng(41)
    orders = [10, 4, 8, 6, 10, 5, 8, 4, 6] * 8
    nconf = len(orders)
    flat, off, n = pack([rng.normal(size=(3, k, k)) * 0.5 for k in orders])
    b = B.Batch(n, 3, 1, stubs=False)
    G = _dev(flat).clone()
    Goff = _dev(off)
    out = torch.zeros(nconf, dtype=torch.float64, device="cuda:0")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.forward(G, Goff, None, -1.0, out, s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        b.forward(G, Goff, None, -1.0, out, s)
    ref = torch.zeros_like(out)
    for k in range(3):
        mats = [rng.normal(size=(3, x, x)) * 0.5 for x in orders]
        G.copy_(_dev(pack(mats)[0]))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = out.clone()
        b.forward(G, Goff, None, -1.0, ref)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), k
        whole = got.cpu().numpy()
        for m in sorted(set(orders)):
            sel = [i for i, x in enumerate(orders) if x == m]
            f2, o2, n2 = pack([mats[i] for i in sel])
            b2 = B.Batch(n2, 3, 1)
            o = torch.full((len(sel),), float("nan"), dtype=torch.float64, device="cuda:0")
            b2.forward(_dev(f2), _dev(o2), None, -1.0, o)
            assert np.array_equal(o.cpu().numpy(), whole[sel]), (k, m)
            b2.close()
    b.close()


def test_graph_replay_adjoint_uneven():
    """The adjoint of an uneven batch (orders 5, 7, 9; three flavours with
    shifts) captured once and replayed with new inputs: S equals an eager call
    bit for bit, the gradients to rounding (their accumulation order varies)."""
    import torch
    from paper_2507_12349_amd import _binding as B
    announce("graph capture / replay of the adjoint, uneven orders")
    rng = np.random.default_rng(9)
    orders = [9, 5, 7, 9, 5, 7, 7]
    mats = [rng.normal(size=(3, k, k)) * 0.5 for k in orders]
    flat, off, n = pack(mats)
    b = B.Batch(n, 3, 1, stubs=True)
    G, Goff = _dev(flat), _dev(off)
    st = _dev(rng.normal(size=(len(orders), 3)) * 0.2)
    ob = _dev(rng.normal(size=len(orders)))
    S, Gb, sb = torch.zeros(len(orders), dtype=torch.float64, device="cuda:0"), torch.zeros_like(G), torch.zeros_like(st)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.adjoint(G, Goff, st, -1.0, ob, S, Gb, sb)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.adjoint(G, Goff, st, -1.0, ob, S, Gb, sb)
    rS, rGb, rsb = torch.zeros_like(S), torch.zeros_like(Gb), torch.zeros_like(sb)
    for k in range(3):
        G.copy_(_dev(np.concatenate([(rng.normal(size=m.shape) * 0.5).reshape(-1) for m in mats])))
        st.copy_(_dev(rng.normal(size=(len(orders), 3)) * 0.2))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        gS, gGb, gsb = S.clone(), Gb.clone(), sb.clone()
        b.adjoint(G, Goff, st, -1.0, ob, rS, rGb, rsb)
        torch.cuda.synchronize()
        assert torch.equal(gS, rS), k
        assert torch.allclose(gGb, rGb, rtol=1e-12, atol=1e-14 * float(rGb.abs().max())), k
        assert torch.allclose(gsb, rsb, rtol=1e-12, atol=1e-14 * float(rsb.abs().max())), k
    b.close()


def test_autograd_function_matches_adjoint():
    import torch
    from paper_2507_12349_amd import _binding as B
    from paper_2507_12349_amd.autograd import ConnectedSum
    from gpu_util import gpu_forward
    announce("autograd ConnectedSum")
    rng = np.random.default_rng(5)
    mats = [rng.normal(size=(1, n, n)) for n in (4, 6, 6)]
    flat, off, n = pack(mats)
    b = B.Batch(n, 3, 0)
    G = _dev(flat).requires_grad_(True)
    S = ConnectedSum.apply(G, None, b, _dev(off), -1.0)
    w = _dev(np.array([0.5, -1.0, 2.0]))
    (S * w).sum().backward()
    S_ref, _, gb, _ = gpu_forward(mats, 3, 0, None, adjoint=True, out_bar=w.cpu().numpy())
    assert np.array_equal(S.detach().cpu().numpy(), S_ref)
    # the gradient accumulators are flushed with atomics: equal up to summation order
    ref = np.concatenate([x.reshape(-1) for x in gb])
    assert np.allclose(G.grad.cpu().numpy(), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    b.close()


def test_phase_timing():
    import torch
    from paper_2507_12349_amd import _binding as B
    announce("phase timing events, 2 adjoint calls + 1 forward, orders 6 and 8")
    rng = np.random.default_rng(11)
    mats = [rng.normal(size=(1, n, n)) * 0.5 for n in (6, 8, 6, 8, 8)]
    flat, off, n = pack(mats)
    b = B.Batch(n, 2, 0)
    G, Goff = _dev(flat), _dev(off)
    out = torch.empty(len(mats), dtype=torch.float64, device="cuda:0")
    Gb = torch.empty_like(G)
    b.timing(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(2):
        b.adjoint(G, Goff, None, -1.0, torch.ones_like(out), out, Gb, None)
    b.forward(G, Goff, None, -1.0, out)
    e1.record()
    ms, calls = b.timing_read()
    torch.cuda.synchronize()
    assert calls == 3
    assert all(v >= 0.0 for v in ms.values())
    assert ms["forward"] > 0.0 and ms["reverse"] > 0.0 and ms["pack"] > 0.0 and ms["unpack"] > 0.0
    # the phases cover the calls: their sum cannot exceed the bracketing events
    assert sum(ms.values()) <= e0.elapsed_time(e1) * 1.01 + 0.05
    ms2, calls2 = b.timing_read()
    assert calls2 == 0 and sum(ms2.values()) == 0.0
    b.timing(False)
    b.close()


def test_autotune_keeps_results():
    """The autotuner picks a launch shape per order; S is bitwise the same under
    every shape, gradients agree to rounding (their accumulation order varies)."""
    import torch
    from paper_2507_12349_amd import _binding as B
    announce("autotune, orders 4, 7, 9 with 3 flavours and shifts")
    rng = np.random.default_rng(21)
    orders = [9, 4, 7, 9, 4, 7, 9]
    mats = [rng.normal(size=(3, n, n)) * 0.5 for n in orders]
    sts = rng.normal(size=(len(orders), 3)) * 0.2
    flat, off, n = pack(mats)
    G, Goff, st = _dev(flat), _dev(off), _dev(sts)
    b = B.Batch(n, 3, 1, stubs=True)
    S0 = torch.empty(len(orders), dtype=torch.float64, device="cuda:0")
    ob = _dev(rng.normal(size=len(orders)))
    Gb0, sb0 = torch.empty_like(G), torch.empty_like(st)
    b.adjoint(G, Goff, st, -1.0, ob, S0, Gb0, sb0)
    S1 = torch.full_like(S0, float("nan"))
    b.autotune(G, Goff, st, -1.0, S1, ob, torch.empty_like(G), torch.empty_like(st))
    shapes = {k: b.launch_shape(k) for k in (4, 7, 9)}
    for k, sh in shapes.items():
        assert sh["fwd_waves"] in (4, 8, 16) and sh["fwd_masks"] in (1, 2, 4, 8, 16), sh
        assert sh["adj_masks"] in (2, 4, 6, 8, 12, 16, 24, 32, 48, 64), sh
    with pytest.raises(B.CosError):
        b.launch_shape(5)
    S2 = torch.full_like(S0, float("nan"))
    b.forward(G, Goff, st, -1.0, S2)
    Gb2, sb2 = torch.empty_like(G), torch.empty_like(st)
    S3 = torch.full_like(S0, float("nan"))
    b.adjoint(G, Goff, st, -1.0, ob, S3, Gb2, sb2)
    torch.cuda.synchronize()
    assert torch.equal(S0, S1) and torch.equal(S0, S2) and torch.equal(S0, S3)
    assert torch.allclose(Gb2, Gb0, rtol=1e-12, atol=1e-14 * float(Gb0.abs().max()))
    assert torch.allclose(sb2, sb0, rtol=1e-12, atol=1e-14 * float(sb0.abs().max()))
    b.close()


def test_many_flavours_fit_lds():
    """16 flavours at n = 10: the forward's per-mask close sums of every flavour
    sit in LDS beside G; the launch shape must shrink to fit.  Equal matrices
    in every flavour reproduce the uniform variant."""
    import torch
    from paper_2507_12349_amd import _binding as B
    announce("16 flavours at n=10 (flavour variant) vs uniform")
    rng = np.random.default_rng(31)
    M = rng.normal(size=(10, 10)) * 0.4
    bf = B.Batch([10], 16, 1)
    bu = B.Batch([10], 16, 0)
    Sf = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda:0")
    Su = torch.full_like(Sf, float("nan"))
    bf.forward(_dev(np.tile(M, (16, 1, 1)).reshape(-1)), None, None, -1.0, Sf)
    bu.forward(_dev(M.reshape(-1)), None, None, -1.0, Su)
    Sa = torch.full_like(Sf, float("nan"))   # the same sum over absolute values
    bu.forward(_dev(np.abs(M).reshape(-1)), None, None, 1.0, Sa)
    torch.cuda.synchronize()
    sf, su, sa = float(Sf[0]), float(Su[0]), float(Sa[0])
    eps = np.finfo(np.float64).eps
    assert np.isfinite(sf) and abs(sf - su) <= 2 * 8 * 10 * 12 * eps * sa, (sf, su, sa)
    bf.close()
    bu.close()


def test_set_launch_shape_keeps_sums():
    """Every launch shape gives the same S bit for bit (each state is written
    once, every sum in a fixed order); out-of-range shapes are rejected."""
    import torch
    from paper_2507_12349_amd import _binding as B
    announce("explicit launch shapes, orders 5 and 9, three flavours")
    rng = np.random.default_rng(23)
    mats = [rng.normal(size=(3, n, n)) * 0.5 for n in [5] * 70 + [9] * 3]
    flat, off, n = pack(mats)
    G, Goff = _dev(flat), _dev(off)
    b = B.Batch(n, 3, 1)
    ref = torch.empty(len(mats), dtype=torch.float64, device="cuda:0")
    b.forward(G, Goff, None, -1.0, ref)
    for waves, masks in ((1, 1), (4, 16), (8, 2), (16, 4), (12, 3)):
        for k in (5, 9):
            b.set_launch_shape(k, waves, masks, 4)
            assert b.launch_shape(k)["fwd_waves"] == waves
        out = torch.full_like(ref, float("nan"))
        b.forward(G, Goff, None, -1.0, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (waves, masks)
    for bad in ((0, 4, 4), (17, 4, 4), (8, 0, 4), (8, 17, 4), (8, 4, 65)):
        with pytest.raises(B.CosError):
            b.set_launch_shape(5, *bad)
    with pytest.raises(B.CosError):
        b.set_launch_shape(6, 8, 4, 4)
    b.close()


def test_graph_replay_of_the_whole_step():
    """The benchmark's step (propagators with dG/dxi, adjoint call, chain rule
    to mu and the shift) captured once; three replays, each after new vertex
    times are written into the captured buffer (eager work and a
    synchronisation between replays), against the same step run eagerly:
    propagators and S bit for bit, the gradients to rounding."""
    import torch
    from paper_2507_12349_amd import _binding as B
    from paper_2507_12349_amd.autograd import Geometry
    from paper_2507_12349_amd.workloads import draw
    announce("graph capture / replay of propagators + adjoint + chain rule (130 x n=8)")
    dd = draw("adjoint", nconf=130).prefix(np.full(130, 8))   # the first 8 vertices of each configuration
    w = dd.workload
    dev = torch.device("cuda:0")
    geo = Geometry(dd, 1, dev)
    mu, alpha = np.array(w.mu[:1]), np.zeros(1)
    nconf = geo.nconf
    G, dG, Gb = (torch.zeros(geo.total, dtype=torch.float64, device=dev) for _ in range(3))
    stub = torch.zeros((nconf, 1), dtype=torch.float64, device=dev)
    sb, S = torch.zeros_like(stub), torch.zeros(nconf, dtype=torch.float64, device=dev)
    ob = torch.ones(nconf, dtype=torch.float64, device=dev)
    mub, alb = torch.zeros(nconf, dtype=torch.float64, device=dev), torch.zeros(nconf, dtype=torch.float64, device=dev)
    b = B.Batch(dd.n, 4, 0, stubs=True)

    def step(st):
        B.build_g0(nconf, geo.n, geo.voff, geo.sites, geo.tau, w.L, w.t, w.beta, mu, alpha, geo.Goff, G, dG, st)
        b.adjoint(G, geo.Goff, stub, -1.0, ob, S, Gb, sb, st)
        B.chain_mu_shift(nconf, geo.n, 1, geo.Goff, Gb, dG, sb, 1, 1.0, mub, alb, st)

    try:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            step(s)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            step(s)
        rng = np.random.default_rng(17)
        main = torch.cuda.current_stream()
        for k in range(3):
            geo.tau.copy_(torch.as_tensor(rng.uniform(0.0, w.beta, size=geo.tau.numel()), device=dev))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            got = [x.clone() for x in (G, S, Gb, mub, alb)]
            step(main)
            torch.cuda.synchronize()
            assert torch.equal(got[0], G) and torch.equal(got[1], S), k
            for a, r in zip(got[2:], (Gb, mub, alb)):
                assert torch.allclose(a, r, rtol=1e-12, atol=1e-13 * float(r.abs().max())), k
            assert float(S.abs().max()) > 0.0
    finally:
        b.close()


def test_chunked_groups_match_one_launch():
    """A batch planned under a tiny workspace bound runs its groups one chunk
    (one group) at a time, forward and reverse; S equals the default plan (all
    groups in each level launch) bit for bit, the gradients to rounding.
    Orders 7 and 9 mixed (several groups each, ragged tails), three flavours
    with shifts."""
    import torch
    from paper_2507_12349_amd import _binding as B
    announce("chunked groups vs one launch (workspace bound)")
    rng = np.random.default_rng(21)
    orders = [7] * 150 + [9] * 70
    mats = [rng.normal(size=(3, k, k)) * 0.5 for k in orders]
    flat, off, n = pack(mats)
    G, Goff = _dev(flat), _dev(off)
    st = _dev(rng.normal(size=(len(orders), 3)) * 0.2)
    ob = _dev(rng.normal(size=len(orders)))
    res = []
    try:
        for limit in (1, 0):
            B.set_workspace_limit(limit)
            b = B.Batch(n, 3, 1, stubs=True)
            S1 = torch.full((len(orders),), float("nan"), dtype=torch.float64, device="cuda:0")
            S2, Gb, sb = torch.full_like(S1, float("nan")), torch.full_like(G, float("nan")), torch.full_like(st, float("nan"))
            b.forward(G, Goff, st, -1.0, S1)
            b.adjoint(G, Goff, st, -1.0, ob, S2, Gb, sb)
            torch.cuda.synchronize()
            res.append((S1.clone(), S2.clone(), Gb.clone(), sb.clone()))
            b.close()
    finally:
        B.set_workspace_limit(0)
    (a1, a2, ag, asb), (b1, b2, bg, bsb) = res
    assert torch.equal(a1, b1) and torch.equal(a2, b2) and torch.equal(a1, a2)
    assert torch.allclose(ag, bg, rtol=1e-12, atol=1e-14 * float(bg.abs().max()))
    assert torch.allclose(asb, bsb, rtol=1e-12, atol=1e-14 * float(bsb.abs().max()))
