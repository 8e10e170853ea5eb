"""The two-segment reverse sweep (cos_batch_set_adjoint_segments): only the
upper levels are stored by the forward, the lower ones are computed again
after the upper levels' reverse.  Same sums bit for bit and the same
gradients up to the summation order of their accumulation as the sweep that
stores every level; about 40% less workspace per group; chosen automatically
when storing every level would split the groups into chunks."""
import time

import numpy as np
import pytest

from gpu_util import announce

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def _run(B, torch, G, st, n, nflav, variant, segments, w=-1.0, limit=0):
    nconf = st.shape[0] if st is not None else G.numel() // ((nflav if variant else 1) * n * n)
    B.set_workspace_limit(limit)
    b = B.Batch(np.full(nconf, n, dtype=np.int32), nflav, variant, stubs=st is not None)
    B.set_workspace_limit(0)
    b.set_adjoint_segments(segments)
    dev = G.device
    out = torch.empty(nconf, dtype=torch.float64, device=dev)
    Gb = torch.empty_like(G)
    sb = None if st is None else torch.empty_like(st)
    ob = torch.linspace(0.5, 1.5, nconf, dtype=torch.float64, device=dev)
    b.adjoint(G, None, st, w, ob, out, Gb, sb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        b.adjoint(G, None, st, w, ob, out, Gb, sb)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / 3 * 1e3
    plan = b.adjoint_plan(n)
    b.close()
    return out.cpu().numpy(), Gb.cpu().numpy(), None if sb is None else sb.cpu().numpy(), plan, ms


@pytest.mark.parametrize("n,nflav,variant,stubs,nconf", [(6, 2, 0, False, 100), (8, 4, 0, True, 150),
                                                         (9, 3, 1, True, 70), (12, 4, 0, False, 512)])
def test_two_segments_match_stored_levels(n, nflav, variant, stubs, nconf):
    import torch
    from paper_2507_12349_amd import _binding as B
    announce("reverse sweep, two segments vs every level stored: n=%d nflav=%d variant=%d stubs=%s nconf=%d"
             % (n, nflav, variant, stubs, nconf))
    rng = np.random.default_rng(500 + n)
    nmat = nflav if variant else 1
    G = torch.as_tensor(rng.normal(size=nconf * nmat * n * n) * 0.3, device="cuda:0")
    st = torch.as_tensor(rng.normal(size=(nconf, nmat)) * 0.2, device="cuda:0") if stubs else None
    S1, g1, s1, p1, ms1 = _run(B, torch, G, st, n, nflav, variant, 1)
    S2, g2, s2, p2, ms2 = _run(B, torch, G, st, n, nflav, variant, 2)
    # the same sweep on |G|, |sigma|, w = +1 bounds the rounding of the gradients
    Ga = G.abs()
    _, ga, sa, _, _ = _run(B, torch, Ga, None if st is None else -st.abs(), n, nflav, variant, 1, w=1.0)
    print("  every level stored: %.1f MB per group, %.2f ms; two segments (split at level %d): %.1f MB per "
          "group, %.2f ms" % (p1["bytes_per_group"] / 1e6, ms1, p2["split_level"], p2["bytes_per_group"] / 1e6, ms2),
          flush=True)
    assert p1["split_level"] == 0 and p2["split_level"] > 0
    assert p2["bytes_per_group"] < 0.75 * p1["bytes_per_group"]
    assert np.array_equal(S1, S2)
    bound = 2 * 8 * n * (n + 2) * EPS * np.abs(ga)
    assert np.all(np.abs(g1 - g2) <= bound + 1e-300)
    if stubs:
        assert np.all(np.abs(s1 - s2) <= 2 * 8 * n * (n + 2) * EPS * np.abs(sa) + 1e-300)


def test_automatic_choice_when_memory_bound():
    """A workspace bound that lets the stored-levels sweep hold only part of
    the groups at once makes the automatic setting take two segments; sums
    and gradients as before."""
    import torch
    from paper_2507_12349_amd import _binding as B
    announce("reverse sweep: automatic two segments under a workspace bound")
    n, nflav, nconf = 8, 2, 256
    rng = np.random.default_rng(808)
    G = torch.as_tensor(rng.normal(size=nconf * n * n) * 0.3, device="cuda:0")
    S1, g1, _, p1, _ = _run(B, torch, G, None, n, nflav, 0, 1)
    limit = int(1.5 * p1["bytes_per_group"])   # stores every level of one group at a time
    S0, g0, _, p0, _ = _run(B, torch, G, None, n, nflav, 0, 0, limit=limit)
    print("  bound %.1f MB: split level %d, %d groups per chunk" % (limit / 1e6, p0["split_level"],
                                                                    p0["groups_per_chunk"]), flush=True)
    assert p0["split_level"] > 0 and p0["groups_per_chunk"] >= 2
    assert np.array_equal(S0, S1)
    assert np.allclose(g0, g1, rtol=0, atol=1e-12 * np.abs(g1).max())
