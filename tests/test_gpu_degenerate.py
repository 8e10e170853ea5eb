"""Degenerate inputs on the GPU, with exact answers: zero propagators, and
identity propagators (only self-loops, which join no two vertices)."""
import numpy as np
import pytest

from gpu_util import announce, gpu_forward

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nflav,variant", [(4, 0), (3, 1)])
def test_zero_propagators_give_zero(nflav, variant):
    announce("zero propagators nflav=%d variant=%d" % (nflav, variant))
    nmat = nflav if variant else 1
    orders = [1, 2, 5, 9, 12] + [7] * 65
    S = gpu_forward([np.zeros((nmat, k, k)) for k in orders], nflav, variant)
    assert np.all(S == 0.0), S


@pytest.mark.parametrize("nflav,variant", [(4, 0), (2, 1)])
def test_identity_propagators(nflav, variant):
    """G = 1: every cycle is a self-loop on one point.  For n >= 2 nothing joins
    two vertices, so S = 0 exactly; for n = 1 the two points either loop each
    on their own (w N)^2 or form one 2-cycle w N: S = N^2 - N with w = -1 (for
    flavour matrices N counts the flavours the same way)."""
    announce("identity propagators nflav=%d variant=%d" % (nflav, variant))
    nmat = nflav if variant else 1
    orders = [1, 2, 3, 6, 10] + [1] * 64
    S = gpu_forward([np.broadcast_to(np.eye(k), (nmat, k, k)).copy() for k in orders], nflav, variant)
    for k, s in zip(orders, S):
        assert s == (float(nflav * nflav - nflav) if k == 1 else 0.0), (k, s)
