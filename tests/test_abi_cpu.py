"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function the public header declares, plans the state space exactly, and
rejects bad arguments before touching a device."""
import ctypes
import json
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "libcos.h")


@pytest.fixture(scope="module")
def B():
    from paper_2507_12349_amd import _binding
    return _binding


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cos_[a-z_0-9]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported(B):
    names = _declared()
    assert len(names) >= 10
    for name in names:
        assert hasattr(B.lib, name), name
    assert sorted(B.EXPORTED) == names


@pytest.mark.parametrize("n", range(1, 13))
def test_plan_counts_match_golden(B, n):
    with open(os.path.join(ROOT, "tests", "golden", "plan_counts.json")) as f:
        g = json.load(f)["counts"][str(n)]
    c = B.plan_counts(n)
    assert (c["states"], c["ext"], c["closes"], c["stub_edges"], c["masks"]) == \
        (g["states"], g["ext"], g["closes"], g["stub_edges"], g["masks"])
    # rows: one per (mask, head); head 0 for every mask, head h >= 1 when m_0 = m_h = 2
    assert c["rows"] == 2 * 3 ** (n - 1) + (n - 1) * 3 ** max(n - 2, 0) * (1 if n >= 2 else 0)


@pytest.mark.parametrize("n", range(1, 7))
def test_sublattice_plan_counts_match_oracle(B, n):
    """The labelled state space the library plans (closed-form rows and current
    slots) against the oracle's breadth-first enumeration."""
    from oracle import sublattice
    c = B.plan_counts_sublattice(n)
    o = sublattice.plan_counts(n)
    assert (c["states"], c["ext"], c["closes"], c["masks"], c["rows"]) == \
        (o["states"], o["ext"], o["closes"], o["masks"], o["rows"])


@pytest.mark.parametrize("n,labelled", [(k, False) for k in range(1, 8)] + [(k, True) for k in range(1, 6)])
def test_mask_only_plan_counts_match_oracle(B, n, labelled):
    """The slots the level kernels visit in mask-only mode (rows with the
    plane of head vertex 0 fixed by its mask digit, closed-form current slots)
    are exactly the states of Alg. 1's DP reachable from its start, found by
    the oracle's breadth-first search."""
    from oracle import maskonly
    assert B.plan_counts_mask_only(n, labelled) == maskonly.plan_counts(n, labelled)


def _st(B, code):
    return B.lib.cos_status_string(code).decode()


def test_argument_validation_without_device(B):
    lib = B.lib
    v = ctypes.c_int64()
    assert lib.cos_plan_counts(0, ctypes.byref(v), None, None, None, None, None) == -2
    assert lib.cos_plan_counts(13, ctypes.byref(v), None, None, None, None, None) == -2
    h = ctypes.c_void_p()
    n = np.array([4, 5], dtype=np.int32)
    assert lib.cos_batch_create(0, n.ctypes.data, 2, 0, 0, ctypes.byref(h)) == -1
    assert lib.cos_batch_create(2, None, 2, 0, 0, ctypes.byref(h)) == -1
    assert lib.cos_batch_create(2, n.ctypes.data, 2, 0, 0, None) == -1
    assert lib.cos_batch_create(2, n.ctypes.data, 0, 0, 0, ctypes.byref(h)) == -2
    assert lib.cos_batch_create(2, n.ctypes.data, 17, 0, 0, ctypes.byref(h)) == -2
    assert lib.cos_batch_create(2, n.ctypes.data, 2, 7, 0, ctypes.byref(h)) == -1
    assert lib.cos_batch_create(2, n.ctypes.data, 2, 0, 16, ctypes.byref(h)) == -1
    assert lib.cos_batch_create(2, n.ctypes.data, 2, 0, 10, ctypes.byref(h)) == -1  # deterministic + labels
    assert lib.cos_batch_create(2, n.ctypes.data, 2, 0, 3, ctypes.byref(h)) == -1   # shifts with sublattices
    big = np.array([4, 9], dtype=np.int32)
    assert lib.cos_batch_create(2, big.ctypes.data, 2, 0, 2, ctypes.byref(h)) == -2  # above the sublattice max
    assert lib.cos_plan_counts_sublattice(9, None, None, None, None, None) == -2
    # mask-only: two spin blocks (COS_FLAVOUR, nflav = 2), no shifts
    assert lib.cos_batch_create(2, n.ctypes.data, 2, 0, 4, ctypes.byref(h)) == -1   # uniform variant
    assert lib.cos_batch_create(2, n.ctypes.data, 3, 1, 4, ctypes.byref(h)) == -1   # three flavours
    assert lib.cos_batch_create(2, n.ctypes.data, 2, 1, 5, ctypes.byref(h)) == -1   # with shifts
    assert lib.cos_batch_create(2, n.ctypes.data, 2, 1, 20, ctypes.byref(h)) == -1  # unknown flag
    assert lib.cos_plan_counts_mask_only(13, 0, None, None, None) == -2
    assert lib.cos_plan_counts_mask_only(9, 2, None, None, None) == -2
    assert lib.cos_plan_counts_mask_only(4, 1, None, None, None) == -1
    bad = np.array([4, 13], dtype=np.int32)
    assert lib.cos_batch_create(2, bad.ctypes.data, 2, 0, 0, ctypes.byref(h)) == -2
    assert "n[1] = 13" in lib.cos_last_error().decode()
    G = np.eye(3)
    out = ctypes.c_double()
    assert lib.cos_connected_sum(3, 2, 0, 0, None, None, -1.0, ctypes.byref(out)) == -1
    assert lib.cos_connected_sum(3, 2, 0, 1, G.ctypes.data, None, -1.0, ctypes.byref(out)) == -1
    assert lib.cos_connected_sum(0, 2, 0, 0, G.ctypes.data, None, -1.0, ctypes.byref(out)) == -2
    assert lib.cos_connected_sum_batched(None, None, None, None, -1.0, None, None) == -1
    assert lib.cos_build_g0(1, 1, 1, 1, 1, 0, 1.0, 1.0, 1, G.ctypes.data, G.ctypes.data, 1, 1, None, None) == -2
    assert lib.cos_chain_mu_shift(0, None, 1, None, None, None, None, 1, 1.0, None, None, None) == -1
    assert lib.cos_batch_autotune(None, None, None, None, -1.0, None, None, None, None, None) == -1
    i1, i2, i3 = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    assert lib.cos_batch_launch_shape(None, 10, ctypes.byref(i1), ctypes.byref(i2), ctypes.byref(i3)) == -1
    assert lib.cos_batch_timing_enable(None, 1) == -1
    ms = (ctypes.c_double * 4)()
    assert lib.cos_batch_timing_read(None, ms, None) == -1
    # the allocation-free forward: every argument checked before the device is touched
    st = lib.cos_connected_sum_static
    assert st(0, 4, 2, 0, 0, G.ctypes.data, None, -1.0, G.ctypes.data, None) == -1      # nconf
    assert st(4, 9, 2, 0, 0, G.ctypes.data, None, -1.0, G.ctypes.data, None) == -2      # above its orders
    assert st(4, 0, 2, 0, 0, G.ctypes.data, None, -1.0, G.ctypes.data, None) == -2
    assert st(4, 4, 0, 0, 0, G.ctypes.data, None, -1.0, G.ctypes.data, None) == -2      # nflav
    assert st(4, 4, 2, 2, 0, G.ctypes.data, None, -1.0, G.ctypes.data, None) == -1      # variant
    assert st(4, 4, 2, 1, 2, G.ctypes.data, None, -1.0, G.ctypes.data, None) == -1      # sublattice flag
    assert st(4, 4, 2, 1, 1, G.ctypes.data, None, -1.0, G.ctypes.data, None) == -1      # shifts without weights
    assert st(4, 4, 2, 1, 0, None, None, -1.0, G.ctypes.data, None) == -1
    assert "orders 1..8" in (st(4, 9, 2, 0, 0, G.ctypes.data, None, -1.0, G.ctypes.data, None),
                             lib.cos_last_error().decode())[1]
    # integer counting mode
    c64 = ctypes.c_int64()
    assert lib.cos_connected_count(0, 1, ctypes.byref(c64)) == -2
    assert lib.cos_connected_count(13, 1, ctypes.byref(c64)) == -2
    assert lib.cos_connected_count(4, 1, None) == -1
    # failure injection: kinds 0 (device allocation) and 1 (kernel launch) only
    assert lib.cos_inject_failures(2, 0, 1) == -1
    assert lib.cos_inject_failures(0, -1, 1) == -1
    assert lib.cos_inject_failures(1, 0, -1) == -1
    assert lib.cos_inject_failures(0, 0, 0) == 0 and lib.cos_inject_failures(1, 0, 0) == 0
    assert _st(B, 0) == "ok" and _st(B, -2) == "argument out of range"


def test_binding_raises_typed_errors(B):
    with pytest.raises(B.CosError) as e:
        B.plan_counts(20)
    assert e.value.status == -2


def test_no_gpu_reports_unsupported(B):
    """Without a usable gfx950 device the library says so instead of computing
    anything elsewhere (skipped where a GPU is present)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(B.CosError) as e:
        B.connected_sum_host(np.eye(3), 2)
    assert e.value.status in (-5, -4)


def test_release_without_handles(B):
    """No handle alive: cos_release frees the cached tables (none on a device
    here) and the next call rebuilds them with the same counts."""
    before = B.plan_counts(7)
    assert B.lib.cos_release() == 0
    assert B.plan_counts(7) == before


def test_device_buffer_check_rejects_host_and_mistyped_buffers(B):
    """The binding's pre-launch check of a device buffer (host logic): host
    tensors and arrays, other dtypes, strided views and short buffers are
    rejected; an absent optional buffer passes."""
    import torch
    B._device_buffer(None, "x", torch.float64, 10)
    with pytest.raises(TypeError):
        B._device_buffer(torch.zeros(10, dtype=torch.float64), "x", torch.float64, 10)   # host memory
    with pytest.raises(TypeError):
        B._device_buffer(np.zeros(10), "x", torch.float64, 10)
    with pytest.raises(TypeError):
        B._device_buffer(object(), "x", torch.float64, 1)


def test_workspace_limit_arguments(B):
    """Host-side argument check of the workspace bound (no device needed)."""
    with pytest.raises(B.CosError):
        B.set_workspace_limit(-1)
    B.set_workspace_limit(1 << 30)
    B.set_workspace_limit(0)   # back to the default
