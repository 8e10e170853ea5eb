"""ctypes binding of libcos.so (argument marshalling only).

Every computation runs in the HIP kernels of ``csrc/``; this module converts
torch tensors / numpy arrays to pointers and status codes to exceptions.
Importing it without a built ``libcos.so`` raises ImportError: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcos.so")

UNIFORM, FLAVOUR = 0, 1
F_STUBS, F_SUBLATTICE, F_MASK_ONLY, F_DETERMINISTIC = 1, 2, 4, 8
NMAX, FMAX, NMAX_SUBLATTICE = 12, 16, 8

EXPORTED = (
    "cos_batch_create", "cos_batch_destroy", "cos_connected_sum_batched",
    "cos_connected_sum_adjoint", "cos_connected_sum", "cos_build_g0", "cos_chain_mu_shift",
    "cos_plan_counts", "cos_status_string", "cos_last_error", "cos_release",
    "cos_batch_timing_enable", "cos_batch_timing_read", "cos_batch_autotune", "cos_batch_launch_shape",
    "cos_plan_counts_sublattice", "cos_build_g0_honeycomb", "cos_mc_sample", "cos_accumulate_moments", "cos_pade",
    "cos_cdet_workspace", "cos_cdet_su2", "cos_plan_counts_mask_only", "cos_batch_set_launch_shape", "cos_set_workspace_limit",
    "cos_connected_sum_static", "cos_inject_failures", "cos_batch_set_adjoint_segments",
    "cos_batch_adjoint_plan", "cos_connected_count",
)
PHASES = ("pack", "forward", "reverse", "unpack")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libcos.so is not built (%s); run __graft_entry__.build() or "
                          "python paper_2507_12349_amd/csrc/build.py" % LIB_PATH)
    # torch ships its own HIP runtime with the same soname as the system one;
    # loading torch first makes libcos bind to that runtime, so that the
    # library and torch's tensors and streams share one runtime per process
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, d, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    P64 = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "cos_batch_create": ([i32, p, i32, i32, i32, ctypes.POINTER(p)], i32),
        "cos_batch_destroy": ([p], i32),
        "cos_connected_sum_batched": ([p, p, p, p, d, p, p], i32),
        "cos_connected_sum_adjoint": ([p, p, p, p, d, p, p, p, p, p], i32),
        "cos_connected_sum": ([i32, i32, i32, i32, p, p, d, p], i32),
        "cos_build_g0": ([i32, p, p, p, p, i32, d, d, i32, p, p, p, p, p, p], i32),
        "cos_chain_mu_shift": ([i32, p, i32, p, p, p, p, i32, d, p, p, p], i32),
        "cos_plan_counts": ([i32, P64, P64, P64, P64, P64, P64], i32),
        "cos_plan_counts_sublattice": ([i32, P64, P64, P64, P64, P64], i32),
        "cos_plan_counts_mask_only": ([i32, i32, P64, P64, P64], i32),
        "cos_build_g0_honeycomb": ([i32, p, p, p, p, i32, d, d, i32, p, p, p, p, p, p, p], i32),
        "cos_mc_sample": ([i32, i32, i32, d, ctypes.c_uint64, i64, p, p, p], i32),
        "cos_accumulate_moments": ([i32, p, p, p], i32),
        "cos_pade": ([i32, i32, p, d, ctypes.POINTER(d), p], i32),
        "cos_cdet_workspace": ([i32, i32, i32, ctypes.POINTER(ctypes.c_uint64)], i32),
        "cos_cdet_su2": ([i32, i32, p, i32, d, p, ctypes.c_uint64, p, p], i32),
        "cos_status_string": ([i32], ctypes.c_char_p),
        "cos_last_error": ([], ctypes.c_char_p),
        "cos_release": ([], i32),
        "cos_set_workspace_limit": ([i64], i32),
        "cos_batch_timing_enable": ([p, i32], i32),
        "cos_batch_timing_read": ([p, ctypes.POINTER(d), ctypes.POINTER(i32)], i32),
        "cos_batch_autotune": ([p, p, p, p, d, p, p, p, p, p], i32),
        "cos_batch_set_launch_shape": ([p, i32, i32, i32, i32], i32),
        "cos_connected_sum_static": ([i32, i32, i32, i32, i32, p, p, d, p, p], i32),
        "cos_inject_failures": ([i32, i32, i32], i32),
        "cos_connected_count": ([i32, i64, P64], i32),
        "cos_batch_set_adjoint_segments": ([p, i32], i32),
        "cos_batch_adjoint_plan": ([p, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), P64], i32),
        "cos_batch_launch_shape": ([p, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


lib = _load()


class CosError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = "%s: %s (%d): %s" % (where, lib.cos_status_string(status).decode(), status,
                                   lib.cos_last_error().decode())
        super().__init__(msg)


def _check(status: int, where: str):
    if status != 0:
        raise CosError(status, where)


def _ptr(x):
    """Device or host address of a torch tensor / numpy array (None -> NULL)."""
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError("expected a torch tensor or numpy array, got %r" % type(x))


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _device_buffer(x, name, dtype, numel):
    """The kernels address device buffers through raw pointers: a host array,
    another element type, a strided view or a buffer shorter than the call
    reads or writes is rejected here, before anything is launched."""
    if x is None:
        return
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda):
        raise TypeError("%s must be a CUDA tensor, got %r" % (name, type(x)))
    if x.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, x.dtype))
    if not x.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if x.numel() < numel:
        raise ValueError("%s holds %d elements, the call needs at least %d" % (name, x.numel(), numel))


def _geometry_buffers(nconf, n, voff, sites, tau, Goff, G, dG):
    """Buffers of the propagator builders.  Only the per-configuration arrays'
    lengths are known on the host; the vertex and matrix arrays are checked
    for type and layout."""
    import torch
    _device_buffer(n, "n", torch.int32, nconf)
    _device_buffer(voff, "voff", torch.int64, nconf)
    _device_buffer(sites, "sites", torch.int32, 2)
    _device_buffer(tau, "tau", torch.float64, 1)
    _device_buffer(Goff, "Goff", torch.int64, nconf)
    _device_buffer(G, "G", torch.float64, 1)
    _device_buffer(dG, "dG", torch.float64, G.numel())


def set_workspace_limit(nbytes: int):
    """Bound each level workspace of batches planned from now on (0: a share
    of the device memory free when the workspace is made)."""
    _check(lib.cos_set_workspace_limit(int(nbytes)), "cos_set_workspace_limit")


def connected_count(n: int, x: int) -> int:
    """Connected diagrams of order n with unit propagators and integer weight x
    per cycle, counted on the device modulo 2^64 (returned as a signed int)."""
    c = ctypes.c_int64()
    _check(lib.cos_connected_count(int(n), int(x), ctypes.byref(c)), "cos_connected_count")
    return c.value


def inject_failures(kind: int, skip: int, count: int):
    """Make the library's next device allocations (kind 0) or kernel launches
    (kind 1) fail after `skip` successes, `count` times (testing aid)."""
    _check(lib.cos_inject_failures(int(kind), int(skip), int(count)), "cos_inject_failures")


def plan_counts(n: int) -> dict:
    vals = [ctypes.c_int64() for _ in range(6)]
    _check(lib.cos_plan_counts(int(n), *[ctypes.byref(v) for v in vals]), "cos_plan_counts")
    return dict(zip(("states", "ext", "closes", "stub_edges", "masks", "rows"), [v.value for v in vals]))


def plan_counts_sublattice(n: int) -> dict:
    vals = [ctypes.c_int64() for _ in range(5)]
    _check(lib.cos_plan_counts_sublattice(int(n), *[ctypes.byref(v) for v in vals]), "cos_plan_counts_sublattice")
    return dict(zip(("states", "ext", "closes", "masks", "rows"), [v.value for v in vals]))


def plan_counts_mask_only(n: int, sublattice: bool = False) -> dict:
    vals = [ctypes.c_int64() for _ in range(3)]
    _check(lib.cos_plan_counts_mask_only(int(n), F_SUBLATTICE if sublattice else 0,
                                         *[ctypes.byref(v) for v in vals]), "cos_plan_counts_mask_only")
    return dict(zip(("states", "ext", "closes"), [v.value for v in vals]))


def connected_sum_host(G: np.ndarray, nflav: int, variant: int = UNIFORM, stub=None, w: float = -1.0,
                       sublattice: bool = False, mask_only: bool = False) -> float:
    """One configuration from host arrays (the GPU kernel does the work);
    with ``sublattice`` G holds 2n x 2n matrices."""
    G = np.ascontiguousarray(G, dtype=np.float64)
    n = G.shape[-1] // 2 if sublattice else G.shape[-1]
    flags = ((F_STUBS if stub is not None else 0) | (F_SUBLATTICE if sublattice else 0)
             | (F_MASK_ONLY if mask_only else 0))
    st = None if stub is None else np.ascontiguousarray(stub, dtype=np.float64).reshape(-1)
    out = ctypes.c_double()
    _check(lib.cos_connected_sum(n, nflav, variant, flags, _ptr(G), _ptr(st), float(w), ctypes.byref(out)),
           "cos_connected_sum")
    return out.value


STATIC_NMAX = 8
STATIC_SCRATCH_BYTES = 64 << 20


def connected_sum_static(G, n: int, nflav: int, variant: int, stub, w: float, out, stream=None):
    """Forward sums of out.numel() configurations of order n stored back to
    back in G, through the entry point that allocates no device memory (its
    workspace is the library's static device array, shared by every call on a
    device: calls must not overlap)."""
    import torch
    nconf = int(out.numel())
    nmat = int(nflav) if variant == FLAVOUR else 1
    _device_buffer(G, "G", torch.float64, nconf * nmat * int(n) * int(n))
    _device_buffer(stub, "stub", torch.float64, nconf * nmat)
    _device_buffer(out, "out", torch.float64, nconf)
    _check(lib.cos_connected_sum_static(nconf, int(n), int(nflav), int(variant), F_STUBS if stub is not None else 0,
                                        _ptr(G), _ptr(stub), float(w), _ptr(out), _stream(stream)),
           "cos_connected_sum_static")


class Batch:
    """Plan for a batch of configurations with orders ``n`` (host sequence)."""

    def __init__(self, n, nflav: int, variant: int = UNIFORM, stubs: bool = False, sublattice: bool = False,
                 mask_only: bool = False, deterministic: bool = False):
        n = np.ascontiguousarray(np.asarray(n, dtype=np.int32).reshape(-1))
        self.n = n
        self.nconf = int(n.size)
        self.nflav = int(nflav)
        self.variant = int(variant)
        self.stubs = bool(stubs)
        self.sublattice = bool(sublattice)
        self.mask_only = bool(mask_only)
        self.deterministic = bool(deterministic)
        self.nmat = self.nflav if self.variant == FLAVOUR else 1
        self.nstub = self.nmat
        h = ctypes.c_void_p()
        flags = ((F_STUBS if self.stubs else 0) | (F_SUBLATTICE if self.sublattice else 0)
                 | (F_MASK_ONLY if self.mask_only else 0) | (F_DETERMINISTIC if self.deterministic else 0))
        _check(lib.cos_batch_create(self.nconf, _ptr(n), self.nflav, self.variant, flags, ctypes.byref(h)),
               "cos_batch_create")
        self._h = h
        self._total = self.goff()[1]

    def _check_buffers(self, G, Goff, stub, out=None, out_bar=None, G_bar=None, stub_bar=None):
        """Types and sizes of the device buffers of a call.  With explicit
        offsets only their count is checked (reading them would synchronise):
        G must then hold every configuration's matrices at its offset."""
        import torch
        f64 = torch.float64
        if G is None:
            raise ValueError("G is required")
        _device_buffer(G, "G", f64, self._total if Goff is None else 1)
        _device_buffer(Goff, "Goff", torch.int64, self.nconf)
        ns = self.nconf * self.nstub
        _device_buffer(stub if self.stubs else None, "stub", f64, ns)
        _device_buffer(out, "out", f64, self.nconf)
        _device_buffer(out_bar, "out_bar", f64, self.nconf)
        _device_buffer(G_bar, "G_bar", f64, G.numel())   # the layout of G
        _device_buffer(stub_bar if self.stubs else None, "stub_bar", f64, ns)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.cos_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def goff(self):
        """Element offsets of each configuration's matrices (back-to-back layout)."""
        side = self.n.astype(np.int64) * (2 if self.sublattice else 1)
        sizes = self.nmat * side ** 2
        off = np.zeros(self.nconf, dtype=np.int64)
        off[1:] = np.cumsum(sizes[:-1])
        return off, int(sizes.sum())

    def forward(self, G, Goff, stub, w, out, stream=None):
        self._check_buffers(G, Goff, stub, out=out)
        _check(lib.cos_connected_sum_batched(self._h, _ptr(G), _ptr(Goff), _ptr(stub), float(w), _ptr(out),
                                             _stream(stream)), "cos_connected_sum_batched")

    def adjoint(self, G, Goff, stub, w, out_bar, out, G_bar, stub_bar, stream=None):
        self._check_buffers(G, Goff, stub, out=out, out_bar=out_bar, G_bar=G_bar, stub_bar=stub_bar)
        _check(lib.cos_connected_sum_adjoint(self._h, _ptr(G), _ptr(Goff), _ptr(stub), float(w), _ptr(out_bar),
                                             _ptr(out), _ptr(G_bar), _ptr(stub_bar), _stream(stream)),
               "cos_connected_sum_adjoint")


    def autotune(self, G, Goff, stub, w, out, out_bar=None, G_bar=None, stub_bar=None, stream=None):
        """Pick the fastest launch shape per order on these inputs (synchronous);
        with out_bar the reverse sweep is tuned too."""
        self._check_buffers(G, Goff, stub, out=out, out_bar=out_bar, G_bar=G_bar, stub_bar=stub_bar)
        _check(lib.cos_batch_autotune(self._h, _ptr(G), _ptr(Goff), _ptr(stub), float(w), _ptr(out_bar), _ptr(out),
                                      _ptr(G_bar), _ptr(stub_bar), _stream(stream)), "cos_batch_autotune")

    def launch_shape(self, n: int):
        vals = [ctypes.c_int32() for _ in range(3)]
        _check(lib.cos_batch_launch_shape(self._h, int(n), *[ctypes.byref(v) for v in vals]), "cos_batch_launch_shape")
        return dict(zip(("fwd_waves", "fwd_masks", "adj_masks"), [v.value for v in vals]))

    def set_launch_shape(self, n: int, fwd_waves: int, fwd_masks: int, adj_masks: int):
        _check(lib.cos_batch_set_launch_shape(self._h, int(n), int(fwd_waves), int(fwd_masks), int(adj_masks)),
               "cos_batch_set_launch_shape")

    def set_adjoint_segments(self, segments: int):
        """0 automatic, 1 store every forward level, 2 two segments (lower
        levels recomputed; less memory)."""
        _check(lib.cos_batch_set_adjoint_segments(self._h, int(segments)), "cos_batch_set_adjoint_segments")

    def adjoint_plan(self, n: int):
        """Reverse-sweep plan of order n after a reverse call: split level,
        groups per chunk, workspace bytes per group."""
        h, c, nb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib.cos_batch_adjoint_plan(self._h, int(n), ctypes.byref(h), ctypes.byref(c), ctypes.byref(nb)),
               "cos_batch_adjoint_plan")
        return {"split_level": h.value, "groups_per_chunk": c.value, "bytes_per_group": nb.value}

    def timing(self, enable: bool = True):
        """Record HIP events at the phase boundaries of every later call."""
        _check(lib.cos_batch_timing_enable(self._h, 1 if enable else 0), "cos_batch_timing_enable")

    def timing_read(self):
        """Device milliseconds per phase summed over the calls since the last
        read (waits for them), and the number of calls."""
        ms = (ctypes.c_double * len(PHASES))()
        nc = ctypes.c_int32()
        _check(lib.cos_batch_timing_read(self._h, ms, ctypes.byref(nc)), "cos_batch_timing_read")
        return dict(zip(PHASES, list(ms))), nc.value


def build_g0(nconf, n, voff, sites, tau, L, t, beta, mu, alpha, Goff, G, dG=None, stream=None):
    """Device propagator builder; n, voff, sites, tau, Goff, G, dG are device tensors,
    mu and alpha host sequences of length nmat."""
    _geometry_buffers(nconf, n, voff, sites, tau, Goff, G, dG)
    mu = np.ascontiguousarray(np.asarray(mu, dtype=np.float64).reshape(-1))
    alpha = np.ascontiguousarray(np.asarray(alpha, dtype=np.float64).reshape(-1))
    _check(lib.cos_build_g0(int(nconf), _ptr(n), _ptr(voff), _ptr(sites), _ptr(tau), int(L), float(t),
                            float(beta), int(mu.size), _ptr(mu), _ptr(alpha), _ptr(Goff), _ptr(G), _ptr(dG),
                            _stream(stream)), "cos_build_g0")


def build_g0_honeycomb(nconf, n, voff, cells, tau, L, t, beta, mu, alpha, delta, Goff, G, stream=None, dG=None):
    """Device honeycomb propagator builder (2n x 2n matrices, index 2k + s);
    n, voff, cells, tau, Goff, G (and dG = dG/dxi, optional) are device
    tensors, mu, alpha, delta host sequences of length nmat."""
    _geometry_buffers(nconf, n, voff, cells, tau, Goff, G, dG)
    mu = np.ascontiguousarray(np.asarray(mu, dtype=np.float64).reshape(-1))
    alpha = np.ascontiguousarray(np.asarray(alpha, dtype=np.float64).reshape(-1))
    delta = np.ascontiguousarray(np.asarray(delta, dtype=np.float64).reshape(-1))
    _check(lib.cos_build_g0_honeycomb(int(nconf), _ptr(n), _ptr(voff), _ptr(cells), _ptr(tau), int(L), float(t),
                                      float(beta), int(mu.size), _ptr(mu), _ptr(alpha), _ptr(delta), _ptr(Goff),
                                      _ptr(G), _ptr(dG), _stream(stream)), "cos_build_g0_honeycomb")


def mc_sample(nconf, n, L, beta, seed, first, sites, tau, stream=None):
    """Device sampler of vertex configurations (vertex 0 at the origin)."""
    import torch
    _device_buffer(sites, "sites", torch.int32, 2 * int(nconf) * int(n))
    _device_buffer(tau, "tau", torch.float64, int(nconf) * int(n))
    _check(lib.cos_mc_sample(int(nconf), int(n), int(L), float(beta), int(seed) & 0xFFFFFFFFFFFFFFFF, int(first),
                             _ptr(sites), _ptr(tau), _stream(stream)), "cos_mc_sample")


def accumulate_moments(count, x, acc, stream=None):
    """acc[0] += sum x, acc[1] += sum x^2 (device)."""
    import torch
    _device_buffer(x, "x", torch.float64, int(count))
    _device_buffer(acc, "acc", torch.float64, 2)
    _check(lib.cos_accumulate_moments(int(count), _ptr(x), _ptr(acc), _stream(stream)), "cos_accumulate_moments")


def pade(a, m: int, k: int, x: float = 1.0):
    """[m/k] Pade approximant of sum_i a_i x^i at x and its gradient in a (host)."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))
    if a.size < m + k + 1:
        raise ValueError("need %d coefficients for [%d/%d]" % (m + k + 1, m, k))
    v = ctypes.c_double()
    g = np.zeros(m + k + 1)
    _check(lib.cos_pade(int(m), int(k), _ptr(a), float(x), ctypes.byref(v), _ptr(g)), "cos_pade")
    return v.value, g


def cdet_su2(A, n: int, precision: int, out, eps: float = 1e-12, stream=None):
    """CDet path on the device: A is a device tensor [nconf][2][2n][2n];
    allocates its workspace with torch (plumbing) and writes out[nconf]."""
    import torch
    nconf = int(out.numel())
    _device_buffer(out, "out", torch.float64, nconf)
    _device_buffer(A, "A", torch.float64, nconf * 2 * (2 * int(n)) ** 2)
    nb = ctypes.c_uint64()
    _check(lib.cos_cdet_workspace(int(n), nconf, int(precision), ctypes.byref(nb)), "cos_cdet_workspace")
    work = torch.empty(int(nb.value), dtype=torch.uint8, device=out.device)
    _check(lib.cos_cdet_su2(nconf, int(n), _ptr(A), int(precision), float(eps), _ptr(work), nb.value, _ptr(out),
                            _stream(stream)), "cos_cdet_su2")
    if hasattr(stream, "cuda_stream"):
        work.record_stream(stream)   # keep the workspace until that stream has used it
    return work


def chain_mu_shift(nconf, n, nmat, Goff, G_bar, dG, stub_bar, nstub, U, mu_bar, alpha_bar, stream=None):
    """Chain rule to mu and alpha per configuration and matrix (device); n
    holds each configuration's matrix side."""
    import torch
    _device_buffer(n, "n", torch.int32, int(nconf))
    _device_buffer(Goff, "Goff", torch.int64, int(nconf))
    _device_buffer(G_bar, "G_bar", torch.float64, 1)
    _device_buffer(dG, "dG", torch.float64, G_bar.numel())
    _device_buffer(stub_bar, "stub_bar", torch.float64, int(nconf) * int(nstub))
    _device_buffer(mu_bar, "mu_bar", torch.float64, int(nconf) * int(nmat))
    _device_buffer(alpha_bar, "alpha_bar", torch.float64, int(nconf) * int(nmat))
    _check(lib.cos_chain_mu_shift(int(nconf), _ptr(n), int(nmat), _ptr(Goff), _ptr(G_bar), _ptr(dG),
                                  _ptr(stub_bar), int(nstub), float(U), _ptr(mu_bar), _ptr(alpha_bar),
                                  _stream(stream)), "cos_chain_mu_shift")
