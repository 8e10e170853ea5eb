"""Oracle for the connected-diagram sum -- TEST INFRASTRUCTURE ONLY.

Plain, slow CPU reference implementations of what the GPU library computes,
written from arXiv 2507.12349 (CoS / SB-CoS).  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import this package.  It shares no code with ``paper_2507_12349_amd``.

Contents
  O1  :func:`brute`       definition by enumeration (C, ``cos_oracle.c``)
  O2  :func:`closed_form` determinant closed form + connected-part recursion
                          (exact rational arithmetic, ``closed_form.py``)
  O3  :func:`dp`, :func:`dp_adjoint`, :func:`dp_subsets`
                          vertex-level dynamic programme and its reverse sweep (C)
  O3L :func:`alg3`        Alg. 3 at point level, no canonicalisation (C)
  G0  :mod:`oracle.g0`    free propagator of the square-lattice model
  counts :mod:`oracle.counts` diagram counts from the exponential formula

Argument conventions shared by all routines: ``G`` is a float64 array of
shape ``(n, n)`` (variant U) or ``(nf, n, n)`` (variant F), indexed by vertex;
``stub`` holds the shift weights sigma (``[1]`` for U, ``[nf]`` for F) or is
None; ``w`` is the weight of one closed cycle (-1 for fermion loops).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cos_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "libcos_oracle.so")
_lib = None

U, F = 0, 1


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (host only)."""
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    i, d, p, i64p = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)
    for sfx, rt in (("_ld", ctypes.c_longdouble), ("_d", ctypes.c_double)):
        f = getattr(lib, "cos_oracle_brute" + sfx)
        f.argtypes = [i, i, i, i, p, p, d, i]
        f.restype = rt
        f = getattr(lib, "cos_oracle_dp" + sfx)
        f.argtypes = [i, i, i, i, p, p, d, i64p]
        f.restype = rt
        f = getattr(lib, "cos_oracle_dp_adjoint" + sfx)
        f.argtypes = [i, i, i, i, p, p, d, p, p]
        f.restype = rt
        f = getattr(lib, "cos_oracle_dp_subsets" + sfx)
        f.argtypes = [i, i, i, i, p, p, d, p]
        f.restype = None
        f = getattr(lib, "cos_oracle_alg3" + sfx)
        f.argtypes = [i, i, i, i, p, p, d]
        f.restype = rt
    _lib = lib
    return lib


def _prep(G, nf, variant, stub):
    G = np.ascontiguousarray(G, dtype=np.float64)
    if variant == U:
        assert G.ndim == 2, "variant U takes one (n, n) matrix"
        n = G.shape[0]
    else:
        assert G.ndim == 3 and G.shape[0] == nf, "variant F takes (nf, n, n)"
        n = G.shape[1]
    assert 1 <= n <= 12 and 1 <= nf <= 16
    use_stubs = stub is not None
    if use_stubs:
        stub = np.ascontiguousarray(stub, dtype=np.float64).reshape(-1)
        assert stub.size == (1 if variant == U else nf)
    else:
        stub = np.zeros(1 if variant == U else nf)
    return G, n, int(use_stubs), stub


def _sfx(precision):
    return "_ld" if precision == "ld" else "_d"


def brute(G, nf, variant=U, stub=None, w=-1.0, connected=True, precision="ld"):
    """O1: enumerate stub sets, permutations and cycle flavours (small n only)."""
    G, n, us, st = _prep(G, nf, variant, stub)
    f = getattr(_load(), "cos_oracle_brute" + _sfx(precision))
    return float(f(n, nf, variant, us, G.ctypes.data, st.ctypes.data, float(w), int(connected)))


def dp(G, nf, variant=U, stub=None, w=-1.0, precision="ld", counts=False):
    """O3: vertex-level DP.  With ``counts`` also returns per-flavour-slot plan
    counts ``dict(states, ext, closes, stub_edges, masks)``."""
    G, n, us, st = _prep(G, nf, variant, stub)
    f = getattr(_load(), "cos_oracle_dp" + _sfx(precision))
    c = (ctypes.c_int64 * 5)()
    S = float(f(n, nf, variant, us, G.ctypes.data, st.ctypes.data, float(w), c))
    if counts:
        return S, dict(zip(("states", "ext", "closes", "stub_edges", "masks"), list(c)))
    return S


def dp_adjoint(G, nf, variant=U, stub=None, w=-1.0, precision="ld"):
    """O3 reverse sweep: returns (S, dS/dG, dS/dsigma) as float64 arrays."""
    G, n, us, st = _prep(G, nf, variant, stub)
    real = np.longdouble if precision == "ld" else np.float64
    gb = np.zeros(G.shape, dtype=real)
    sb = np.zeros(st.shape, dtype=real)
    f = getattr(_load(), "cos_oracle_dp_adjoint" + _sfx(precision))
    S = float(f(n, nf, variant, us, G.ctypes.data, st.ctypes.data, float(w), gb.ctypes.data, sb.ctypes.data))
    return S, gb.astype(np.float64), sb.astype(np.float64)


def dp_subsets(G, nf, variant=U, stub=None, w=-1.0, precision="ld"):
    """Connected sums c(S) of every vertex subset S containing vertex 0 (array
    indexed by subset bitmask), read off the DP's dropped closes."""
    G, n, us, st = _prep(G, nf, variant, stub)
    real = np.longdouble if precision == "ld" else np.float64
    out = np.zeros(1 << n, dtype=real)
    f = getattr(_load(), "cos_oracle_dp_subsets" + _sfx(precision))
    f(n, nf, variant, us, G.ctypes.data, st.ctypes.data, float(w), out.ctypes.data)
    return out.astype(np.float64)


def alg3(G, nf, variant=U, stub=None, w=-1.0, precision="ld"):
    """O3L: Alg. 3 at point level (tiny n only)."""
    G, n, us, st = _prep(G, nf, variant, stub)
    f = getattr(_load(), "cos_oracle_alg3" + _sfx(precision))
    return float(f(n, nf, variant, us, G.ctypes.data, st.ctypes.data, float(w)))


from . import closed_form, counts, g0  # noqa: E402,F401
from .closed_form import closed_form as closed_form_sum  # noqa: E402,F401
