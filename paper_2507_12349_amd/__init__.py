"""MI355X-native connected-diagram sums of the SU(N) Hubbard model (CoS / SB-CoS,
arXiv 2507.12349).

The work runs in hand-written HIP kernels for gfx950 behind the C ABI of
``include/libcos.h`` (``libcos.so``); ``_binding`` is the thin ctypes layer and
``autograd`` the torch.autograd wrappers.  Names of the binding are loaded on
first use: touching any of them without the built library raises ImportError
(there is no CPU fallback).  ``workloads`` (seeded inputs) needs no library.
"""
_BINDING = {"Batch", "CosError", "connected_sum_host", "plan_counts", "plan_counts_sublattice", "build_g0", "build_g0_honeycomb", "mc_sample",
            "accumulate_moments", "pade", "cdet_su2", "plan_counts_mask_only", "F_MASK_ONLY",
            "chain_mu_shift", "UNIFORM", "FLAVOUR", "F_STUBS", "F_SUBLATTICE", "NMAX", "FMAX", "NMAX_SUBLATTICE",
            "LIB_PATH", "EXPORTED", "lib", "set_workspace_limit"}


def __getattr__(name):
    if name in _BINDING:
        from . import _binding
        return getattr(_binding, name)
    raise AttributeError("module %r has no attribute %r" % (__name__, name))
