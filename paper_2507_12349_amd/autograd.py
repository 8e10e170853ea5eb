"""torch.autograd wrappers over the HIP kernels.

``ConnectedSum`` maps per-configuration propagator matrices (and shift
weights) to the connected sums S_c; its backward runs the reverse sweep kernel
(forward layers recomputed inside, none stored by autograd).
``G0Propagator`` maps per-flavour (mu, alpha) to the propagator matrices of a
fixed set of vertex configurations; its backward is the chain-rule kernel.
``HoneycombPropagator`` does the same for the honeycomb lattice (2n x 2n
matrices for sublattice batches).
PyTorch only provides device memory, streams and the autograd tape.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _binding as B


class ConnectedSum(torch.autograd.Function):
    """S = ConnectedSum.apply(G, stub, batch, Goff, w).

    G: float64 CUDA tensor, all configurations' matrices back to back (layout
    of ``Batch.goff``); stub: float64 [nconf, nstub] or None; Goff: int64
    CUDA tensor of offsets; w: cycle weight (-1 for fermion loops)."""

    @staticmethod
    def forward(ctx, G, stub, batch, Goff, w):
        if not G.is_cuda or G.dtype != torch.float64:
            raise TypeError("G must be a float64 tensor on the GPU")
        G = G.contiguous()
        stub_c = None if stub is None else stub.contiguous()
        out = torch.empty(batch.nconf, dtype=torch.float64, device=G.device)
        batch.forward(G, Goff, stub_c, w, out)
        ctx.batch, ctx.w, ctx.has_stub = batch, float(w), stub is not None
        ctx.save_for_backward(G, Goff, *([stub_c] if stub is not None else []))
        return out

    @staticmethod
    def backward(ctx, gout):
        saved = ctx.saved_tensors
        G, Goff = saved[0], saved[1]
        stub = saved[2] if ctx.has_stub else None
        Gb = torch.empty_like(G)
        sb = torch.empty_like(stub) if stub is not None else None
        ctx.batch.adjoint(G, Goff, stub, ctx.w, gout.contiguous(), None, Gb, sb)
        return Gb, sb, None, None, None


class G0Propagator(torch.autograd.Function):
    """G = G0Propagator.apply(mu, alpha, geom): per-flavour free propagators.

    mu, alpha: float64 CPU tensors [nmat]; geom: a ``Geometry``.  The matrices
    land on the geometry's device; backward returns dL/dmu, dL/dalpha."""

    @staticmethod
    def forward(ctx, mu, alpha, geom):
        G = torch.empty(geom.total, dtype=torch.float64, device=geom.device)
        dG = torch.empty_like(G)
        B.build_g0(geom.nconf, geom.n, geom.voff, geom.sites, geom.tau, geom.L, geom.t, geom.beta,
                   mu.detach().cpu().numpy(), alpha.detach().cpu().numpy(), geom.Goff, G, dG)
        ctx.geom = geom
        ctx.nmat = int(mu.numel())
        ctx.save_for_backward(dG)
        return G

    @staticmethod
    def backward(ctx, gG):
        (dG,) = ctx.saved_tensors
        g = ctx.geom
        mub = torch.empty(g.nconf * ctx.nmat, dtype=torch.float64, device=g.device)
        alb = torch.empty_like(mub)
        B.chain_mu_shift(g.nconf, g.side, ctx.nmat, g.Goff, gG.contiguous(), dG, None, 1, 1.0, mub, alb)
        # per-configuration contributions -> totals over the batch
        mub = mub.view(g.nconf, ctx.nmat).sum(0).cpu()
        alb = alb.view(g.nconf, ctx.nmat).sum(0).cpu()
        return mub, alb, None


class HoneycombPropagator(torch.autograd.Function):
    """G = HoneycombPropagator.apply(mu, alpha, delta, geom): per-flavour free
    propagators of the honeycomb lattice (``geom`` built with
    ``sublattice=True``; delta: the staggered field, a host sequence, held
    fixed).  Backward returns dL/dmu, dL/dalpha."""

    @staticmethod
    def forward(ctx, mu, alpha, delta, geom):
        G = torch.empty(geom.total, dtype=torch.float64, device=geom.device)
        dG = torch.empty_like(G)
        B.build_g0_honeycomb(geom.nconf, geom.n, geom.voff, geom.sites, geom.tau, geom.L, geom.t, geom.beta,
                             mu.detach().cpu().numpy(), alpha.detach().cpu().numpy(),
                             np.asarray(delta, dtype=np.float64), geom.Goff, G, dG=dG)
        ctx.geom = geom
        ctx.nmat = int(mu.numel())
        ctx.save_for_backward(dG)
        return G

    @staticmethod
    def backward(ctx, gG):
        (dG,) = ctx.saved_tensors
        g = ctx.geom
        mub = torch.empty(g.nconf * ctx.nmat, dtype=torch.float64, device=g.device)
        alb = torch.empty_like(mub)
        B.chain_mu_shift(g.nconf, g.side, ctx.nmat, g.Goff, gG.contiguous(), dG, None, 1, 1.0, mub, alb)
        mub = mub.view(g.nconf, ctx.nmat).sum(0).cpu()
        alb = alb.view(g.nconf, ctx.nmat).sum(0).cpu()
        return mub, alb, None, None


class Geometry:
    """Vertex configurations (sites or unit cells, times) resident on the GPU.
    With ``sublattice`` the matrices are 2n x 2n (index 2k + s)."""

    def __init__(self, draw, nmat: int, device="cuda", sublattice: bool = False):
        w = draw.workload
        self.device = torch.device(device)
        self.nconf = int(draw.n.size)
        self.L, self.t, self.beta = w.L, w.t, w.beta
        self.n_host = draw.n
        self.n = torch.as_tensor(draw.n, device=self.device)
        self.voff = torch.as_tensor(draw.voff, device=self.device)
        self.sites = torch.as_tensor(draw.sites, device=self.device).contiguous()
        self.tau = torch.as_tensor(draw.tau, device=self.device)
        side = draw.n.astype(np.int64) * (2 if sublattice else 1)
        self.side = torch.as_tensor(side.astype(np.int32), device=self.device)   # matrix side per config
        sizes = nmat * side ** 2
        off = np.zeros(self.nconf, dtype=np.int64)
        off[1:] = np.cumsum(sizes[:-1])
        self.Goff_host = off
        self.Goff = torch.as_tensor(off, device=self.device)
        self.total = int(sizes.sum())
