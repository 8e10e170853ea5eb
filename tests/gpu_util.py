"""Helpers for the GPU tests: run the HIP path through the C ABI on device
tensors, and build the oracle's reference from the oracle's own inputs."""
import sys

import numpy as np


def announce(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


def pack(mats):
    """List of (nmat, n, n) arrays -> (flat float64, int64 offsets, orders)."""
    n = np.array([m.shape[-1] for m in mats], dtype=np.int32)
    sizes = np.array([m.size for m in mats], dtype=np.int64)
    off = np.zeros(len(mats), dtype=np.int64)
    off[1:] = np.cumsum(sizes[:-1])
    return np.concatenate([m.reshape(-1) for m in mats]), off, n


def gpu_forward(mats, nflav, variant, stubs=None, w=-1.0, adjoint=False, out_bar=None):
    """Batched forward (and optionally the adjoint) on the GPU.
    mats: list of (nmat, n, n) float64 arrays; stubs: (nconf, nstub) or None."""
    import torch
    from paper_2507_12349_amd import _binding as B
    flat, off, n = pack(mats)
    dev = torch.device("cuda:0")
    G = torch.as_tensor(flat, device=dev)
    Goff = torch.as_tensor(off, device=dev)
    st = None if stubs is None else torch.as_tensor(np.ascontiguousarray(stubs, dtype=np.float64), device=dev)
    b = B.Batch(n, nflav, variant, stubs=stubs is not None)
    out = torch.full((len(mats),), float("nan"), dtype=torch.float64, device=dev)
    b.forward(G, Goff, st, w, out)
    torch.cuda.synchronize()
    S = out.cpu().numpy()
    if not adjoint:
        b.close()
        return S
    ob = torch.as_tensor(np.ones(len(mats)) if out_bar is None else out_bar, device=dev, dtype=torch.float64)
    Gb = torch.full_like(G, float("nan"))
    sb = None if st is None else torch.full_like(st, float("nan"))
    out2 = torch.full_like(out, float("nan"))
    b.adjoint(G, Goff, st, w, ob, out2, Gb, sb)
    torch.cuda.synchronize()
    b.close()
    gbar = Gb.cpu().numpy()
    gb_list = [gbar[off[i]:off[i] + mats[i].size].reshape(mats[i].shape) for i in range(len(mats))]
    return S, out2.cpu().numpy(), gb_list, (None if sb is None else sb.cpu().numpy())


def oracle_args(M, variant):
    """(nmat, n, n) -> the oracle's G argument."""
    return M[0] if variant == 0 else M


def scale(oracle, M, nf, variant, st, w=-1.0):
    G = np.abs(oracle_args(M, variant))
    return oracle.dp(G, nf, variant, None if st is None else -np.abs(st), abs(w))
