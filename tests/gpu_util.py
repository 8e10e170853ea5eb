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


def workload_params(draw):
    """(nmat, nflav, variant, mu, alpha, stubs per config or None) of a workload."""
    w = draw.workload
    nmat = w.nflav if w.variant == 1 else 1
    mu = np.asarray(w.mu[:nmat], dtype=np.float64)
    alpha = np.asarray(draw.delta[:nmat], dtype=np.float64) if w.variant == 1 else np.zeros(1)
    stubs = None
    if w.stubs:
        sig = (draw.delta[:nmat] / w.U) if w.variant == 1 else np.zeros(1)
        stubs = np.tile(sig, (draw.n.size, 1))
    return nmat, w.nflav, w.variant, mu, alpha, stubs


def gpu_workload(draw, adjoint=False, tune=False):
    """Propagators (G0 kernel) and connected sums (forward kernel) of a drawn
    workload, all on the GPU; returns host copies.  tune=True first runs the
    autotuner (the launch shapes bench.py times)."""
    import torch
    from paper_2507_12349_amd import _binding as B
    from paper_2507_12349_amd.autograd import Geometry
    nmat, nflav, variant, mu, alpha, stubs = workload_params(draw)
    geo = Geometry(draw, nmat)
    G = torch.empty(geo.total, dtype=torch.float64, device=geo.device)
    dG = torch.empty_like(G)
    B.build_g0(geo.nconf, geo.n, geo.voff, geo.sites, geo.tau, geo.L, geo.t, geo.beta, mu, alpha, geo.Goff, G, dG)
    b = B.Batch(draw.n, nflav, variant, stubs=stubs is not None)
    st = None if stubs is None else torch.as_tensor(stubs, device=geo.device)
    out = torch.full((geo.nconf,), float("nan"), dtype=torch.float64, device=geo.device)
    if tune:
        ob = torch.ones(geo.nconf, dtype=torch.float64, device=geo.device)
        b.autotune(G, geo.Goff, st, -1.0, out, ob if adjoint else None, torch.empty_like(G) if adjoint else None,
                   None if st is None else torch.empty_like(st))
        out.fill_(float("nan"))
    b.forward(G, geo.Goff, st, -1.0, out)
    res = dict(G=G.cpu().numpy(), dG=dG.cpu().numpy(), S=None, Goff=geo.Goff_host, nmat=nmat, nflav=nflav,
               variant=variant, mu=mu, alpha=alpha, stubs=stubs)
    torch.cuda.synchronize()
    res["S"] = out.cpu().numpy()
    if adjoint:
        ob = torch.ones(geo.nconf, dtype=torch.float64, device=geo.device)
        Gb = torch.full_like(G, float("nan"))
        sb = None if st is None else torch.full_like(st, float("nan"))
        out2 = torch.full_like(out, float("nan"))
        b.adjoint(G, geo.Goff, st, -1.0, ob, out2, Gb, sb)
        mub = torch.empty(geo.nconf * nmat, dtype=torch.float64, device=geo.device)
        alb = torch.empty_like(mub)
        B.chain_mu_shift(geo.nconf, geo.n, nmat, geo.Goff, Gb, dG, sb, 1 if st is None else st.shape[1],
                         draw.workload.U, mub, alb)
        torch.cuda.synchronize()
        res["shape"] = b.launch_shape(int(draw.n[0]))
        res.update(S2=out2.cpu().numpy(), Gb=Gb.cpu().numpy(), sb=None if sb is None else sb.cpu().numpy(),
                   mub=mub.cpu().numpy().reshape(geo.nconf, nmat), alb=alb.cpu().numpy().reshape(geo.nconf, nmat))
    b.close()
    return res


def config_mats(res, draw, c):
    n = int(draw.n[c])
    a = int(res["Goff"][c])
    return res["G"][a:a + res["nmat"] * n * n].reshape(res["nmat"], n, n)
