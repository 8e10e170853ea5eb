"""End-to-end parity on the five synthetic workloads: propagators from the
G0 kernel vs the oracle's numpy builder, and connected sums of the GPU
pipeline vs the oracle run on the oracle's own propagators.  Full batches run
on the GPU in the launch configuration the benchmark uses; sampled
configurations are checked one by one against the oracle (long double).

Gate: relative 1e-10 for every sampled configuration.  The FP64 bound
8 n (n + 2) eps S_abs (kappa = S_abs / |S| measures the cancellation) is printed
beside it; it replaces the gate only for the named exceptions, configurations
whose cancellation lets FP64 rounding alone exceed 1e-10."""
import numpy as np
import pytest

from gpu_util import announce, config_mats, gpu_workload, oracle_args
from paper_2507_12349_amd.workloads import draw

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps
# kappa 2.8e9: measured 1.4e-10 relative, 2.3e-7 of its FP64 bound
EXCEPTIONS = {("sym_broken", 96)}


def _check_sample(oracle_mod, d, res, idx):
    from oracle import g0
    w = d.workload
    worst = 0.0
    for c in idx:
        n = int(d.n[c])
        sites, tau = d.config(c)
        Go, _ = g0.build_g0(w.L, w.t, w.beta, res["mu"], res["alpha"], sites, tau)
        Gg = config_mats(res, d, c)
        assert np.allclose(Gg, Go, rtol=0, atol=2e-15), (c, np.abs(Gg - Go).max())
        st = None if res["stubs"] is None else res["stubs"][c]
        ref = oracle_mod.dp(oracle_args(Go, res["variant"]), res["nflav"], res["variant"], st)
        sa = oracle_mod.dp(np.abs(oracle_args(Go, res["variant"])), res["nflav"], res["variant"],
                           None if st is None else -np.abs(st), 1.0)
        err = abs(res["S"][c] - ref)
        bound = 8 * n * (n + 2) * EPS * sa
        exc = (w.name, int(c)) in EXCEPTIONS
        print("  config %d n=%d S=%.6e ref=%.6e rel=%.2e kappa=%.1e err/FP64 bound=%.1e%s"
              % (c, n, res["S"][c], ref, err / abs(ref), sa / abs(ref), err / bound,
                 " (named exception)" if exc else ""), flush=True)
        assert err <= (bound if exc else 1e-10 * abs(ref)), (c, n, res["S"][c], ref)
        if not exc:
            worst = max(worst, err / abs(ref))
    return worst


def _sample(d, k, seed, maxn=12):
    rng = np.random.default_rng(seed)
    ok = np.nonzero(d.n <= maxn)[0]
    return sorted(rng.choice(ok, size=min(k, ok.size), replace=False).tolist())


def test_plain_single(oracle_mod):
    announce("workload plain_single")
    d = draw("plain_single")
    res = gpu_workload(d)
    _check_sample(oracle_mod, d, res, [0])


def test_plain_batch(oracle_mod):
    announce("workload plain_batch (4096 x n=8, SU(4))")
    d = draw("plain_batch")
    res = gpu_workload(d)
    assert np.all(np.isfinite(res["S"]))
    _check_sample(oracle_mod, d, res, _sample(d, 24, 2))


def test_sym_broken(oracle_mod):
    announce("workload sym_broken (1024 x n=10, SU(3) flavour mu)")
    d = draw("sym_broken")
    res = gpu_workload(d)
    assert np.all(np.isfinite(res["S"]))
    _check_sample(oracle_mod, d, res, _sample(d, 4, 3))


def test_uneven_prefix(oracle_mod):
    """First 512 configurations of the uneven SU(6) shift workload (orders 6..12,
    level launches per order): every configuration of order <= 7 against the
    oracle, and samples of orders 8 to 11 (the oracle takes about 10 s per
    configuration at n = 11; order 12 is covered by the adjoint tests)."""
    announce("workload uneven prefix 512")
    d = draw("uneven", nconf=512)
    res = gpu_workload(d)
    assert np.all(np.isfinite(res["S"]))
    idx = np.nonzero(d.n <= 7)[0].tolist()
    rng = np.random.default_rng(4)
    for k, cnt in ((8, 4), (9, 2), (10, 1), (11, 1)):
        ok = np.nonzero(d.n == k)[0]
        idx += sorted(rng.choice(ok, size=min(cnt, ok.size), replace=False).tolist())
    assert len(idx) > 100
    _check_sample(oracle_mod, d, res, idx)


def test_adjoint_workload_forward(oracle_mod):
    announce("workload adjoint forward (2048 x n=10, SU(4))")
    d = draw("adjoint")
    res = gpu_workload(d)
    assert np.all(np.isfinite(res["S"]))
    _check_sample(oracle_mod, d, res, _sample(d, 8, 5))


def test_uneven_full(oracle_mod):
    """All 8192 configurations of the uneven SU(6) shift workload in one batch
    (orders 6..12, one group of launches per order, order 12 in chunks of
    groups where the workspace limit asks for it, orders 11..6 on the
    library's side stream beside order 12): every sum finite; the first 512 bitwise equal to the
    same configurations run as a batch of their own (a configuration's sum does
    not depend on the rest of the batch); samples of every order up to 11
    against the oracle."""
    announce("workload uneven full (8192 configurations, orders 6..12)")
    d = draw("uneven")
    assert d.n.size == 8192 and set(np.unique(d.n)) == set(range(6, 13))
    res = gpu_workload(d)
    assert np.all(np.isfinite(res["S"]))
    head = gpu_workload(draw("uneven", nconf=512))
    assert np.array_equal(res["S"][:512], head["S"])
    rng = np.random.default_rng(44)
    idx = []
    for k, cnt in ((6, 3), (7, 3), (8, 2), (9, 2), (10, 2), (11, 1)):
        ok = np.nonzero(d.n[512:] == k)[0] + 512
        idx += sorted(rng.choice(ok, size=cnt, replace=False).tolist())
    _check_sample(oracle_mod, d, res, idx)
