"""GPU parity of the multi-index Monte Carlo driver (mlmc_mimc) against the
oracle's estimator on the same random numbers."""
import math
import sys

import numpy as np
import pytest

import oracle
import seeded_inputs as si

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def _ctx(**kw):
    from paper_2503_05533_amd import MLMC, Config
    return MLMC(Config(**kw), device="cuda:0")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle(n0, K, s2, lam, seed, idx, N, K0):
    L = max(l for l, _ in idx)
    phis = {l: oracle.kl_basis(n0 << l, K, s2, lam) for l in range(L + 1)}
    solve = lambda l, xi: oracle.solve_batch(n0 << l, phis[l], xi)
    normals = lambda i, count: si.splitmix64_normals(seed, 8192 + i, 0, count, K)
    return oracle.mimc(idx, N, K0, K, solve, normals)


def test_mimc_matches_oracle_fp64():
    """A full 3 x 3 box of (grid, truncation) indices on grids 4/8/16 with 8
    modes (2, 4, 8 kept): FP64 direct solves give the oracle's per-index means
    and variances of the mixed differences."""
    _torch()
    n0, L, K, K0, s2, lam, seed = 4, 2, 8, 2, 1.0, 0.3, 4242
    idx = [(l, k) for l in range(L + 1) for k in range(3)]
    N = [24 + 3 * i for i in range(len(idx))]
    ctx = _ctx(n0=n0, L_max=L, K=K, sigma2=s2, corr_len=lam, seed=seed)
    r = ctx.mimc(idx, N, K0, opts=[dict(dtype="f64", solver="direct")] * len(idx), seed=seed)
    ref = _oracle(n0, K, s2, lam, seed, idx, N, K0)
    _say("gpu", r["mean"], "oracle", ref["mean"])
    qmax = 0.1
    for i in range(len(idx)):
        assert abs(r["mean"][i] - ref["mean"][i]) <= 4e-12 * qmax, (idx[i], r["mean"][i], ref["mean"][i])
        assert abs(r["var"][i] - ref["var"][i]) <= 1e-12 * qmax ** 2 + 1e-9 * ref["var"][i], idx[i]
    assert abs(r["estimate"] - ref["estimate"]) <= 4e-11 * qmax
    assert r["n_noconv"] == [0] * len(idx) and r["n_promoted"] == [0] * len(idx)
    # solves: one per (grid, truncation) term of each index
    assert r["solves"] == sum((2 if l else 1) * (2 if k else 1) for l, k in idx)
    ctx.close()


def test_mimc_chunked_index_matches_oracle():
    """One index on the 64-cell grid with 5000 samples, more than one chunk of
    the driver's workspace budget: chunk sums added in order give the oracle's
    mean and variance."""
    _torch()
    n0, K, K0, s2, lam, seed = 16, 32, 8, 1.0, 0.3, 777
    idx, N = [(2, 1)], [5000]
    ctx = _ctx(n0=n0, L_max=2, K=K, sigma2=s2, corr_len=lam, seed=seed)
    r = ctx.mimc(idx, N, K0, opts=[dict(dtype="f64", solver="direct")], seed=seed)
    ref = _oracle(n0, K, s2, lam, seed, idx, N, K0)
    _say("gpu", r["mean"], r["var"], r["solves"], "oracle", ref["mean"], ref["var"])
    assert r["solves"] > 4, "expected more than one chunk"
    assert abs(r["mean"][0] - ref["mean"][0]) <= 4e-12 * 0.1
    assert abs(r["var"][0] - ref["var"][0]) <= 1e-8 * ref["var"][0]
    ctx.close()


def test_mimc_mixed_precision_within_accuracy_targets():
    """A total-degree index set (l + k <= 2) on grids 16/32/64 with 64 modes
    (16, 32, 64 kept): FP32 factors refined to the accuracy targets of Sec. 4.5
    (grid l to delta_l) against FP64 direct solves on the same samples; every
    mean within the targets' bound, no sample left unconverged, and the
    estimates far closer than the statistical error."""
    _torch()
    n0, L, K, K0, s2, lam, seed = 16, 2, 64, 16, 1.0, 0.3, 31337
    idx = [(l, k) for l in range(L + 1) for k in range(L + 1) if l + k <= L]
    N = [int(3000 * 4.0 ** (-l) * 2.0 ** (-k)) for l, k in idx]
    ctx = _ctx(n0=n0, L_max=L, K=K, sigma2=s2, corr_len=lam, seed=seed)
    eps = ctx.accuracy_targets(L)
    o64 = [dict(dtype="f64", solver="direct")] * len(idx)
    omx = [dict(dtype="f32", solver="direct_ir", eps_fine=eps[l], eps_coarse=eps[l - 1] if l else 0.0)
           for l, _ in idx]
    r64 = ctx.mimc(idx, N, K0, opts=o64, seed=seed)
    rmx = ctx.mimc(idx, N, K0, opts=omx, seed=seed)
    se = math.sqrt(r64["var_estimate"])
    _say("fp64", r64["estimate"], "mixed", rmx["estimate"], "se", se, "noconv", rmx["n_noconv"])
    assert rmx["n_noconv"] == [0] * len(idx)
    qmax = 0.1
    for i, (l, k) in enumerate(idx):
        bound = 4.0 * (eps[l] + (eps[l - 1] if l else 0.0)) * qmax
        assert abs(rmx["mean"][i] - r64["mean"][i]) <= bound, ((l, k), rmx["mean"][i], r64["mean"][i])
    assert abs(rmx["estimate"] - r64["estimate"]) <= 0.1 * se
    ctx.close()
