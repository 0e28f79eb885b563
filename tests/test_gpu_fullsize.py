"""Parity at the workloads' full sizes, on sampled outputs.

Every batch runs at its full sample count in the launch configuration the
benchmark uses (all levels concurrent, one replayed HIP graph, or one level
call per grid); a sample of rows is then checked against the FP64 oracle,
which solves those rows one by one.  The mixed-precision bound is the one of
the residual test: |Q - Q~| <= (||r||/||b||) ||u|| ||b|| / (b^T u) with the
oracle's u, applied to the fine and the coarse partner of each Y_l.
"""
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


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


_PHI = {}


def _phi(n, K, s2, lam):
    key = (n, K, s2, lam)
    if key not in _PHI:
        _PHI[key] = oracle.kl_basis(n, K, s2, lam)
    return _PHI[key]


def _picks(N, k, seed):
    rng = np.random.default_rng(seed)
    extra = rng.choice(np.arange(1, max(N - 1, 1)), size=min(k, max(N - 2, 0)), replace=False)
    return sorted(set([0, N - 1] + [int(i) for i in extra]))


_ORQ = {}


def _oracle_q(n, K, s2, lam, seed, level, idx):
    """Q and the residual-bound factor ||u|| ||b|| / (b^T u) of the given sample rows."""
    key = (n, K, s2, lam, seed, level, tuple(idx))
    if key not in _ORQ:
        xi = np.vstack([si.splitmix64_normals(seed, level, i, 1, K) for i in idx])
        q, u = oracle.solve_batch(n, _phi(n, K, s2, lam), xi, want_u=True)
        bound = np.linalg.norm(u, axis=1) * (math.sqrt(u.shape[1]) / n ** 2) / q
        _ORQ[key] = (q, bound)
    return _ORQ[key]


def _check_y(y, idx, w, level, eps_f, eps_c, fp64=False):
    n0, K, s2, lam, seed = w["n0"], w["K"], w["sigma2"], w["corr_len"], w["seed"]
    nf = n0 << level
    qf, bf = _oracle_q(nf, K, s2, lam, seed, level, idx)
    if level > 0:
        qc, bc = _oracle_q(nf // 2, K, s2, lam, seed, level, idx)
    else:
        qc, bc = np.zeros_like(qf), np.zeros_like(qf)
    yref = qf - qc
    got = np.asarray(y)[idx]
    if fp64:
        tol = 1e-12 * (np.abs(qf) + np.abs(qc))
    else:
        tol = (eps_f * bf * np.abs(qf) + eps_c * bc * np.abs(qc)) * (1 + 1e-6)
    err = np.abs(got - yref)
    assert np.all(err <= tol + 1e-16), (level, err.max(), tol.min())
    return float(np.max(err / (np.abs(qf) + np.abs(qc))))


@pytest.mark.parametrize("use_graph", [False, True])
@pytest.mark.parametrize("dtype,solver", [("f32", "direct_ir"), ("f64", "direct")])
def test_bench_step_fullsize(dtype, solver, use_graph):
    """mlmc4_n16-128_K64 at N_l = 20000/5000/1250/300: the eager one-stream-per-queue
    schedule (the bench step) and the replayed graph."""
    torch = _torch()
    from paper_2503_05533_amd import MLMC, Config
    w = si.workload("mlmc4_n16-128_K64")
    levels, Ns, K = w["levels"], w["N"], w["K"]
    ctx = MLMC(Config(n0=w["n0"], L_max=3, K=K, sigma2=w["sigma2"], corr_len=w["corr_len"],
                      seed=w["seed"], ir_max_iter=10), device="cuda:0")
    eps = ctx.accuracy_targets(3)
    xis = [ctx.fill_xi(l, 0, N) for l, N in zip(levels, Ns)]
    opts = [dict(dtype=dtype, solver=solver, eps_fine=eps[l], eps_coarse=eps[l - 1] if l else 0.0)
            for l in levels]
    plan = ctx.plan_levels(levels, xis, opts, use_graph=use_graph)
    plan.run()
    out = plan.run(stats=True)
    torch.cuda.synchronize()
    for i, l in enumerate(levels):
        st = out["stats"][i]
        assert st["n"] == Ns[i] and st["n_noconv"] == 0, st
        y = out["y"][i].cpu().numpy()
        assert np.isfinite(y).all()
        assert st["sum_y"] == pytest.approx(float(y.sum()), rel=1e-9, abs=1e-15)
        idx = _picks(Ns[i], 10, 100 + l)
        worst = _check_y(y, idx, w, l, eps[l], eps[l - 1] if l else 0.0, fp64=(dtype == "f64"))
        _say("bench step %s graph=%d level %d: %d sampled rows, max rel err %.2e"
             % (dtype, use_graph, l, len(idx), worst))
    ctx.close()


def test_step_schedules_identical():
    """The eager and the graph schedule run the same kernels on different streams:
    Y and the level sums agree bit for bit (mixed path, full bench workload)."""
    torch = _torch()
    from paper_2503_05533_amd import MLMC, Config
    w = si.workload("mlmc4_n16-128_K64")
    levels, Ns, K = w["levels"], w["N"], w["K"]
    ctx = MLMC(Config(n0=w["n0"], L_max=3, K=K, sigma2=w["sigma2"], corr_len=w["corr_len"],
                      seed=w["seed"], ir_max_iter=10), device="cuda:0")
    eps = ctx.accuracy_targets(3)
    xis = [ctx.fill_xi(l, 0, N) for l, N in zip(levels, Ns)]
    opts = [dict(dtype="f32", solver="direct_ir", eps_fine=eps[l], eps_coarse=eps[l - 1] if l else 0.0)
            for l in levels]
    res = []
    for g in (False, True, False):
        out = ctx.plan_levels(levels, xis, opts, use_graph=g).run(stats=True)
        torch.cuda.synchronize()
        res.append(([y.cpu().numpy().copy() for y in out["y"]], [st["sum_y"] for st in out["stats"]]))
    for ys, sums in res[1:]:
        for i in range(len(levels)):
            assert np.array_equal(ys[i], res[0][0][i]), i
            assert sums[i] == res[0][1][i], i
    ctx.close()


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
def test_precision_sweep_fullsize(dtype):
    """sweep5_n16-256_K128: every level at full N with the given factor storage."""
    torch = _torch()
    from paper_2503_05533_amd import MLMC, Config
    w = si.workload("sweep5_n16-256_K128")
    levels, Ns, K = w["levels"], w["N"], w["K"]
    ctx = MLMC(Config(n0=w["n0"], L_max=4, K=K, sigma2=w["sigma2"], corr_len=w["corr_len"],
                      seed=w["seed"], ir_max_iter=10), device="cuda:0")
    eps = ctx.accuracy_targets(4)
    for l, N in zip(levels, Ns):
        xi = ctx.fill_xi(l, 0, N)
        out = ctx.sample_level(l, xi, dtype=dtype, solver="direct_ir", eps_fine=eps[l],
                               eps_coarse=eps[l - 1] if l else 0.0)
        st = out["stats"]
        assert st["n_noconv"] == 0, (l, st)
        status = out["status"].cpu().numpy()
        assert np.all(status & 1) and (l == 0 or np.all(status & 16)), l
        idx = _picks(N, 6 if l < 4 else 3, 200 + l)
        worst = _check_y(out["y"].cpu().numpy(), idx, w, l, eps[l], eps[l - 1] if l else 0.0)
        _say("sweep %s level %d N=%d: promoted %d, mean corrections %.3f, max rel err %.2e"
             % (dtype, l, N, st["n_promoted"], st["mean_iters"], worst))
        del xi, out
        torch.cuda.synchronize()
    ctx.close()


@pytest.mark.parametrize("solver", ["direct_ir", "minres"])
def test_all_levels_one_graph_fullsize(solver):
    """batched5_n16-256_K128: the five levels (40000 ... 200 samples) in one graph."""
    torch = _torch()
    from paper_2503_05533_amd import MLMC, Config
    w = si.workload("batched5_n16-256_K128")
    levels, Ns, K = w["levels"], w["N"], w["K"]
    ctx = MLMC(Config(n0=w["n0"], L_max=4, K=K, sigma2=w["sigma2"], corr_len=w["corr_len"],
                      seed=w["seed"], ir_max_iter=10, minres_max_iter=20000), device="cuda:0")
    eps = ctx.accuracy_targets(4)
    xis = [ctx.fill_xi(l, 0, N) for l, N in zip(levels, Ns)]
    opts = [dict(dtype="f32", solver=solver, eps_fine=eps[l], eps_coarse=eps[l - 1] if l else 0.0)
            for l in levels]
    out = ctx.plan_levels(levels, xis, opts, use_graph=True).run(stats=True)
    torch.cuda.synchronize()
    for i, l in enumerate(levels):
        st = out["stats"][i]
        assert st["n"] == Ns[i] and st["n_noconv"] == 0, (l, st)
        idx = _picks(Ns[i], 5 if l < 4 else 2, 300 + l)
        worst = _check_y(out["y"][i].cpu().numpy(), idx, w, l, eps[l], eps[l - 1] if l else 0.0)
        _say("one graph %s level %d: mean iterations %.2f, max rel err %.2e" % (solver, l, st["mean_iters"], worst))
    ctx.close()


def test_adjoint_fullsize():
    """adjoint_n128_K128: dQ/dxi for 4096 samples at n = 128; sampled rows vs the oracle gradient."""
    torch = _torch()
    from paper_2503_05533_amd import MLMC, Config
    w = si.workload("adjoint_n128_K128")
    K, N = w["K"], w["N"][0]
    ctx = MLMC(Config(n0=w["n0"], L_max=0, K=K, sigma2=w["sigma2"], corr_len=w["corr_len"],
                      seed=w["seed"]), device="cuda:0")
    xi = ctx.fill_xi(0, 0, N)
    q, g = ctx.grad(0, xi, None, eps_adjoint=1e-10, dtype="f32", solver="direct_ir", eps=1e-10)
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    assert np.isfinite(g).all()
    idx = _picks(N, 4, 400)
    xr = np.vstack([si.splitmix64_normals(w["seed"], 0, i, 1, K) for i in idx])
    ref = oracle.grad_batch(128, _phi(128, K, w["sigma2"], w["corr_len"]), xr)
    for k, i in enumerate(idx):
        rel = np.linalg.norm(g[i] - ref[k]) / np.linalg.norm(ref[k])
        assert rel <= 1e-7, (i, rel)
    qref = oracle.solve_batch(128, _phi(128, K, w["sigma2"], w["corr_len"]), xr)
    assert np.allclose(q.cpu().numpy()[idx], qref, rtol=1e-9, atol=0)
    ctx.close()


def test_estimate_chunks_fp64_fullsize():
    """Algorithm 4.1 at the bench tolerance on the FP64 path: level 0 takes ~1.6M
    samples, streamed as many chunks on one queue stream with per-chunk sums added
    in order.  The FP64 solves do not depend on the round's accuracy targets, so an
    independent pass over the same xi ranges (other chunk sizes) must give every
    level's mean and variance to rounding."""
    torch = _torch()
    from paper_2503_05533_amd import MLMC, Config
    w = si.workload("mlmc4_n16-128_K64")
    ctx = MLMC(Config(n0=w["n0"], L_max=3, K=w["K"], sigma2=w["sigma2"], corr_len=w["corr_len"],
                      seed=w["seed"]), device="cuda:0")
    res = ctx.estimate(2e-5, n_init=1000, dtypes=["f64"] * 4, solver="direct", mixed=False)
    assert res["converged"] and res["L"] == 3
    assert res["N"][0] > 3 * (1 << 18), res["N"]  # several estimator chunks
    step = 200000
    for l, N in enumerate(res["N"]):
        s1 = s2 = 0.0
        for first in range(0, N, step):
            cnt = min(step, N - first)
            out = ctx.sample_level(l, ctx.fill_xi(l, first, cnt), dtype="f64", solver="direct")
            y = out["y"]
            s1 += float(y.sum())
            s2 += float((y * y).sum())
            del out, y
        torch.cuda.synchronize()
        mean = s1 / N
        var = max(s2 / N - mean * mean, 0.0)
        _say("level %d N=%d: estimator %.15e / %.6e, independent pass %.15e / %.6e"
             % (l, N, res["Yhat"][l], res["s2"][l], mean, var))
        assert mean == pytest.approx(res["Yhat"][l], rel=1e-11, abs=1e-16)
        assert var == pytest.approx(res["s2"][l], rel=1e-8, abs=1e-18)
    ctx.close()
