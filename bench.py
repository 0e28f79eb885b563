"""Benchmark of the batched per-level sample solve on one MI355X.

A step is one pass of the whole hot path over one batch: for every level l
of the workload, N_l samples, each a fine solve on grid l and (l >= 1) a
coarse solve on grid l-1 from the same xi row, paired into Y_l, with the
level sums.  All levels run concurrently: the grids are spread over one
stream per hardware queue, the fine grid of the finest level alone on the
first (--graph: the two-streams-per-level fork/join replayed as one HIP
graph instead).  The mixed path factorises in FP32 and
refines in FP64 to the level accuracy delta_l of the adaptive rule; the FP64
path factorises and solves in FP64.  Inputs (xi) are resident in HBM before
the timed region.

Legs:
  * timed: W warm-up steps, then K steps between two device synchronisations
    (the value); a step draws every level's xi on the device (counter-based
    generator) and runs all levels;
  * profiled: the same K steps launched eagerly with HIP events around each
    kernel launch on its own stream (per-kernel device time; the roofline of
    the dominant kernel);
  * per level: each level alone, event-timed (samples/s per level);
  * FP64: the same timed leg with the FP64 direct path;
  * time to RMSE: Algorithm 4.1 (adaptive MLMC) to an absolute tolerance,
    mixed and FP64, over R seeds: median wall time on the host (the first
    call allocates the estimator's workspace and is not counted) and the
    achieved RMSE against an FP64 reference at TOL/5, with a 95% interval;
  * other workloads (legs): the single-level FP64 workload, the per-level
    precision sweep (FP32/BF16/FP16 and FP64 per level), all five levels in
    one captured graph (refinement vs MINRES and MINRES-IR), the adjoint
    batch, and the paper's two direct-solver examples on its own
    discretisation and field (P1 elements, trigonometric field): the Table 1
    precisions and the quarter-precision example (FP8 factor on level 0),
    each at fixed N_l, MSE against FP64 over many runs with shared xi, and
    the stored-bytes count; and its iterative-solver comparison (adaptive
    MPML against standard MLMC at a fixed 1e-6, MINRES and multigrid CG);
    and multilevel MCMC with FP64 and mixed-precision solves;
  * CPU: the FP64 oracle on a bounded sample of the workload, host cores,
    one core, and LAPACK's banded Cholesky on the same systems.

Prints one JSON line.  --gpus N > 1 is refused: the path runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PDE samples/s per level + MLMC time-to-RMSE, mixed+IR vs FP64 on same GPU"
PEAK = {"f64": 78.6, "f32": 157.3, "hbm": 8000.0}  # TFLOP/s (FP64, FP32 MFMA), GB/s
DT_BYTES = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}  # factor storage bytes


# HBM bytes per sample measured with FETCH_SIZE / WRITE_SIZE counters (scaled
# by a copy kernel of known size) for the mixed FP32 step; valid only while the
# kernel sources hash to TRAFFIC_SRC (otherwise the field is reported as null).
TRAFFIC_SRC = "815c97f5bfbd08c8"
TRAFFIC = {("factor", 128, "f32"): 10.4705e6, ("factor", 64, "f32"): 1.5585e6,
           ("factor", 32, "f32"): 0.2540e6, ("factor", 16, "f32"): 0.0467e6,
           ("solve", 128, "f32"): 11.6568e6, ("solve", 64, "f32"): 1.7648e6,
           ("solve", 32, "f32"): 0.0249e6, ("solve", 16, "f32"): 0.0052e6}


def kernel_src_hash():
    import hashlib
    d = os.path.join(ROOT, "paper_2503_05533_amd", "csrc")
    src = b"".join(open(os.path.join(d, f), "rb").read()
                   for f in ("factor_mfma.hip", "refine_blk.hip", "blk_common.h", "kernels.h", "dtypes.h",
                             "ir_common.h"))
    return hashlib.sha256(src).hexdigest()[:16]


def factor_flops(n):
    """Algorithmic flops of one grid factorisation: (n-1)^4."""
    return float((n - 1) ** 4)


def factor_entries(n, dtype):
    """Entries of the stored factor per sample: m diagonal blocks of the
    block-tridiagonal LDL^T, each the symmetric inverse Schur complement of
    size n (padded), stored as its lower tr x tr tiles (16 x 16 MFMA tiles
    on every grid for the low-precision factors, at n = 16 and from n = 64
    for FP64)."""
    m = n - 1
    blk = n >= (64 if dtype == "f64" else 16) or n == 16
    tr = 16 if blk else (2 if n <= 16 else 4)
    tn = n // tr
    return m * tn * (tn + 1) // 2 * tr * tr


def refine_bytes(n, trips, dtype):
    """Algorithmic HBM bytes per sample of the refinement kernel: each of the
    `trips` corrections reads the factor twice (forward and backward block
    sweeps); the initial solve reads it not at all where the factorisation
    ran both sweeps (n = 16, and the low-precision factors' twisted layouts
    at n = 32..128), once where it ran the forward sweep (the low-precision
    factors elsewhere) and twice for FP64; each solve also the row couplings
    and scaling; every residual (1 + trips) reads the nodal coefficient and
    the iterate; x is written."""
    m = n - 1
    N = m * n
    f_pass = factor_entries(n, dtype) * DT_BYTES[dtype]
    if n == 16 or (dtype != "f64" and n <= 128):
        initial = 0
    else:
        initial = (1 if dtype != "f64" else 2) * f_pass + 3 * N * 8
    per_corr = 2 * f_pass + 3 * N * 8
    per_resid = (n + 1) ** 2 * 8 + N * 8
    return initial + trips * per_corr + (1 + trips) * per_resid + N * 8


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="mlmc4_n16-128_K64")
    p.add_argument("--dtype", default="f32")
    p.add_argument("--graph", action="store_true",
                   help="time the step as one replayed HIP graph (two streams per level) instead of the "
                        "eager one-stream-per-hardware-queue schedule")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-fp64", action="store_true")
    p.add_argument("--no-per-level", action="store_true")
    p.add_argument("--no-autotune", action="store_true",
                   help="skip the autotuner (refinement waves per row pair, FP16/BF16 product precision)")
    p.add_argument("--ttr-tol", type=float, default=2e-5,
                   help="absolute tolerance of the time-to-RMSE leg (0 skips it)")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--ttr-runs", type=int, default=20, help="seeds of the time-to-RMSE leg")
    p.add_argument("--legs", default="c0,c2,c3,c4,q43,paper5,paper_iterative,mlmcmc,mimc",
                   help="comma-separated other-workload legs to run (empty: none)")
    p.add_argument("--q43-runs", type=int, default=1000, help="runs of the quarter-precision leg")
    p.add_argument("--paper5-runs", type=int, default=300, help="runs of the Table 1 precision leg")
    p.add_argument("--copy-probe-mib", type=int, default=0,
                   help="run one plain streaming kernel (y = 2x, FP32) over this many MiB first; "
                        "its HBM counters calibrate the kernel traffic counters")
    return p.parse_args()


def log(*a):
    print("bench:", *a, flush=True)


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _ctx_for(wname, **over):
    import seeded_inputs as si
    from paper_2503_05533_amd import MLMC, Config
    w = si.workload(wname)
    kw = dict(n0=w["n0"], L_max=max(w["levels"]), K=w["K"], sigma2=w["sigma2"], corr_len=w["corr_len"],
              seed=w["seed"], ir_max_iter=10, field=w.get("field", 0), field_q=w.get("field_q", 2.0),
              k_p=w.get("k_p", 0.05), disc=w.get("disc", 0))
    kw.update(over)
    return w, MLMC(Config(**kw), device="cuda:0")


def _event_ms(fn, reps=2):
    """Device time of fn() (one untimed call first), mean over reps."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def _ci95_mse(err):
    """MSE of the errors and a 95% bootstrap interval (2000 resamples)."""
    import numpy as np
    err = np.asarray(err, dtype=float)
    mse = float(np.mean(err ** 2))
    rng = np.random.default_rng(12345)
    bs = np.mean(err[rng.integers(0, len(err), size=(2000, len(err)))] ** 2, axis=1)
    return mse, [float(np.quantile(bs, 0.025)), float(np.quantile(bs, 0.975))]


def leg_time_to_rmse(ctx, a, L, seed0):
    """Algorithm 4.1 at TOL over R seeds, mixed and FP64 with the same seed per
    run (shared xi); the reference is one FP64 run at TOL/5 with a seed of its
    own.  Reports the median host wall time per run and the achieved RMSE
    against the reference with a 95% bootstrap interval."""
    import numpy as np
    tol, R = a.ttr_tol, a.ttr_runs
    out = dict(tol=tol, runs=R)
    ctx.set_seed(seed0 + 7777)
    ref = ctx.estimate(tol / 5, n_init=1000, dtypes=["f64"] * (L + 1), solver="direct", mixed=False)
    out["reference"] = dict(tol=tol / 5, estimate=ref["estimate"], rmse_est=ref["var_est"] ** 0.5, N=ref["N"],
                            L=ref["L"])
    paths = [("mixed", [a.dtype] * (L + 1), "direct_ir", True)]
    if not a.no_fp64:
        paths.append(("fp64", ["f64"] * (L + 1), "direct", False))
    for name, d, solver, mixed in paths:
        ctx.set_seed(seed0)
        ctx.estimate(tol, n_init=1000, dtypes=d, solver=solver, mixed=mixed)  # allocates the workspace
        walls, ests, Ls, N0 = [], [], [], []
        for r in range(R):
            ctx.set_seed(seed0 + r)
            res = ctx.estimate(tol, n_init=1000, dtypes=d, solver=solver, mixed=mixed)
            walls.append(res["wall_s"])
            ests.append(res["estimate"])
            Ls.append(res["L"])
            N0.append(res["N"][0])
        mse, ci = _ci95_mse(np.array(ests) - ref["estimate"])
        out[name] = dict(median_wall_s=float(np.median(walls)), min_wall_s=float(np.min(walls)),
                         rmse=mse ** 0.5, rmse_ci95=[ci[0] ** 0.5, ci[1] ** 0.5],
                         rmse_over_tol=mse ** 0.5 / tol, L_counts={str(k): Ls.count(k) for k in sorted(set(Ls))},
                         mean_N0=float(np.mean(N0)))
        log("time to RMSE %s" % name, out[name])
    ctx.set_seed(seed0)
    if "fp64" in out:
        out["speedup"] = out["fp64"]["median_wall_s"] / out["mixed"]["median_wall_s"]
    return out


def leg_c0(a):
    """single_n32_K16: one level, n = 32, K = 16, 1000 samples; FP64 direct
    (and the FP32 factor with FP64 refinement to 1e-10), xi drawn in the step."""
    w, ctx = _ctx_for("single_n32_K16")
    N = w["N"][0]
    xi = ctx.fill_xi(0, 0, N)
    out = dict(workload="single_n32_K16", N=N)
    for name, o in (("fp64", dict(dtype="f64", solver="direct")),
                    ("mixed_f32_ir_1e-10", dict(dtype="f32", solver="direct_ir", eps_fine=1e-10))):
        plan = ctx.plan_levels([0], [xi], [o], use_graph=False)

        def run():
            ctx.fill_xi(0, 0, N, out=xi)
            plan.run()
        ms = _event_ms(run, reps=5)
        out[name] = dict(ms=ms, samples_per_s=N / (ms / 1e3))
    ctx.close()
    return out


def leg_c2(a):
    """sweep5_n16-256_K128: each level alone with each factor precision
    (FP32, BF16, FP16 with FP64 refinement to delta_l; FP64 direct):
    samples/s, promotions and mean corrections per level."""
    w, ctx = _ctx_for("sweep5_n16-256_K128")
    L = max(w["levels"])
    eps = ctx.accuracy_targets(L)
    out = dict(workload="sweep5_n16-256_K128", eps=eps, levels={})
    for l, N in zip(w["levels"], w["N"]):
        xi = ctx.fill_xi(l, 0, N)
        row = {}
        for dt in ("f64", "f32", "bf16", "f16"):
            o = dict(dtype=dt, solver="direct" if dt == "f64" else "direct_ir", eps_fine=eps[l],
                     eps_coarse=eps[l - 1] if l else 0.0)
            tuned = None if (a.no_autotune or dt == "f64") else ctx.autotune(l, xi, **o)
            plan = ctx.plan_levels([l], [xi], [o], use_graph=False)
            ms = _event_ms(plan.run, reps=2)
            st = plan.run(stats=True)["stats"][0]
            row[dt] = dict(ms=ms, samples_per_s=N / (ms / 1e3), promoted=st["n_promoted"],
                           noconv=st["n_noconv"], mean_corrections=st["mean_iters"],
                           mean_corrections_coarse=st["mean_iters_coarse"], autotuned=tuned)
            del plan
        best = min((d for d in ("f32", "bf16", "f16") if row[d]["noconv"] == 0), key=lambda d: row[d]["ms"])
        row["fastest_mixed"] = best
        row["speedup_vs_fp64"] = row["f64"]["ms"] / row[best]["ms"]
        out["levels"][str(ctx.level_cells(l))] = row
        del xi
    ctx.close()
    return out


def leg_c3(a):
    """batched5_n16-256_K128: all five levels (40000 ... 200 samples) as one
    replayed HIP graph, FP32 factor + FP64 refinement against batched MINRES
    (FP64), MINRES-IR (FP32 inner vectors) and multigrid-preconditioned CG
    (the gamma = 2 solver), all to delta_l; and the eager schedule for the
    refinement path."""
    w, ctx = _ctx_for("batched5_n16-256_K128", minres_max_iter=20000)
    levels, Ns = w["levels"], w["N"]
    L = max(levels)
    eps = ctx.accuracy_targets(L)
    xis = [ctx.fill_xi(l, 0, N) for l, N in zip(levels, Ns)]
    out = dict(workload="batched5_n16-256_K128", N=Ns, eps=eps)
    for name, solver, graph in (("direct_ir_graph", "direct_ir", True), ("direct_ir_eager", "direct_ir", False),
                                ("minres_graph", "minres", True), ("minres_ir_graph", "minres_ir", True),
                                ("mgcg_graph", "mgcg", True)):
        o = [dict(dtype="f32", solver=solver, eps_fine=eps[l], eps_coarse=eps[l - 1] if l else 0.0)
             for l in levels]
        plan = ctx.plan_levels(levels, xis, o, use_graph=graph)
        ms = _event_ms(plan.run, reps=3)
        st = plan.run(stats=True)["stats"]
        out[name] = dict(ms=ms, samples_per_s=sum(Ns) / (ms / 1e3),
                         mean_iters=[x["mean_iters"] for x in st], noconv=[x["n_noconv"] for x in st],
                         promoted=[x["n_promoted"] for x in st])
        del plan
    out["direct_ir_vs_minres"] = out["minres_graph"]["ms"] / out["direct_ir_graph"]["ms"]
    out["minres_ir_vs_minres"] = out["minres_graph"]["ms"] / out["minres_ir_graph"]["ms"]
    out["mgcg_vs_direct_ir"] = out["direct_ir_graph"]["ms"] / out["mgcg_graph"]["ms"]
    ctx.close()
    return out


def leg_c4(a):
    """adjoint_n128_K128: dQ/dxi for 4096 samples at n = 128 (FP32 factor
    reused by the adjoint, FP64 refinement): the forward solve and the
    adjoint, at 1e-10 and at 1e-5."""
    import torch
    w, ctx = _ctx_for("adjoint_n128_K128")
    N = w["N"][0]
    xi = ctx.fill_xi(0, 0, N)
    out = dict(workload="adjoint_n128_K128", N=N)
    for eps in (1e-10, 1e-5):
        fw = ctx.solve(0, xi, dtype="f32", solver="direct_ir", eps=eps, promote=True, own_workspace=True)
        ms_f = _event_ms(lambda: ctx.solve(0, xi, dtype="f32", solver="direct_ir", eps=eps, promote=True),
                         reps=2)
        fw = ctx.solve(0, xi, dtype="f32", solver="direct_ir", eps=eps, promote=True, own_workspace=True)
        ws = fw["ws"]
        ms_g = _event_ms(lambda: ctx.grad_from(0, xi, ws, None, eps_adjoint=eps, dtype="f32",
                                               solver="direct_ir", eps=eps), reps=2)
        out["eps_%g" % eps] = dict(forward_ms=ms_f, adjoint_ms=ms_g,
                                   gradients_per_s=N / ((ms_f + ms_g) / 1e3))
        del fw, ws
        torch.cuda.synchronize()
    ctx.close()
    return out


def stored_bytes(n, dtype, trips):
    """Bytes of the factor and the vectors one solve computes and stores
    (the paper's memory-reference count of sec. 5.2, each entry at the
    precision this library stores it in): the stored factor, plus the FP64
    vectors z and x of the initial solve and r, z, x of every correction
    (FP64 direct: z and x)."""
    b = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2, "fp8": 1}[dtype]
    m = n - 1
    vec = m * n
    return factor_entries(n, dtype if dtype in DT_BYTES else "f32") * b + vec * 8 * (2 + 3 * trips)


def _paper_leg(a, wname, dts_of, vec_bytes_of, tol2, n_init, runs):
    """The paper's fixed-sample comparison (sec. 5.2): N_l from one standard
    (FP64) adaptive run at TOL^2 = tol2; then `runs` runs with those N_l, run r
    drawing samples r*N_l ... of each level, shared by the mixed path (factor
    precision dts_of(L)[l], FP64 refinement to delta_l) and the FP64 direct
    path; the MSE of both against an FP64 reference (adaptive at TOL/10,
    seed of its own), their relative difference, and the stored-bytes count
    (stored_bytes) with this library's vector precisions and with the
    paper's (vec_bytes_of(L)[l] bytes per vector entry)."""
    import numpy as np
    w, ctx = _ctx_for(wname)
    Lm = max(w["levels"])
    tol = tol2 ** 0.5
    ctx.set_seed(w["seed"] + 1)
    ref = ctx.estimate(tol / 10, n_init=n_init, dtypes=["f64"] * (Lm + 1), solver="direct", mixed=False)
    ctx.set_seed(w["seed"])
    std = ctx.estimate(tol, n_init=n_init, dtypes=["f64"] * (Lm + 1), solver="direct", mixed=False)
    Lr, N = std["L"], std["N"]
    eps = ctx.accuracy_targets(Lr)
    dts = dts_of(Lr)
    est = {"mixed": [], "fp64": []}
    trips = np.zeros((Lr + 1, 2))
    promoted = np.zeros(Lr + 1, dtype=np.int64)
    noconv = {"mixed": 0, "fp64": 0}
    gpu_ms = {"mixed": 0.0, "fp64": 0.0}
    for r in range(runs):
        q = {"mixed": 0.0, "fp64": 0.0}
        for l in range(Lr + 1):
            xi = ctx.fill_xi(l, r * N[l], N[l])
            for name, o in (("mixed", dict(dtype=dts[l], solver="direct_ir", eps_fine=eps[l],
                                           eps_coarse=eps[l - 1] if l else 0.0)),
                            ("fp64", dict(dtype="f64", solver="direct"))):
                st = ctx.sample_level(l, xi, **o)["stats"]
                noconv[name] += st["n_noconv"]
                q[name] += st["sum_y"] / N[l]
                gpu_ms[name] += st["gpu_ms"]
                if name == "mixed":
                    trips[l] += (st["mean_iters"], st["mean_iters_coarse"])
                    promoted[l] += st["n_promoted"]
        for k in q:
            est[k].append(q[k])
    out = dict(workload=wname, disc=w.get("disc", 0), tol2=tol2, runs=runs, n_init=n_init, N=N, L=Lr,
               eps=eps, precision=dts, reference=dict(tol=tol / 10, estimate=ref["estimate"], N=ref["N"]))
    for k in est:
        mse, ci = _ci95_mse(np.array(est[k]) - ref["estimate"])
        out[k] = dict(mse=mse, mse_ci95=ci, gpu_ms_per_run=gpu_ms[k] / runs)
    d = np.array(est["mixed"]) - np.array(est["fp64"])
    out["mse_rel_diff"] = out["mixed"]["mse"] / out["fp64"]["mse"] - 1.0
    out["max_abs_estimate_diff"] = float(np.max(np.abs(d)))
    out["promoted_per_level"] = promoted.tolist()
    out["noconv"] = noconv
    mean_trips = trips / runs
    out["mean_corrections"] = mean_trips.tolist()
    # stored bytes per level: the fine and the coarse solve of every Y_l sample
    vb = vec_bytes_of(Lr)
    fbytes = {"fp8": 1, "f16": 2, "bf16": 2, "f32": 4}
    by_m, by_d, by_p = [], [], []
    for l in range(Lr + 1):
        nf = w["n0"] << l
        grids = [(nf, mean_trips[l][0])] + ([(nf // 2, mean_trips[l][1])] if l else [])
        bm = sum(stored_bytes(nn, dts[l], t) for nn, t in grids)
        bd = sum(stored_bytes(nn, "f64", 0) for nn, _ in grids)
        bp = sum(factor_entries(nn, "f32") * fbytes[dts[l]] + (nn - 1) * nn * vb[l] * (2 + 3 * t) for nn, t in grids)
        by_m.append(N[l] * bm)
        by_d.append(N[l] * bd)
        by_p.append(N[l] * bp)
    out["stored_bytes_ratio_per_level"] = [x / y for x, y in zip(by_d, by_m)]
    out["stored_bytes_ratio_total"] = sum(by_d) / sum(by_m)
    out["stored_bytes_ratio_paper_precisions_per_level"] = [x / y for x, y in zip(by_d, by_p)]
    out["stored_bytes_ratio_paper_precisions"] = sum(by_d) / sum(by_p)
    ctx.close()
    return out


def leg_q43(a):
    """The paper's quarter-precision example (sec. 5.2, last paragraph): P1
    elements, h0 = 1/4 (4..32 cells), trigonometric field s = 1, sigma = 1,
    k_p = 0.4, TOL^2 = 2e-6; level 0 `qhhh` -> FP8 factor, levels 1-3 `hhss`
    -> FP16 factor; the paper's vectors: half on level 0, single above."""
    return _paper_leg(a, "q43_n4-32_trig1", lambda L: ["fp8"] + ["f16"] * L, lambda L: [2] + [4] * L,
                      2e-6, 100, a.q43_runs)


def leg_paper5(a):
    """The paper's direct-solver example (sec. 5.2): P1 elements, h0 = 1/8,
    trigonometric field s = 4, q = 2, sigma = 2, k_p = 0.05, TOL^2 = 2e-6; the
    precisions of Table 1 (right): level 0 `hhss` -> FP16 factor, level 1
    `ssss` -> FP32, levels 2+ `ssdd` -> FP32; the paper's vectors: single on
    levels 0-1, double from level 2."""
    return _paper_leg(a, "paper5_n8-128_trig4", lambda L: ["f16", "f32"] + ["f32"] * (L - 1),
                      lambda L: [4, 4] + [8] * (L - 1), 2e-6, 100, a.paper5_runs)


def leg_paper_iterative(a):
    """The paper's iterative-solver comparison (sec. 5.1): adaptive MPML
    (Algorithm 4.1 with its accuracy targets delta_l) against standard MLMC
    (every solve to a fixed relative residual 1e-6) with the same iterative
    solver, on the paper's first example (P1 elements, trigonometric field
    s = 4, q = 2, sigma = 2, h0 = 1/8, k_p = 0.05), at TOL^2 = 8e-6 and 2e-6,
    10 seeds each (MPML and MLMC share each seed's xi): median host wall
    time, mean device time, the cost ratio MLMC / MPML (the paper reports
    ~1.5x in FLOPs with MINRES), and the RMSE of both against an FP64 direct
    reference at TOL/10; for FP64 MINRES and for multigrid CG."""
    import numpy as np
    w, ctx = _ctx_for("paper5_n8-128_trig4", minres_max_iter=20000)
    Lm = max(w["levels"])
    out = dict(workload="paper5_n8-128_trig4", std_eps=1e-6, runs=10)
    ctx.set_seed(w["seed"] + 99)
    tol_min = (2e-6) ** 0.5
    ref = ctx.estimate(tol_min / 10, n_init=100, dtypes=["f64"] * (Lm + 1), solver="direct", mixed=False)
    out["reference"] = dict(estimate=ref["estimate"], tol=tol_min / 10)
    for solver in ("minres", "mgcg"):
        res_s = {}
        for tol2 in (8e-6, 2e-6):
            tol = tol2 ** 0.5
            row = {}
            for name, mixed in (("mpml", True), ("mlmc", False)):
                ctx.set_seed(w["seed"])
                ctx.estimate(tol, n_init=100, dtypes=["f64"] * (Lm + 1), solver=solver, mixed=mixed)
                walls, gms, ests, Ls = [], [], [], []
                for r in range(10):
                    ctx.set_seed(w["seed"] + r)
                    e = ctx.estimate(tol, n_init=100, dtypes=["f64"] * (Lm + 1), solver=solver, mixed=mixed)
                    walls.append(e["wall_s"])
                    gms.append(e["gpu_ms"])
                    ests.append(e["estimate"])
                    Ls.append(e["L"])
                mse, ci = _ci95_mse(np.array(ests) - ref["estimate"])
                row[name] = dict(median_wall_s=float(np.median(walls)), mean_gpu_ms=float(np.mean(gms)),
                                 rmse=mse ** 0.5, L_counts={str(k): Ls.count(k) for k in sorted(set(Ls))})
            row["wall_ratio_mlmc_over_mpml"] = row["mlmc"]["median_wall_s"] / row["mpml"]["median_wall_s"]
            row["gpu_ratio_mlmc_over_mpml"] = row["mlmc"]["mean_gpu_ms"] / row["mpml"]["mean_gpu_ms"]
            res_s["tol2_%g" % tol2] = row
        out[solver] = res_s
    ctx.close()
    return out


def leg_mlmcmc(a):
    """Multilevel MCMC (mlmc_mcmc) on the paper's first example (P1
    elements, trigonometric field s = 4, q = 2, sigma = 2, h0 = 1/8, levels
    8/16/32 cells): data at nine interior nodes from a fixed parameter, noise
    1e-3; 1024 chains per level, 100/60/40 recorded steps after 20 of burn-in,
    the coarse chain subsampled 10 times with pCN step 0.8; FP64 direct solves
    against FP32 factors refined to the accuracy targets: wall time, device
    solves, the estimate and its standard error, acceptance rates."""
    import numpy as np
    import torch
    w, ctx = _ctx_for("paper5_n8-128_trig4")
    L, C = 2, 1024
    n_t = 64
    xs = [0.25, 0.5, 0.75]
    truth = torch.tensor([[0.6, -0.8, 0.5, -0.3]], dtype=torch.float64)
    # data from a fixed parameter on a finer grid of the same library (FP64)
    wt, ctx_t = _ctx_for("paper5_n8-128_trig4", n0=n_t, L_max=0)
    out_t = ctx_t.solve(0, truth, dtype="f64", solver="direct", want_u=True)
    u = out_t["u"].cpu().numpy()[0]
    ctx_t.close()
    obs = [(x, y, float(u[(round(y * n_t) - 1) * (n_t - 1) + round(x * n_t) - 1])) for y in xs for x in xs]
    eps = ctx.accuracy_targets(L)
    runs = {}
    for name, opts in (("fp64", [dict(dtype="f64", solver="direct")] * (L + 1)),
                       ("mixed", [dict(dtype="f32", solver="direct_ir", eps_fine=eps[l],
                                       eps_coarse=eps[l - 1] if l else 0.0) for l in range(L + 1)])):
        ctx.mcmc(L, 64, [4, 4, 4], obs, 1e-3, burn_in=2, subsample=2, pcn_beta=0.8, opts=opts)  # warm-up
        r = ctx.mcmc(L, C, [100, 60, 40], obs, 1e-3, burn_in=20, subsample=10, pcn_beta=0.8, opts=opts)
        r["se"] = float(np.sqrt(sum(r["var_mean"])))
        runs[name] = r
    ctx.close()
    runs["speedup"] = runs["fp64"]["wall_s"] / runs["mixed"]["wall_s"]
    runs["estimate_diff_over_se"] = abs(runs["mixed"]["estimate"] - runs["fp64"]["estimate"]) / runs["fp64"]["se"]
    runs["chains"] = C
    return runs


def leg_mimc(a):
    """Multi-index Monte Carlo (mlmc_mimc) on the step's field and grids: index
    l the grid (16 to 128 cells), index k the field truncated to 16 2^k of its
    64 modes, the total-degree set l + k <= 3 (9 indices) with
    N = 20000 4^-l 2^-k samples; FP64 direct solves against FP32 factors
    refined to the accuracy targets (grid l to delta_l): wall time of the
    second of two identical calls, the estimate and its standard error, the
    per-index means, device solves and convergence counts."""
    import numpy as np
    w, ctx = _ctx_for("mlmc4_n16-128_K64")
    L, K0 = 3, 16
    idx = [(l, k) for l in range(L + 1) for k in range(3) if l + k <= L]
    N = [int(round(20000 * 4.0 ** (-l) * 2.0 ** (-k))) for l, k in idx]
    eps = ctx.accuracy_targets(L)
    runs = {"indices": idx, "N": N, "K0": K0}
    for name, opts in (("fp64", [dict(dtype="f64", solver="direct")] * len(idx)),
                       ("mixed", [dict(dtype="f32", solver="direct_ir", eps_fine=eps[l],
                                       eps_coarse=eps[l - 1] if l else 0.0) for l, _ in idx])):
        ctx.mimc(idx, N, K0, opts=opts)
        r = ctx.mimc(idx, N, K0, opts=opts)
        r["se"] = float(np.sqrt(r["var_estimate"]))
        runs[name] = r
    ctx.close()
    runs["speedup"] = runs["fp64"]["wall_s"] / runs["mixed"]["wall_s"]
    runs["estimate_diff_over_se"] = abs(runs["mixed"]["estimate"] - runs["fp64"]["estimate"]) / runs["fp64"]["se"]
    return runs


def cpu_single_and_lapack(oracle, si, w, ctx, levels, Ns, phis, budget):
    """One-core oracle time and LAPACK's banded Cholesky (dpbtrf/dpbtrs via
    SciPy, on the band matrices the oracle assembles; the assembly is not
    timed) on bounded samples, scaled to the workload like the main line."""
    import numpy as np
    import scipy.linalg as sl
    nthr = oracle.num_threads()
    K = w["K"]
    t1, tl, desc = [], [], []
    per = budget / len(levels)
    for l, N in zip(levels, Ns):
        nf = ctx.level_cells(l)
        grids = [nf, nf // 2] if l > 0 else [nf]
        # one core
        oracle.set_threads(1)
        xi = si.splitmix64_normals(w["seed"], l, 0, 1, K)
        t0 = time.perf_counter()
        for nn in grids:
            oracle.solve_batch(nn, phis[nn], xi)
        dt = time.perf_counter() - t0
        s = int(max(1, min(N, per / 2 / max(dt, 1e-9))))
        xi = si.splitmix64_normals(w["seed"], l, 0, s, K)
        t0 = time.perf_counter()
        for nn in grids:
            oracle.solve_batch(nn, phis[nn], xi)
        t1.append((time.perf_counter() - t0) / s)
        oracle.set_threads(nthr)
        # LAPACK banded Cholesky, one process
        s2 = max(1, min(s, 64))
        tt = 0.0
        for k in range(s2):
            for nn in grids:
                ab = oracle.band_matrix(nn, phis[nn], xi[k:k + 1])
                b = np.full(ab.shape[1], 1.0 / nn ** 2)
                t0 = time.perf_counter()
                sl.solveh_banded(ab, b, lower=True, check_finite=False)
                tt += time.perf_counter() - t0
        tl.append(tt / s2)
        desc.append("%d/%d" % (s, N))
    total = float(sum(Ns))
    return dict(single_core_value=total / sum(t * N for t, N in zip(t1, Ns)),
                lapack_band_value=total / sum(t * N for t, N in zip(tl, Ns)),
                lapack_band_kind="scipy.linalg.solveh_banded (LAPACK dpbtrf/dpbtrs), one process",
                single_core_sample="oracle with one thread on the first %s samples per level" % ",".join(desc))


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: the path runs on one GPU; --gpus %d is not supported "
              "(samples are independent: see the sharding notes in the design document)" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    import seeded_inputs as si
    from paper_2503_05533_amd import MLMC, Config

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if a.copy_probe_mib:
        x = torch.rand(a.copy_probe_mib << 18, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        torch.mul(x, 2.0, out=y)
        torch.cuda.synchronize()
        log("copy probe: %d MiB read, %d MiB written" % (a.copy_probe_mib, a.copy_probe_mib))
        del x, y
    w = si.workload(a.workload)
    levels, Ns, K = w["levels"], w["N"], w["K"]
    L = max(levels)
    cfg = Config(n0=w["n0"], L_max=L, K=K, sigma2=w["sigma2"], corr_len=w["corr_len"],
                 seed=w["seed"], ir_max_iter=10)
    ctx = MLMC(cfg, device="cuda:0")
    eps = ctx.accuracy_targets(L)
    cells = [ctx.level_cells(l) for l in levels]
    log("workload %s cells %s N %s eps %s" % (a.workload, cells, Ns, ["%.3e" % e for e in eps]))
    xis = [ctx.fill_xi(l, 0, N) for l, N in zip(levels, Ns)]
    torch.cuda.synchronize()

    def opts(dtype, solver):
        return [dict(dtype=dtype, solver=solver, eps_fine=eps[l],
                     eps_coarse=eps[l - 1] if l > 0 else 0.0) for l in levels]

    om, o64 = opts(a.dtype, "direct_ir"), opts("f64", "direct")
    tuned = None
    if not a.no_autotune:
        tuned = {cells[i]: ctx.autotune(l, xis[i], **{k: v for k, v in om[i].items() if k != "promote"})
                 for i, l in enumerate(levels)}
        log("autotuned (fine, coarse): waves per row pair | fp32 products << 4", tuned)
    total = float(sum(Ns))

    def step(plan):
        # a step draws every level's xi into the plan's input buffers, then
        # runs all levels (both on the current stream's order)
        for i, l in enumerate(plan.levels):
            ctx.fill_xi(l, 0, plan.xis[i].shape[0], out=plan.xis[i])
        plan.run()

    def timed(plan, steps, warmup):
        for _ in range(warmup):
            step(plan)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step(plan)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    # ---- mixed path: the timed leg (the concurrent step)
    plan_m = ctx.plan_levels(levels, xis, om, use_graph=a.graph)
    ms_mixed = timed(plan_m, a.steps, a.warmup)
    value = total / (ms_mixed / 1e3)
    log("mixed %.3f ms/step, %.4g samples/s" % (ms_mixed, value))
    st_m = ctx.plan_levels(levels, xis, om, use_graph=False).run(stats=True)["stats"]

    # ---- profiled leg: the same concurrent step launched eagerly
    eager = ctx.plan_levels(levels, xis, om, use_graph=False)
    step(eager)
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step(eager)
    torch.cuda.synchronize()
    ms_eager = (time.perf_counter() - t0) * 1e3 / a.steps
    prof = {}
    grids = sorted(set(cells + [c // 2 for c in cells if c > w["n0"]]))
    for kind in ctx.KINDS:
        for n in grids:
            r = ctx.profile_read(kind, n)
            if r["launches"]:
                prof[(kind, n)] = r
    ctx.profile(False)

    # mean corrections per grid (fine and coarse uses weighted by samples)
    trips = {}
    for i, l in enumerate(levels):
        for n, t in [(cells[i], st_m[i]["mean_iters"])] + \
                    ([(cells[i] // 2, st_m[i]["mean_iters_coarse"])] if l > 0 else []):
            s0, t0_ = trips.get(n, (0, 0.0))
            trips[n] = (s0 + Ns[i], t0_ + Ns[i] * t)
    trips = {n: v[1] / v[0] for n, v in trips.items()}

    # ---- roofline of the dominant kernel of the mixed step: the longest
    # launch (the levels run concurrently, and the step's critical path runs
    # through its longest kernel)
    (kind, n), r = max(prof.items(), key=lambda kv: kv[1]["ms"] / kv[1]["launches"])
    avg_ms = r["ms"] / r["launches"]
    per_launch = r["samples"] / r["launches"]
    if kind == "factor":
        work = factor_flops(n) * per_launch
        achieved = work / (avg_ms * 1e-3) / 1e12
        peak = PEAK["f64"] if a.dtype == "f64" else PEAK["f32"]
        roof = dict(bound="mfma", achieved=achieved, peak=peak, unit="TFLOP/s", frac=achieved / peak,
                    traffic=None)
        per_unit = "%.4g flops per sample ((n-1)^4)" % factor_flops(n)
    else:
        per = refine_bytes(n, trips.get(n, 1.0), a.dtype)
        work = per * per_launch
        achieved = work / (avg_ms * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=achieved, peak=PEAK["hbm"], unit="GB/s",
                    frac=achieved / PEAK["hbm"], traffic=None)
        per_unit = "%.4g bytes per sample at %.3f mean corrections" % (per, trips.get(n, 1.0))
    tb = TRAFFIC.get((kind, n, a.dtype))
    if tb is not None and kernel_src_hash() == TRAFFIC_SRC:
        roof["traffic"] = tb * per_launch
        roof["traffic_unit"] = "bytes per launch (HBM, counters)"
    roof.update(kernel="%s n=%d" % (kind, n), avg_launch_ms=avg_ms, launches=r["launches"],
                samples_per_launch=per_launch, per_unit=per_unit)
    # The same kernel with its level running alone (in the step it shares the
    # CUs with the other levels' kernels): context for frac, not the figure.
    if n in cells:
        i_dom = cells.index(n)
        p1 = ctx.plan_levels([levels[i_dom]], [xis[i_dom]], [om[i_dom]], use_graph=False)
        p1.run()
        torch.cuda.synchronize()
        ctx.profile(True)
        for _ in range(3):
            p1.run()
        torch.cuda.synchronize()
        r1 = ctx.profile_read(kind, n)
        ctx.profile(False)
        del p1
        if r1["launches"]:
            alone_ms = r1["ms"] / r1["launches"]
            roof["alone_avg_launch_ms"] = alone_ms
            roof["alone_frac"] = roof["frac"] * avg_ms / alone_ms
    log("dominant kernel", roof)

    # ---- per-level throughput (each level alone)
    def per_level(o):
        out = []
        for i, l in enumerate(levels):
            p = ctx.plan_levels([l], [xis[i]], [o[i]], use_graph=False)
            p.run()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            p.run()
            e1.record()
            e1.synchronize()
            out.append(Ns[i] / (e0.elapsed_time(e1) / 1e3))
        return out

    lvl_m = None if a.no_per_level else per_level(om)

    # ---- FP64 path on the same workload
    fp64 = None
    if not a.no_fp64:
        plan_d = ctx.plan_levels(levels, xis, o64, use_graph=a.graph)
        ms64 = timed(plan_d, a.steps, a.warmup)
        log("fp64 %.3f ms/step" % ms64)
        fp64 = dict(ms_per_step=ms64, samples_per_s=total / (ms64 / 1e3),
                    per_level_samples_per_s=None if a.no_per_level else per_level(o64),
                    path="FP64 direct solves with the same block LDL^T (explicit inverse Schur "
                         "complements) kernels in FP64, no refinement; same schedule")
        del plan_d

    # ---- time to RMSE: Algorithm 4.1 at an absolute tolerance, R seeds
    ttr = None
    if a.ttr_tol > 0:
        ttr = leg_time_to_rmse(ctx, a, L, w["seed"])
    # ---- CPU baseline: the oracle on a bounded sample of the same workload
    cpu = None
    if not a.no_cpu:
        import oracle
        phis = {}
        t_per = []
        budget = a.cpu_seconds / len(levels)
        samples_desc = []
        for l, N in zip(levels, Ns):
            nf = ctx.level_cells(l)
            for nn in ([nf, nf // 2] if l > 0 else [nf]):
                if nn not in phis:
                    phis[nn] = oracle.kl_basis(nn, K, w["sigma2"], w["corr_len"])
            xi = si.splitmix64_normals(w["seed"], l, 0, min(N, 64), K)
            # probe, then size the sample to the per-level budget
            t0 = time.perf_counter()
            k = min(N, oracle.num_threads())
            oracle.solve_batch(nf, phis[nf], xi[:k])
            if l > 0:
                oracle.solve_batch(nf // 2, phis[nf // 2], xi[:k])
            dt = (time.perf_counter() - t0) / k
            s = int(max(1, min(N, budget / max(dt, 1e-9))))
            xi = si.splitmix64_normals(w["seed"], l, 0, s, K)
            t0 = time.perf_counter()
            oracle.solve_batch(nf, phis[nf], xi)
            if l > 0:
                oracle.solve_batch(nf // 2, phis[nf // 2], xi)
            t_per.append((time.perf_counter() - t0) / s)
            samples_desc.append("%d/%d" % (s, N))
        cpu_time = sum(t * N for t, N in zip(t_per, Ns))
        cpu = dict(value=total / cpu_time, unit="samples/s", cores=oracle.num_threads(), kind="oracle",
                   sample="FP64 banded Cholesky on the first %s samples of each level (fine+coarse), "
                          "per-sample time scaled to the full workload" % ",".join(samples_desc),
                   cpu_model=cpu_model())
        cpu.update(cpu_single_and_lapack(oracle, si, w, ctx, levels, Ns, phis, a.cpu_seconds / 3))
        log("cpu oracle", cpu)

    # ---- other workloads
    legs = {}
    sel = [x for x in a.legs.split(",") if x]
    ctx_main = ctx
    for name in sel:
        fn = {"c0": leg_c0, "c2": leg_c2, "c3": leg_c3, "c4": leg_c4, "q43": leg_q43, "paper5": leg_paper5,
              "paper_iterative": leg_paper_iterative, "mlmcmc": leg_mlmcmc, "mimc": leg_mimc}[name]
        t0 = time.perf_counter()
        legs[name] = fn(a)
        legs[name]["leg_wall_s"] = time.perf_counter() - t0
        log("leg %s" % name, legs[name])
        torch.cuda.empty_cache()
    ctx = ctx_main

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_mixed,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "xi_in_step": True,
        "config": {"workload": a.workload, "cells": cells, "N_l": Ns, "K": K,
                   "sigma2": w["sigma2"], "corr_len": w["corr_len"], "eps_l": eps,
                   "path": "%s factor + FP64 residual/refinement/sums, all levels concurrent, "
                           "%s" % (a.dtype, "one HIP graph per step" if a.graph else "eager, one stream per hardware queue")},
        "per_level_samples_per_s": lvl_m,
        "fp64": fp64,
        "speedup_vs_fp64": (value / fp64["samples_per_s"]) if fp64 else None,
        "mean_corrections": {str(k): v for k, v in sorted(trips.items())},
        "promoted": [s["n_promoted"] for s in st_m],
        "time_to_rmse": ttr,
        "roofline": roof,
        "eager_ms_per_step": ms_eager,
        "kernel_ms_per_step": {"%s_n%d" % k: v["ms"] / a.steps for k, v in sorted(prof.items())},
        "autotuned": tuned,
        "legs": legs,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
