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
    (the value);
  * profiled: the same K steps launched eagerly with HIP events around each
    kernel launch on its own stream (per-kernel device time; the roofline of
    the dominant kernel);
  * per level: each level alone, event-timed (samples/s per level);
  * FP64: the same timed leg with the FP64 direct path;
  * time to RMSE: Algorithm 4.1 (adaptive MLMC) to an absolute tolerance,
    mixed and FP64, wall time on the host of the second of two identical
    runs (the first allocates the estimator's workspace);
  * CPU: the FP64 oracle on a bounded sample of the workload, host cores.

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
DT_BYTES = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}


# HBM bytes per sample measured with FETCH_SIZE / WRITE_SIZE counters (scaled
# by a copy kernel of known size) for the mixed FP32 step; valid only while the
# kernel sources hash to TRAFFIC_SRC (otherwise the field is reported as null).
TRAFFIC_SRC = "80594da28cee6ab6"
TRAFFIC = {("factor", 128, "f32"): 5.2358e6, ("factor", 64, "f32"): 0.7834e6,
           ("factor", 32, "f32"): 0.1298e6, ("factor", 16, "f32"): 0.0467e6,
           ("solve", 128, "f32"): 17.0690e6, ("solve", 64, "f32"): 2.5307e6,
           ("solve", 32, "f32"): 0.1489e6, ("solve", 16, "f32"): 0.0052e6}


def kernel_src_hash():
    import hashlib
    d = os.path.join(ROOT, "paper_2503_05533_amd", "csrc")
    src = b"".join(open(os.path.join(d, f), "rb").read()
                   for f in ("factor_mfma.hip", "kernels.h", "dtypes.h", "ir_common.h"))
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
    sweeps), the initial solve once where the factorisation ran the forward
    sweep (the low-precision factors, and FP64 at n = 16) and twice for
    FP64 elsewhere, each solve also the row couplings and scaling; every
    residual (1 + trips) reads the nodal coefficient and the iterate; x is
    written."""
    m = n - 1
    N = m * n
    f_pass = factor_entries(n, dtype) * DT_BYTES[dtype]
    fused = dtype != "f64" or n == 16
    initial = (1 if fused else 2) * f_pass + 3 * N * 8
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
    p.add_argument("--autotune", action="store_true")
    p.add_argument("--ttr-tol", type=float, default=2e-5,
                   help="absolute tolerance of the time-to-RMSE leg (0 skips it)")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--copy-probe-mib", type=int, default=0,
                   help="run one plain streaming kernel (y = 2x, FP32) over this many MiB first; "
                        "its HBM counters calibrate the kernel traffic counters")
    return p.parse_args()


def log(*a):
    print("bench:", *a, flush=True)


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
    if a.autotune:
        tuned = {cells[i]: ctx.autotune(l, xis[i], **{k: v for k, v in om[i].items() if k != "promote"})
                 for i, l in enumerate(levels)}
        log("autotuned refinement variants", tuned)
    total = float(sum(Ns))

    def timed(plan, steps, warmup):
        for _ in range(warmup):
            plan.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.run()
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
    eager.run()
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(a.steps):
        eager.run()
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

    # ---- roofline of the dominant kernel of the mixed step
    (kind, n), r = max(prof.items(), key=lambda kv: kv[1]["ms"])
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
                    per_level_samples_per_s=None if a.no_per_level else per_level(o64))
        del plan_d

    # ---- time to RMSE: Algorithm 4.1 at an absolute tolerance
    ttr = None
    if a.ttr_tol > 0:
        dts = [a.dtype] * (L + 1)
        ttr = dict(tol=a.ttr_tol)
        runs = [("mixed", dts, "direct_ir", True)]
        if not a.no_fp64:
            runs.append(("fp64", ["f64"] * (L + 1), "direct", False))
        for name, d, solver, mixed in runs:
            # one untimed run first: the estimator's workspace (tens of GB)
            # is allocated on the first call and kept by the context
            ctx.estimate(a.ttr_tol, n_init=1000, dtypes=d, solver=solver, mixed=mixed)
            res = ctx.estimate(a.ttr_tol, n_init=1000, dtypes=d, solver=solver, mixed=mixed)
            ttr[name] = dict(wall_s=res["wall_s"], gpu_ms=res["gpu_ms"], estimate=res["estimate"],
                             rmse_est=res["var_est"] ** 0.5, L=res["L"], N=res["N"],
                             converged=res["converged"])
            log("time to RMSE %s" % name, ttr[name])
        if "fp64" in ttr:
            ttr["speedup"] = ttr["fp64"]["wall_s"] / ttr["mixed"]["wall_s"]

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
                          "per-sample time scaled to the full workload" % ",".join(samples_desc))
        log("cpu oracle", cpu)

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
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
