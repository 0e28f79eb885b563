"""Benchmark of the batched per-level sample solve on one MI355X.

A step is one pass of the whole hot path over one batch: for every level l
of the workload, N_l samples, each a fine solve on grid l and (l >= 1) a
coarse solve on grid l-1 from the same xi row, paired into Y_l, with the
level sums.  The mixed path factorises in FP32 and refines in FP64 to the
level accuracy delta_l of the adaptive rule; the FP64 path factorises and
solves in FP64.  Inputs (xi) are resident in HBM before the timed region.

Prints one JSON line (rank 0).  --gpus N > 1 is refused: this build runs on
one GPU.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PDE samples/s per level + MLMC time-to-RMSE, mixed+IR vs FP64 on same GPU"
PEAK = {"f64_alu": 78.6, "f32_alu": 157.3, "hbm": 8000.0}  # TFLOP/s, TFLOP/s, GB/s


def factor_flops(n):
    """Algorithmic flops of one grid factorisation: (n-1)^4."""
    return float((n - 1) ** 4)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--workload", default="mlmc4_n16-128_K64")
    p.add_argument("--dtype", default="f32")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-fp64", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    return p.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    import seeded_inputs as si
    from paper_2503_05533_amd import MLMC, Config

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    w = si.workload(a.workload)
    levels, Ns, K = w["levels"], w["N"], w["K"]
    L = max(levels)
    cfg = Config(n0=w["n0"], L_max=L, K=K, sigma2=w["sigma2"], corr_len=w["corr_len"],
                 seed=w["seed"], ir_max_iter=10)
    ctx = MLMC(cfg, device="cuda:0")
    eps = ctx.accuracy_targets(L)
    cells = [ctx.level_cells(l) for l in levels]
    print("bench: workload %s levels %s N %s eps %s" % (a.workload, cells, Ns, eps), flush=True)
    xis = [ctx.fill_xi(l, 0, N) for l, N in zip(levels, Ns)]
    torch.cuda.synchronize()

    def step(dtype, solver):
        out = []
        for l, N, xi in zip(levels, Ns, xis):
            r = ctx.sample_level(l, xi, dtype=dtype, solver=solver, eps_fine=eps[l],
                                 eps_coarse=eps[l - 1] if l > 0 else 0.0, stats=False)
            out.append(r)
        return out

    def timed(dtype, solver, steps, warmup, per_level=False, profile=False):
        for _ in range(warmup):
            step(dtype, solver)
        torch.cuda.synchronize()
        if profile:
            ctx.profile(True)  # kernel events over the timed steps only
        lvl_ms = [0.0] * len(levels)
        t0 = time.perf_counter()
        for _ in range(steps):
            if per_level:
                for i, (l, xi) in enumerate(zip(levels, xis)):
                    ev0 = torch.cuda.Event(enable_timing=True)
                    ev1 = torch.cuda.Event(enable_timing=True)
                    ev0.record()
                    ctx.sample_level(l, xi, dtype=dtype, solver=solver, eps_fine=eps[l],
                                     eps_coarse=eps[l - 1] if l > 0 else 0.0, stats=False)
                    ev1.record()
                    ev1.synchronize()
                    lvl_ms[i] += ev0.elapsed_time(ev1)
            else:
                step(dtype, solver)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        return ms, [v / steps for v in lvl_ms]

    # ---- mixed path (timed region with per-kernel events)
    ms_mixed, _ = timed(a.dtype, "direct_ir", a.steps, a.warmup, profile=True)
    prof = {}
    for kind in ("field", "assembly", "factor", "solve", "residual"):
        for n in sorted(set(cells + [c // 2 for c in cells if c > w["n0"]])):
            r = ctx.profile_read(kind, n)
            if r["launches"]:
                prof[(kind, n)] = r
    ctx.profile(False)
    _, lvl_mixed = timed(a.dtype, "direct_ir", 1, 0, per_level=True)
    st = ctx.sample_level(levels[-1], xis[-1], dtype=a.dtype, solver="direct_ir",
                          eps_fine=eps[levels[-1]], eps_coarse=eps[levels[-1] - 1], stats=True)
    total = float(sum(Ns))
    value = total / (ms_mixed / 1e3)

    # ---- FP64 path on the same workload
    fp64 = None
    if not a.no_fp64:
        ms64, lvl64 = timed("f64", "direct", max(1, a.steps // 2), 1)
        _, lvl64 = timed("f64", "direct", 1, 0, per_level=True)
        fp64 = dict(ms_per_step=ms64, samples_per_s=total / (ms64 / 1e3),
                    per_level_samples_per_s=[N / (t / 1e3) for N, t in zip(Ns, lvl64)])

    # ---- roofline of the dominant kernel of the mixed step
    dom = max(prof.items(), key=lambda kv: kv[1]["ms"])
    (kind, n), r = dom
    avg_ms = r["ms"] / r["launches"]
    if kind == "factor":
        work = factor_flops(n) * r["samples"] / r["launches"]
        achieved = work / (avg_ms * 1e-3) / 1e12
        peak = PEAK["f32_alu"] if a.dtype != "f64" else PEAK["f64_alu"]
        roof = dict(bound="alu", achieved=achieved, peak=peak, unit="TFLOP/s", frac=achieved / peak,
                    traffic=None)
    else:
        m = n - 1
        nbytes = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}[a.dtype]
        T = (n // 8) * (n // 8 + 1) // 2 * 64 if n >= 64 else (m + 1) * m
        work = 2.0 * m * T * nbytes * r["samples"] / r["launches"]
        achieved = work / (avg_ms * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=achieved, peak=PEAK["hbm"], unit="GB/s",
                    frac=achieved / PEAK["hbm"], traffic=None)
    roof["kernel"] = "%s n=%d" % (kind, n)
    roof["avg_launch_ms"] = avg_ms
    roof["launches"] = r["launches"]

    # ---- CPU baseline: the oracle on a bounded sample of the same workload
    cpu = None
    if not a.no_cpu:
        import numpy as np
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
                   sample="FP64 banded Cholesky on %s samples per level (fine+coarse), scaled to "
                          "the full workload" % ",".join(samples_desc))

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
        "dtype": a.dtype,
        "data": "synthetic",
        "config": {"workload": a.workload, "cells": cells, "N_l": Ns, "K": K,
                   "sigma2": w["sigma2"], "corr_len": w["corr_len"], "eps_l": eps,
                   "path": "%s factor + FP64 refinement; residual, update, sums FP64" % a.dtype},
        "per_level_samples_per_s": [N / (t / 1e3) for N, t in zip(Ns, lvl_mixed)],
        "fp64": fp64,
        "speedup_vs_fp64": (value / fp64["samples_per_s"]) if fp64 else None,
        "mean_ir_trips_finest": st["stats"]["mean_iters"],
        "roofline": roof,
        "kernel_ms_per_step": {"%s_n%d" % k: v["ms"] / a.steps for k, v in prof.items()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
