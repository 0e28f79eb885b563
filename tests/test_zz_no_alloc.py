"""The no-allocation entry point (mlmc_sample_level_noalloc) against
mlmc_sample_level on the same inputs, through the C ABI: bit-identical Q,
Y, status and level sums (the same kernels on the same inputs), on two
calls in a row on the shared scratch, the second with fewer samples, and
the size limit."""
import ctypes

import numpy as np
import pytest
import torch

import seeded_inputs as si

pytestmark = pytest.mark.gpu


def _ctx():
    from paper_2503_05533_amd import MLMC, Config
    return MLMC(Config(n0=16, L_max=2, K=64, sigma2=1.0, corr_len=0.3, seed=1001), device="cuda:0")


@pytest.mark.parametrize("dtype,solver", [("f32", "direct_ir"), ("f64", "direct"), ("f16", "direct_ir")])
def test_noalloc_matches_sample_level(dtype, solver):
    ctx = _ctx()
    try:
        eps = ctx.accuracy_targets(2)
        for level, S in ((1, 120), (1, 37), (2, 16), (0, 500)):
            xi = torch.from_numpy(si.splitmix64_normals(1001, level, 0, S, 64)).cuda()
            ef, ec = eps[level], (eps[level - 1] if level > 0 else 0.0)
            need = ctx.workspace_bytes(level, S, dtype=dtype, solver=solver, eps_fine=ef,
                                       eps_coarse=ec)
            assert need <= 64 << 20, need
            ref = ctx.sample_level(level, xi, dtype=dtype, solver=solver, eps_fine=ef, eps_coarse=ec)
            got = ctx.sample_level_noalloc(level, xi, dtype=dtype, solver=solver, eps_fine=ef,
                                           eps_coarse=ec)
            torch.cuda.synchronize()
            print("noalloc", dtype, level, S, got["rc"], flush=True)
            assert got["rc"] == ref["rc"] == 0
            for k in ("qf", "y", "status") + (("qc",) if level > 0 else ()):
                assert torch.equal(got[k], ref[k]), (k, level, S)
            for k in ("n", "sum_y", "sum_y2", "sum_qf", "sum_qc", "n_promoted", "n_noconv",
                      "mean_iters", "mean_iters_coarse"):
                assert got["stats"][k] == ref["stats"][k], (k, level, S)
    finally:
        ctx.close()


def test_noalloc_rejects_beyond_the_scratch():
    from paper_2503_05533_amd import MLMCError
    ctx = _ctx()
    try:
        S = 4000
        assert ctx.workspace_bytes(2, S, dtype="f32", solver="direct_ir", eps_fine=1e-6,
                                   eps_coarse=1e-6) > 64 << 20
        xi = torch.zeros((S, 64), dtype=torch.float64, device="cuda:0")
        with pytest.raises(MLMCError, match="scratch"):
            ctx.sample_level_noalloc(2, xi, dtype="f32", solver="direct_ir", eps_fine=1e-6,
                                     eps_coarse=1e-6)
        # a fitting call afterwards still works on the shared scratch
        xi = torch.from_numpy(si.splitmix64_normals(1001, 0, 0, 64, 64)).cuda()
        got = ctx.sample_level_noalloc(0, xi, dtype="f32", solver="direct_ir", eps_fine=1e-6)
        ref = ctx.sample_level(0, xi, dtype="f32", solver="direct_ir", eps_fine=1e-6)
        assert torch.equal(got["qf"], ref["qf"])
    finally:
        ctx.close()
