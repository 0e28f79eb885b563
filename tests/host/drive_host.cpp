// Host-only driver of the C ABI against the stub runtime: the multi-level
// step (graph and eager, FP32 refinement and FP64 direct) with the four-level
// workload shapes, three times each, then the adaptive estimator (mixed and
// standard), its checkpoint and resume, the no-allocation entry point and the
// multi-index driver.  Run under AddressSanitizer by tests/test_host_logic.py, once
// as is and once with the stub reporting a non-converged sample per chunk.
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "mlmc.h"
int main()
{
    mlmc_config c{};
    c.n0 = 16; c.m = 2; c.L_max = 3; c.K = 64; c.sigma2 = 1.0; c.corr_len = 0.3; c.f = 1.0; c.k_p = 0.05;
    c.alpha = 2; c.beta = 4; c.gamma = 4; c.ir_max_iter = 10; c.minres_max_iter = 5000; c.seed = 1001;
    mlmc_ctx *ctx = nullptr;
    int rc = mlmc_create(&c, &ctx);
    printf("create rc=%d\n", rc);
    int32_t lv[4] = {0, 1, 2, 3};
    int64_t N[4] = {20000, 5000, 1250, 300};
    for (int dt = 1; dt >= 0; --dt) {
        mlmc_level_opts o[4];
        double eps[16];
        mlmc_accuracy_targets(ctx, 3, eps);
        for (int i = 0; i < 4; ++i) {
            o[i] = mlmc_level_opts{};
            o[i].factor_dtype = (mlmc_dtype)dt;
            o[i].solver = dt ? MLMC_DIRECT_IR : MLMC_DIRECT;
            o[i].eps_fine = eps[i];
            o[i].eps_coarse = i ? eps[i - 1] : 0.0;
            o[i].promote = 1;
        }
        size_t nb = mlmc_levels_workspace_bytes(ctx, 4, lv, N, o);
        printf("dt=%d ws %zu bytes\n", dt, nb);
        // fake device pointers: the stub launchers never touch them
        void *ws = (void *)(uintptr_t)0x100000000ull;
        std::vector<double> xi0(1), y0(1);
        const double *xi[4] = {xi0.data(), xi0.data(), xi0.data(), xi0.data()};
        double *y[4] = {y0.data(), y0.data(), y0.data(), y0.data()};
        for (int g = 1; g >= 0; --g)
            for (int r = 0; r < 3; ++r) {
                rc = mlmc_sample_levels(ctx, 4, lv, N, xi, o, ws, nb, y, nullptr, g, nullptr);
                printf("dt=%d graph=%d rep=%d rc=%d %s\n", dt, g, r, rc, rc ? mlmc_last_error(ctx) : "");
            }
    }
    {
        mlmc_dtype dts[4] = {MLMC_F32, MLMC_F32, MLMC_F32, MLMC_F32};
        mlmc_result res;
        for (int mixed = 1; mixed >= 0; --mixed) {
            rc = mlmc_estimate(ctx, 2e-5, 1000, dts, MLMC_DIRECT_IR, mixed, &res, nullptr);
            printf("estimate mixed=%d rc=%d L=%d N0=%lld noconv0=%lld conv=%d %s\n", mixed, rc, res.L,
                   (long long)res.N[0], (long long)res.n_noconv[0], res.converged, rc ? mlmc_last_error(ctx) : "");
        }
    }
    {
        // checkpoint and resume: one round per call from a saved state reaches
        // the uninterrupted run's levels, sample counts and estimate
        mlmc_dtype dts[4] = {MLMC_F32, MLMC_F32, MLMC_F32, MLMC_F32};
        mlmc_result full, part;
        rc = mlmc_estimate(ctx, 2e-5, 1000, dts, MLMC_DIRECT_IR, 1, &full, nullptr);
        mlmc_estimate_state sa, sb;
        int calls = 0;
        rc = mlmc_estimate_resumable(ctx, 2e-5, 1000, dts, MLMC_DIRECT_IR, 1, nullptr, 1, &sa, &part, nullptr);
        ++calls;
        while (rc == MLMC_PAUSED && calls < 100) {
            sb = sa;
            rc = mlmc_estimate_resumable(ctx, 2e-5, 1000, dts, MLMC_DIRECT_IR, 1, &sb, 1, &sa, &part, nullptr);
            ++calls;
        }
        bool same = part.L == full.L && part.estimate == full.estimate && part.converged == full.converged;
        for (int l = 0; l <= full.L; ++l) same = same && part.N[l] == full.N[l];
        printf("resume rc=%d calls=%d rounds=%d same=%d\n", rc, calls, sa.rounds, (int)same);
        // a state from another tolerance is refused
        rc = mlmc_estimate_resumable(ctx, 1e-5, 1000, dts, MLMC_DIRECT_IR, 1, &sb, 1, &sa, &part, nullptr);
        printf("resume mismatch rc=%d\n", rc);
    }
    {
        // the no-allocation entry point: a level that fits the scratch, then one that does not
        mlmc_level_opts o{};
        o.factor_dtype = MLMC_F32;
        o.solver = MLMC_DIRECT_IR;
        o.eps_fine = 1e-6;
        o.eps_coarse = 1e-6;
        o.promote = 1;
        std::vector<double> xi0(1), q0(1);
        mlmc_level_stats st;
        const int64_t ns[2] = {64, 200000};
        for (int k = 0; k < 2; ++k) {
            rc = mlmc_sample_level_noalloc(ctx, 1, ns[k], xi0.data(), &o, q0.data(), q0.data(), q0.data(),
                                           nullptr, &st, nullptr);
            printf("noalloc n=%lld rc=%d\n", (long long)ns[k], rc);
        }
    }
    {
        // multi-index Monte Carlo: three indices (chunked by the driver's
        // budget), then a repeated index
        mlmc_mimc_config mc{};
        mc.n_idx = 3;
        const int il[3] = {0, 1, 3}, ik[3] = {0, 1, 0};
        const int64_t nn[3] = {1000, 500, 300};
        double eps[16];
        mlmc_accuracy_targets(ctx, 3, eps);
        for (int i = 0; i < 3; ++i) {
            mc.idx_l[i] = il[i];
            mc.idx_k[i] = ik[i];
            mc.N[i] = nn[i];
            mc.opts[i].factor_dtype = MLMC_F32;
            mc.opts[i].solver = MLMC_DIRECT_IR;
            mc.opts[i].eps_fine = eps[il[i]];
            mc.opts[i].eps_coarse = il[i] ? eps[il[i] - 1] : 0.0;
            mc.opts[i].promote = 1;
        }
        mc.K0 = 16;
        mc.seed = 5;
        mlmc_mimc_result mr;
        rc = mlmc_mimc(ctx, &mc, &mr, nullptr);
        printf("mimc rc=%d solves=%lld noconv0=%lld\n", rc, (long long)mr.solves, (long long)mr.n_noconv[0]);
        mc.idx_l[2] = 1;
        mc.idx_k[2] = 1;
        rc = mlmc_mimc(ctx, &mc, &mr, nullptr);
        printf("mimc repeated rc=%d\n", rc);
    }
    mlmc_destroy(ctx);
    return 0;
}
