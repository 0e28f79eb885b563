"""The synthetic workloads (grid sizes, field parameters, sample counts, seeds).

Domain (0,1)^2, f = 1, u = 0 on the boundary, nodal lognormal coefficient
a = exp(Z) with Z a truncated separable exponential-covariance KL expansion
(field 0) or the trigonometric expansion of the paper's sec. 5.1 (field 1);
finite volumes with harmonic faces (disc 0) or the paper's P1 elements on
right triangles (disc 1).
Level l has n_l = n0 * 2**l cells per side.  Seeds are 1000 + workload id.
"""

WORKLOADS = {
    # single level, FP64 direct, n=32, K=16
    "single_n32_K16": dict(id=0, n0=32, levels=[0], K=16, sigma2=1.0, corr_len=0.3,
                           N=[1000], seed=1000),
    # four-level MLMC, 16..128 cells per side, coarse partner shares xi
    "mlmc4_n16-128_K64": dict(id=1, n0=16, levels=[0, 1, 2, 3], K=64, sigma2=1.0,
                              corr_len=0.3, N=[20000, 5000, 1250, 300], seed=1001),
    # precision sweep over five levels, 16..256 cells per side
    "sweep5_n16-256_K128": dict(id=2, n0=16, levels=[0, 1, 2, 3, 4], K=128, sigma2=2.0,
                                corr_len=0.1, N=[40000, 10637, 2828, 752, 200], seed=1002),
    # all five levels batched together, geometric sample counts
    "batched5_n16-256_K128": dict(id=3, n0=16, levels=[0, 1, 2, 3, 4], K=128, sigma2=2.0,
                                  corr_len=0.1, N=[40000, 10637, 2828, 752, 200], seed=1003),
    # the paper's quarter-precision example (sec. 5.2): h0 = 1/4, trigonometric
    # field with s = 1, sigma = 1, k_p = 0.4; N_l from standard MLMC at TOL^2 = 2e-6
    "q43_n4-32_trig1": dict(id=5, n0=4, levels=[0, 1, 2, 3], K=1, sigma2=1.0, corr_len=0.3,
                            field=1, field_q=2.0, k_p=0.4, disc=1, N=None, seed=1005),
    # the paper's direct-solver example (sec. 5.2): P1 elements, h0 = 1/8, trigonometric
    # field s = 4, q = 2, sigma = 2, k_p = 0.05; N_l from standard MLMC at TOL^2 = 2e-6
    "paper5_n8-128_trig4": dict(id=6, n0=8, levels=[0, 1, 2, 3, 4], K=4, sigma2=4.0, corr_len=0.3,
                                field=1, field_q=2.0, k_p=0.05, disc=1, N=None, seed=1006),
    # adjoint gradient at n=128, 4096 samples
    "adjoint_n128_K128": dict(id=4, n0=128, levels=[0], K=128, sigma2=2.0, corr_len=0.1,
                              N=[4096], seed=1004),
}


def workload(name):
    return dict(WORKLOADS[name])


def level_cells(n0, level, m=2):
    return n0 * m ** level
