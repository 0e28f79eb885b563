// Internal launch interface between the host API and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mlmc {

// Internal per-sample state bits (the low nibble matches the public status bits).
enum : uint32_t {
    ST_CONVERGED = 1u,
    ST_PROMOTED = 2u,
    ST_NONFINITE = 4u,
    ST_IMAX = 8u,
    ST_STALL = 16u,      // residual stopped decreasing
    ST_BREAKDOWN = 32u,  // non-positive pivot in the factorisation
    ST_DONE = 1u << 31,  // no further refinement work for this sample
};

// Whether grid n with factor dtype (mlmc_dtype code) uses the block-layout
// factor and solves (else the register-tile kernels): from n = 16 for the
// low-precision factors; for FP64 the n = 16 grid (one-row-per-lane kernels)
// and n >= 64 (MFMA kernels), the tile kernels being faster at n = 32.  The
// grids below 16 keep the tile kernels.
inline bool use_blk(int dtype, int n) { return n == 16 || n >= (dtype == 0 ? 64 : 16); }
// Grids on which a factor dtype is available: FP8 (code 4) on the grids
// below 16 (the tile kernels) only.
inline bool dtype_on_grid(int dtype, int n) { return dtype != 4 || n < 16; }

size_t factor_entries_per_sample(int dtype, int n);

// Size of the per-device scratch array behind mlmc_sample_level_noalloc.
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
// Device address of that array on `device`, which must be the current
// device; taken once per device (hipGetSymbolAddress) and kept.
hipError_t scratch_device_ptr(int device, void **out);

// Arguments of the per-sample refinement kernel (one workgroup per sample b:
// sample idx[b] (or b), factor slot slot_base + b; b >= *count exits).
struct ir_args {
    int n, nblocks;
    double fconst;
    const double *a, *sc, *beta;
    const void *factor;
    double *x, *r, *z;
    double eps;
    int imax, direct;
    const int *idx, *count;
    int64_t slot_base;
    uint32_t *state;
    double *relres, *q;
    int32_t *iters;
    int variant;  // refinement-kernel variant (0: built-in default; n >= 64: waves per row pair)
    int fwd_done;  // the factorisation wrote the forward sweep of the initial solve to z (2: all of it, x0 in x)
    int disc;      // edge coefficients: 0 harmonic means (finite volumes), 1 P1 elements
};

hipError_t launch_fill_xi(uint64_t seed, int level, int64_t first, int64_t n, int K, double *xi,
                          hipStream_t st);
hipError_t launch_field(int S, int K, int P, const double *xi, const double *phit, double *a,
                        hipStream_t st);
// Z = xi Phi^T, a = exp(Z) on FP64 MFMA (xi [S x K], phit [K x P], a [S x P]).
hipError_t launch_field_mfma(int S, int K, int P, const double *xi, const double *phit, double *a,
                             hipStream_t st);
hipError_t launch_grad_gemm(int S, int K, int P, const double *gz, const double *phit,
                            const double *gq, double *grad, hipStream_t st);
// disc: edge coefficients, 0 harmonic means (finite volumes), 1 P1 elements
// on right triangles (node_faces in ir_common.h).
hipError_t launch_coeffs(int n, int S, const double *a, double *sc, double *gam, double *beta, int disc,
                         hipStream_t st);
// Factorisation of the scaled operator.  It reads the couplings beta, gam,
// except where factor_forms_coeffs(n): there it reads the nodal coefficient a
// and forms them itself, writing the scaling sc and beta for the refinement
// (not in a pass over promoted samples, idx != NULL, which forms the same
// values).  With fz != NULL (and factor_fuses_forward) it also runs the
// forward sweep of the solve for the right-hand side frhs (constant, interior
// unknowns) scaled by sc, writing z to fz (the refinement's z buffer); where
// factor_solves_initial(dtype, n), with x0 != NULL, the back sweep as well,
// writing the initial solve to x0 (n = 16, and the twisted block layouts,
// whose two wave groups run the two back sweeps at once).  variant (the autotuner's choice, 0 default): 1
// forms the FP16/BF16 factors' MFMA products in FP32 instead of their format.
hipError_t launch_factor(int dtype, int n, int nblocks, const double *a, double *sc, double *beta,
                         const double *gam, void *factor, const int *idx, const int *count,
                         int64_t slot_base, uint32_t *state, double frhs, double *fz, double *x0,
                         int disc, int variant, hipStream_t st);
bool factor_fuses_forward(int dtype, int n);
inline bool factor_forms_coeffs(int n) { return n == 16; }
bool factor_solves_initial(int dtype, int n);
// Initial solve + refinement loop of Algorithm 2.1, one workgroup per sample
// (16 samples per workgroup at n = 16).  fwd_done: 1, the factorisation ran
// the forward sweep (z in the z buffer), or at n = 16 the whole initial solve
// (x0 in x); 2 (block layouts), the whole initial solve (x0 in x).
hipError_t launch_ir(int dtype, const ir_args &g, hipStream_t st);
hipError_t launch_factor_blk(int dtype, int n, int nblocks, const double *a, double *sc, double *beta,
                             const double *gam, void *factor, const int *idx, const int *count,
                             int64_t slot_base, uint32_t *state, double frhs, double *fz, double *x0,
                             int disc, int variant, hipStream_t st);
hipError_t launch_ir_blk(int dtype, const ir_args &g, hipStream_t st);
// MINRES (low = 0: FP64 inner vectors) or MINRES with FP64 iterative
// refinement around an inner solve with FP32 vectors (low = 1); vecs holds
// 7 vectors per workgroup of the inner precision.  Workgroup b solves sample
// idx[b] (or b); with count != NULL, workgroups b >= *count exit.
hipError_t launch_minres(int n, int S, double fconst, const double *a, const double *sc,
                         const double *gam, const double *beta, double *x, double *r, void *vecs,
                         int low, double eps, int maxit, int max_outer, const int *idx, const int *count,
                         uint32_t *state, double *relres, double *q, int32_t *iters, int disc, hipStream_t st);
// Conjugate gradients in FP64 preconditioned by an FP32 geometric multigrid
// V-cycle (gamma = 2 solver), one workgroup per sample: the solution into the
// padded layout x; vecs holds 5 (n+1)^2 doubles and mg
// mgcg_floats_per_sample(n) floats per sample.
size_t mgcg_floats_per_sample(int n);
hipError_t launch_mgcg(int n, int S, double fconst, const double *a, double *x, double *vecs, float *mg,
                       double eps, int maxit, uint32_t *state, double *relres, double *q, int32_t *iters, int disc,
                       hipStream_t st);
// Multilevel MCMC steps (mcmc.hip); obs_node[j] = fx + 1024 fy with the
// node at (fx / 1024, fy / 1024).
hipError_t launch_pcn_propose(int C, int K, double b, const double *theta, const double *w, double *out,
                              hipStream_t st);
hipError_t launch_mcmc_accept(int C, int K, int n, int mode, int n_obs, const int *obs_node, const double *obs_val,
                              double noise_sd, const double *x, const double *qp, const double *prop,
                              const double *llcp, const double *z, double *theta, double *ll, double *llc,
                              double *q, int64_t *accepted, int count, hipStream_t st);
hipError_t launch_mcmc_loglik(int C, int n, int n_obs, const int *obs_node, const double *obs_val, double noise_sd,
                              const double *x, double *ll, hipStream_t st);
hipError_t launch_mcmc_record(int C, const double *qf, const double *qc, double *sums, hipStream_t st);
// Multi-index Monte Carlo: coefficients from mode `keep` on set to zero, and
// the mixed difference q0 - q1 - q2 + q3 (NULL terms absent) with the
// combined convergence state of its solves.
hipError_t launch_mask_modes(int C, int K, int keep, const double *xi, double *out, hipStream_t st);
hipError_t launch_mimc_combine(int C, const double *q0, const double *q1, const double *q2, const double *q3,
                               const uint32_t *s0, const uint32_t *s1, const uint32_t *s2, const uint32_t *s3,
                               double *y, uint32_t *st, hipStream_t stream);
hipError_t launch_adjoint_gz(int n, int S, const double *a, const double *u, const double *lam,
                             double *gz, int disc, hipStream_t st);
hipError_t launch_unpad(int n, int S, const double *x, double *u, hipStream_t st);
hipError_t launch_init_state(int S, uint32_t *state, double *relres, hipStream_t st);
hipError_t launch_reset_subset(int P, const int *idx, const int *count, uint32_t *state,
                               double *relres, hipStream_t st);
hipError_t launch_zero_int(int *p, int n, hipStream_t st);
hipError_t launch_collect(int S, const uint32_t *state, int *idx, int *cnt, hipStream_t st);
hipError_t launch_pair_sums(int S, const double *qf, const double *qc, const uint32_t *stf,
                            const uint32_t *stc, const int32_t *itf, const int32_t *itc, double *y,
                            uint8_t *status, double *sums, hipStream_t st);

}  // namespace mlmc
