// Device steps of the multilevel Markov chain Monte Carlo driver
// (mlmc_mcmc): a batch of independent chains, one entry per chain, advanced
// together so that every step's forward solves are one batched solve.
//
// Bayesian set-up: prior xi ~ N(0, I_K); data d_j = u(x_j) + noise at
// observation nodes, noise N(0, s^2); the log-likelihood of level l is
// -sum_j (d_j - u_l(x_j))^2 / (2 s^2) with u_l the level's discrete solution.
// Chains on level 0 use the preconditioned Crank-Nicolson proposal
// xi' = sqrt(1 - b^2) xi + b w, w ~ N(0, I) (reversible for the prior, so a
// step accepts with probability min(1, L_0(xi') / L_0(xi))).  A chain on
// level l >= 1 proposes the current state of a chain targeting the level
// l-1 posterior (an independence proposal drawn from pi_{l-1}) and accepts
// with min(1, L_l(xi') L_{l-1}(xi) / (L_l(xi) L_{l-1}(xi'))).
// Acceptance uniforms are Phi(z) of counter-based normals z.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "kernels.h"

namespace mlmc {

// out = sqrt(1 - b^2) theta + b w, C x K.
__global__ void k_pcn_propose(int64_t CK, double b, const double *__restrict__ theta, const double *__restrict__ w,
                              double *__restrict__ out)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= CK) return;
    out[g] = sqrt(1.0 - b * b) * theta[g] + b * w[g];
}

// Log-likelihood of each chain's proposal from its solution x (padded
// layout of grid n: unknown (ix, iy) at (iy-1) n + (ix-1)), then the
// Metropolis-Hastings decision and the state update:
//   mode 0 (pCN):        log a = llp - ll
//   mode 1 (two-level):  log a = (llp - ll) - (llcp - llc)
// accepted: theta <- prop, ll <- llp, q <- qp, llc <- llcp (mode 1).
__global__ void k_mcmc_accept(int C, int K, int n, int mode, int n_obs, const int *__restrict__ obs_node,
                              const double *__restrict__ obs_val, double noise_sd, const double *__restrict__ x,
                              const double *__restrict__ qp, const double *__restrict__ prop,
                              const double *__restrict__ llcp, const double *__restrict__ z,
                              double *__restrict__ theta, double *__restrict__ ll, double *__restrict__ llc,
                              double *__restrict__ q, int64_t *__restrict__ accepted, int count)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const int m = n - 1;
    const double *xs = x + (size_t)c * m * n;
    double llp = 0.0;
    for (int j = 0; j < n_obs; ++j) {
        const int node = obs_node[j];  // ix + iy * 1024, interior node of every grid (scaled below)
        const int fx = node & 1023, fy = node >> 10;
        const int ix = fx * n / 1024, iy = fy * n / 1024;
        const double u = xs[(iy - 1) * n + (ix - 1)];
        const double d = obs_val[j] - u;
        llp -= d * d / (2.0 * noise_sd * noise_sd);
    }
    const double la = mode ? (llp - ll[c]) - (llcp[c] - llc[c]) : llp - ll[c];
    const double uz = 0.5 * erfc(-z[c] * 0.70710678118654752440);  // Phi(z)
    const bool acc = isfinite(llp) && (la >= 0.0 || uz < exp(la));
    if (acc) {
        for (int k = 0; k < K; ++k) theta[(size_t)c * K + k] = prop[(size_t)c * K + k];
        ll[c] = llp;
        q[c] = qp[c];
        if (mode) llc[c] = llcp[c];
        if (count) accepted[c] += 1;
    }
}

// Log-likelihood only (the initial states): ll = -sum (d - u)^2 / (2 s^2).
__global__ void k_mcmc_loglik(int C, int n, int n_obs, const int *__restrict__ obs_node,
                              const double *__restrict__ obs_val, double noise_sd, const double *__restrict__ x,
                              double *__restrict__ ll)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const int m = n - 1;
    const double *xs = x + (size_t)c * m * n;
    double l = 0.0;
    for (int j = 0; j < n_obs; ++j) {
        const int node = obs_node[j];
        const int ix = (node & 1023) * n / 1024, iy = (node >> 10) * n / 1024;
        const double d = obs_val[j] - xs[(iy - 1) * n + (ix - 1)];
        l -= d * d / (2.0 * noise_sd * noise_sd);
    }
    ll[c] = l;
}

// Per chain: sum and sum of squares of Y = qf - qc (qc may be NULL).
__global__ void k_mcmc_record(int C, const double *__restrict__ qf, const double *__restrict__ qc,
                              double *__restrict__ sums)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const double y = qf[c] - (qc ? qc[c] : 0.0);
    sums[2 * c] += y;
    sums[2 * c + 1] += y * y;
}

hipError_t launch_pcn_propose(int C, int K, double b, const double *theta, const double *w, double *out,
                              hipStream_t st)
{
    const int64_t CK = (int64_t)C * K;
    hipLaunchKernelGGL(k_pcn_propose, dim3((unsigned)((CK + 255) / 256)), dim3(256), 0, st, CK, b, theta, w, out);
    return hipGetLastError();
}

hipError_t launch_mcmc_accept(int C, int K, int n, int mode, int n_obs, const int *obs_node, const double *obs_val,
                              double noise_sd, const double *x, const double *qp, const double *prop,
                              const double *llcp, const double *z, double *theta, double *ll, double *llc,
                              double *q, int64_t *accepted, int count, hipStream_t st)
{
    hipLaunchKernelGGL(k_mcmc_accept, dim3((C + 127) / 128), dim3(128), 0, st, C, K, n, mode, n_obs, obs_node,
                       obs_val, noise_sd, x, qp, prop, llcp, z, theta, ll, llc, q, accepted, count);
    return hipGetLastError();
}

hipError_t launch_mcmc_loglik(int C, int n, int n_obs, const int *obs_node, const double *obs_val, double noise_sd,
                              const double *x, double *ll, hipStream_t st)
{
    hipLaunchKernelGGL(k_mcmc_loglik, dim3((C + 127) / 128), dim3(128), 0, st, C, n, n_obs, obs_node, obs_val,
                       noise_sd, x, ll);
    return hipGetLastError();
}

hipError_t launch_mcmc_record(int C, const double *qf, const double *qc, double *sums, hipStream_t st)
{
    hipLaunchKernelGGL(k_mcmc_record, dim3((C + 127) / 128), dim3(128), 0, st, C, qf, qc, sums);
    return hipGetLastError();
}

}  // namespace mlmc
