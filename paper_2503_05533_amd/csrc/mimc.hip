// Device steps of the multi-index Monte Carlo driver (mlmc_mimc): the
// truncated coefficient vectors of an index's samples and the mixed
// difference of its four solves,
//   D_(l,k) = Q_(l,k) - Q_(l-1,k) - Q_(l,k-1) + Q_(l-1,k-1),
// Q_(l,k)(xi) the quantity on grid l with every coefficient of xi from mode
// K_k on set to zero (the modes are ordered by decreasing variance).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace mlmc {

// out[s, k] = k < keep ? xi[s, k] : 0 for C samples of K coefficients.
__global__ void k_mask_modes(int64_t CK, int K, int keep, const double *__restrict__ xi, double *__restrict__ out)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= CK) return;
    out[g] = (int)(g % K) < keep ? xi[g] : 0.0;
}

// y = q[0] - q[1] - q[2] + q[3] (absent terms NULL) and the combined state:
// converged when every present solve converged, promoted when any was.
__global__ void k_mimc_combine(int C, const double *__restrict__ q0, const double *__restrict__ q1,
                               const double *__restrict__ q2, const double *__restrict__ q3,
                               const uint32_t *__restrict__ s0, const uint32_t *__restrict__ s1,
                               const uint32_t *__restrict__ s2, const uint32_t *__restrict__ s3,
                               double *__restrict__ y, uint32_t *__restrict__ st)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    // (q0 - q1) - (q2 - q3): the grid difference at each truncation, then
    // their difference
    const double a = q0[c] - (q1 ? q1[c] : 0.0);
    const double b = q2 ? q2[c] - (q3 ? q3[c] : 0.0) : 0.0;
    y[c] = a - b;
    uint32_t conv = s0[c] & ST_CONVERGED, prom = s0[c] & ST_PROMOTED;
    if (s1) { conv &= s1[c]; prom |= s1[c] & ST_PROMOTED; }
    if (s2) { conv &= s2[c]; prom |= s2[c] & ST_PROMOTED; }
    if (s3) { conv &= s3[c]; prom |= s3[c] & ST_PROMOTED; }
    st[c] = (conv & ST_CONVERGED) | prom;
}

hipError_t launch_mask_modes(int C, int K, int keep, const double *xi, double *out, hipStream_t st)
{
    const int64_t CK = (int64_t)C * K;
    if (CK == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mask_modes, dim3((unsigned)((CK + 255) / 256)), dim3(256), 0, st, CK, K, keep, xi, out);
    return hipGetLastError();
}

hipError_t launch_mimc_combine(int C, const double *q0, const double *q1, const double *q2, const double *q3,
                               const uint32_t *s0, const uint32_t *s1, const uint32_t *s2, const uint32_t *s3,
                               double *y, uint32_t *st, hipStream_t stream)
{
    if (C == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mimc_combine, dim3((C + 255) / 256), dim3(256), 0, stream, C, q0, q1, q2, q3, s0, s1, s2,
                       s3, y, st);
    return hipGetLastError();
}

}  // namespace mlmc
