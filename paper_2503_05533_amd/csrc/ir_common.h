// Device pieces shared by the per-sample refinement kernels: the FP64
// matrix-free residual of the 5-point finite-volume operator and the stop
// test of Algorithm 2.1.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace mlmc {

__device__ inline double hmean2(double p, double q) { return 2.0 * p * q / (p + q); }

// Fixed-order tree sum over the NT threads of a workgroup (deterministic).
template <int NT>
__device__ inline double wg_sum(double v, double *red)
{
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

struct resid_out { double rr, bb, sx; };

// r = b - A x (FP64, padded block layout, pads 0) for one sample; returns the
// workgroup-reduced ||r||^2, ||b||^2 and sum(x).  b = h^2 fconst.
template <int NT>
__device__ inline resid_out residual_pass(int n, double fconst, const double *__restrict__ as,
                                          const double *__restrict__ xs, double *__restrict__ rs,
                                          double *red)
{
    const int m = n - 1, M = n, np = n + 1;
    const double h = 1.0 / n, bval = h * h * fconst;
    double rr = 0.0, bb = 0.0, sx = 0.0;
    for (int e = threadIdx.x; e < m * M; e += NT) {
        const int j = e / M, i = e % M;
        if (i >= m) {
            if (rs) rs[e] = 0.0;
            continue;
        }
        const int p = (j + 1) * np + (i + 1);
        const double c = as[p];
        const double aw = hmean2(c, as[p - 1]), ae = hmean2(c, as[p + 1]);
        const double asu = hmean2(c, as[p - np]), an = hmean2(c, as[p + np]);
        const double xv = xs[e];
        double ax = (aw + ae + asu + an) * xv;
        if (i > 0) ax -= aw * xs[e - 1];
        if (i + 1 < m) ax -= ae * xs[e + 1];
        if (j > 0) ax -= asu * xs[e - M];
        if (j + 1 < m) ax -= an * xs[e + M];
        const double rv = bval - ax;
        if (rs) rs[e] = rv;
        rr += rv * rv;
        bb += bval * bval;
        sx += xv;
    }
    resid_out o;
    o.rr = wg_sum<NT>(rr, red);
    o.bb = wg_sum<NT>(bb, red);
    o.sx = wg_sum<NT>(sx, red);
    return o;
}

// Stop test of Algorithm 2.1 after `trip` corrections: converged when
// relres < eps (strict); otherwise done at the trip limit, on a non-finite
// value, or when the residual stopped decreasing.  Returns the new state.
__device__ inline uint32_t ir_decide(uint32_t st, double rel, double prev, double sx, double eps,
                                     int trip, int imax, int direct)
{
    if (!isfinite(rel) || !isfinite(sx)) return st | ST_NONFINITE | ST_DONE;
    if (direct || rel < eps) return st | ST_CONVERGED | ST_DONE;
    if (trip >= imax) return st | ST_IMAX | ST_DONE;
    if (trip > 0 && !(rel < prev)) return st | ST_STALL | ST_DONE;
    return st;
}

}  // namespace mlmc
