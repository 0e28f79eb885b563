// Device pieces shared by the per-sample refinement kernels: the FP64
// matrix-free residual of the 5-point finite-volume operator and the stop
// test of Algorithm 2.1.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace mlmc {

__device__ inline double hmean2(double p, double q) { return 2.0 * p * q / (p + q); }

// Edge coefficients of the 5-point operator from the nodal coefficient.
// disc 0 (vertex-centred finite volumes): the harmonic mean of the edge's
// end nodes.  disc 1 (P1 elements, Sec. 3, on the right triangles of cells
// cut along the diagonal (x, y)-(x+h, y+h), the coefficient interpolated
// linearly, so a triangle weighs its vertex mean): every mesh edge parallel
// to an axis is a leg of its two triangles, each contributing half its
// weight, and the diagonals couple nothing:
//   edge L = (x, y) - R = (x+h, y): (2 a_L + 2 a_R + a(x+h, y+h) + a(x, y-h)) / 6,
//   edge B = (x, y) - T = (x, y+h): (2 a_B + 2 a_T + a(x+h, y+h) + a(x-h, y)) / 6.
__device__ inline double face_x(int disc, double aL, double aR, double aRN, double aLS)
{
    return disc ? (2.0 * (aL + aR) + aRN + aLS) / 6.0 : hmean2(aL, aR);
}
__device__ inline double face_y(int disc, double aB, double aT, double aTE, double aBW)
{
    return disc ? (2.0 * (aB + aT) + aTE + aBW) / 6.0 : hmean2(aB, aT);
}

// The four edge coefficients around node p of the (n+1)^2 node array (row
// length np); the diagonal neighbours are read for disc 1 only.
struct faces4 { double w, e, s, n; };
__device__ inline faces4 node_faces(int disc, const double *__restrict__ as, int p, int np)
{
    const double c = as[p], w = as[p - 1], e = as[p + 1], sv = as[p - np], nv = as[p + np];
    if (!disc) return faces4{hmean2(c, w), hmean2(c, e), hmean2(c, sv), hmean2(c, nv)};
    const double ne = as[p + np + 1], sw = as[p - np - 1];
    return faces4{face_x(1, w, c, nv, sw), face_x(1, c, e, ne, sv), face_y(1, sv, c, e, sw),
                  face_y(1, c, nv, ne, w)};
}

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
                                          double *red, int disc)
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
        const faces4 f = node_faces(disc, as, p, np);
        const double aw = f.w, ae = f.e, asu = f.s, an = f.n;
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

// The same three sums in one tree (red holds 3 NT doubles): the order of
// each sum is that of wg_sum, with a third of the barriers.
template <int NT>
__device__ inline resid_out wg_sum3(double a, double b, double c, double *red)
{
    const int t = threadIdx.x;
    red[t] = a;
    red[NT + t] = b;
    red[2 * NT + t] = c;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (t < s) {
            red[t] += red[t + s];
            red[NT + t] += red[NT + t + s];
            red[2 * NT + t] += red[2 * NT + t + s];
        }
        __syncthreads();
    }
    resid_out o;
    o.rr = red[0];
    o.bb = red[NT];
    o.sx = red[2 * NT];
    __syncthreads();
    return o;
}

// residual_pass for a compile-time block size M = n: the same arithmetic
// and per-thread order, with shift/mask indexing, a fixed trip count
// unrolled by four, and branch-free neighbours (clamped indices, selected
// terms; x - 0.0 and r + 0.0 are exact), so that the loads of several
// unknowns are in flight together (four, two for n <= 32, whose one-wave
// refinement kernel keeps four waves per SIMD that way).  red holds 3 NT
// doubles; D is the edge rule.
template <int NT, int M, int D>
__device__ inline resid_out residual_pass_m(double fconst, const double *__restrict__ as,
                                            const double *__restrict__ xs, double *__restrict__ rs,
                                            double *red)
{
    constexpr int disc = D;  // the edge rule, a compile-time constant here
    constexpr int m = M - 1, np = M + 1, TOT = m * M, IT = (TOT + NT - 1) / NT, UNR = M <= 32 ? 2 : 4;
    const double h = 1.0 / M, bval = h * h * fconst;
    double rr = 0.0, bb = 0.0, sx = 0.0;
#pragma unroll UNR
    for (int k = 0; k < IT; ++k) {
        const int e = threadIdx.x + k * NT;
        const bool live = e < TOT;
        const int ec = live ? e : TOT - 1;
        const int j = ec / M, i = ec % M;
        const bool in = live && i < m;
        // node of the unknown; for the pad entry (i = m) it is a boundary node
        // whose axis neighbours are still inside the node array (values
        // unused); P1 faces also read diagonal neighbours, outside the array
        // for that node, so the pad then reads the node west of it instead
        const int p = (j + 1) * np + (i + 1);
        const faces4 f = node_faces(disc, as, (disc && !in) ? p - 1 : p, np);
        const double aw = f.w, ae = f.e, asu = f.s, an = f.n;
        const double xv = xs[ec];
        const double xw = xs[ec > 0 ? ec - 1 : 0], xe = xs[ec + 1 < TOT ? ec + 1 : TOT - 1];
        const double xsn = xs[ec >= M ? ec - M : 0], xn = xs[ec + M < TOT ? ec + M : TOT - 1];
        double ax = (aw + ae + asu + an) * xv;
        ax -= i > 0 ? aw * xw : 0.0;
        ax -= i + 1 < m ? ae * xe : 0.0;
        ax -= j > 0 ? asu * xsn : 0.0;
        ax -= j + 1 < m ? an * xn : 0.0;
        const double rv = bval - ax;
        if (rs && live) rs[ec] = in ? rv : 0.0;
        rr += in ? rv * rv : 0.0;
        bb += in ? bval * bval : 0.0;
        sx += in ? xv : 0.0;
    }
    return wg_sum3<NT>(rr, bb, sx, red);
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
