// Batched MINRES (Sec. 2.2: the Krylov solver of the paper's iterative
// experiments, stopped on the relative residual) and MINRES with iterative
// refinement (Sec. 2.3 applied to a Krylov inner solver): one workgroup per
// sample.
//
// Both run an outer loop in FP64: x = 0, r = b; an inner MINRES solves the
// Jacobi-scaled correction equation Ahat y = S r (Ahat = S A S,
// S = diag(A)^(-1/2), which keeps the operator symmetric) until its
// recurrence residual estimate falls below tau ||S r||; then x += S y and
// the true FP64 residual r = b - A x of the unscaled system is formed from
// the nodal coefficient.  The sample has converged when ||r|| / ||b|| < eps
// (strict).  The inner solve's vectors (and the scaled couplings it applies
// Ahat with) are stored in T:
//   T = double (MLMC_MINRES): tau = 0.9 eps / rel, so one inner solve
//     normally suffices; a later outer step restarts from the true residual;
//   T = float (MLMC_MINRES_IR): tau = max(eps / (2 rel), 1e-5), so each
//     inner solve asks of FP32 no more than it can deliver and the outer
//     FP64 refinement removes the rest.  Where the operator is too badly
//     conditioned for FP32 vectors the refinement stalls; the host then
//     re-solves those samples with T = double (promotion, as for the
//     low-precision factors).
//
// The inner iteration, restated from the Lanczos process and a QR
// factorisation of the Lanczos tridiagonal matrix by Givens rotations:
//   Lanczos:  b_{k+1} v_{k+1} = Ahat v_k - a_k v_k - b_k v_{k-1},
//             a_k = v_k^T Ahat v_k, b_1 v_1 = c (the right-hand side),
//             v_0 = 0 (so b_1 plays no part in column 1 of T_k);
//   column k of T_k, (b_k, a_k, b_{k+1}) in rows (k-1, k, k+1), is turned
//   by the two previous rotations into (e_k, d_k, g_k) in rows (k-2, k-1, k):
//             e_k = s_{k-2} b_k,  t = c_{k-2} b_k,
//             d_k = c_{k-1} t + s_{k-1} a_k,  g_k = c_{k-1} a_k - s_{k-1} t,
//   and the new rotation (c_k, s_k) = (g_k, b_{k+1}) / r_k,
//   r_k = |(g_k, b_{k+1})|, makes row k + 1 zero;
//   the rotated right-hand side gives the step length c_k h and the new
//   residual norm estimate |h| <- |s_k h| (h starts at b_1);
//   directions:  p_k = (v_k - d_k p_{k-1} - e_k p_{k-2}) / r_k,
//   iterate:     y_k = y_{k-1} + c_k h p_k.
// Dot products: per-thread partial sums in FP64, a butterfly within each
// wave, then the wave partials in wave order (deterministic), one barrier.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ir_common.h"
#include "kernels.h"

namespace mlmc {

// Two sums over the workgroup: a xor butterfly inside each wave (every lane
// ends with the wave total), the wave totals in wave order.  slots holds
// two alternating sets so that one barrier per call suffices.
template <int NT>
__device__ inline void wg_sum2_fast(double &a, double &b, double (*slots)[NT / 64][2], int &phase)
{
    constexpr int W = NT / 64;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        slots[phase][w][0] = a;
        slots[phase][w][1] = b;
    }
    __syncthreads();
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        sa += slots[phase][k][0];
        sb += slots[phase][k][1];
    }
    a = sa;
    b = sb;
    phase ^= 1;
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_minres_ir(int n, double fconst, const double *__restrict__ a,
                                                  const double *__restrict__ sc,
                                                  const double *__restrict__ gam,
                                                  const double *__restrict__ beta,
                                                  double *__restrict__ x, double *__restrict__ r,
                                                  T *__restrict__ vecs, double eps, int maxit, int max_outer,
                                                  const int *__restrict__ idx, const int *__restrict__ count,
                                                  uint32_t *__restrict__ state,
                                                  double *__restrict__ relres,
                                                  double *__restrict__ q, int32_t *__restrict__ iters, int disc)
{
    constexpr bool LOW = sizeof(T) == 4;
    __shared__ double slots[2][NT / 64][2];
    __shared__ double red[3 * NT];
    const int m = n - 1, M = n;
    const int N = m * M;
    // workgroup b solves sample idx[b] (or b) with work-vector slot b; b >= *count exits
    const int b = blockIdx.x;
    if (count && b >= *count) return;
    const int s = idx ? idx[b] : b;
    const size_t vo = (size_t)s * N;
    const double *scs = sc + vo;
    double *xs = x + vo, *rs = r + vo;
    // work vectors per sample (T): y, v_prev / u, v, p1, p2, and the scaled
    // couplings gam, beta in T (roles of the first five rotate by index)
    T *base = vecs + (size_t)b * 7 * N;
    auto V = [&](int k) { return base + (size_t)k * N; };
    T *yv = V(0), *gT = V(5), *bT = V(6);
    const double *as = a + (size_t)s * (n + 1) * (n + 1);
    const double h = 1.0 / n, bval = h * h * fconst;
    const int t = threadIdx.x;
    int phase = 0;

    // the operator's couplings in T; x = 0, r = b
    for (int e = t; e < N; e += NT) {
        gT[e] = (T)gam[vo + e];
        bT[e] = (T)beta[vo + e];
        xs[e] = 0.0;
        rs[e] = ((e % M) < m) ? bval : 0.0;
    }
    uint32_t st = state[s] & ~(uint32_t)ST_DONE;
    double rel = 1.0, sx = 0.0, prev = INFINITY;
    int it = 0;
    const bool zero_rhs = !(bval != 0.0);
    for (int outer = 0; !zero_rhs; ++outer) {
        if (outer > 0) {
            const resid_out o = residual_pass<NT>(n, fconst, as, xs, rs, red, disc);
            rel = sqrt(o.rr) / sqrt(o.bb);
            sx = o.sx;
            if (!isfinite(rel)) {
                st |= ST_NONFINITE;
                break;
            }
            if (rel < eps) {
                st |= ST_CONVERGED;
                break;
            }
            if (it >= maxit || outer > max_outer) {
                st |= ST_IMAX;
                break;
            }
            if (!(rel < prev)) {
                st |= ST_STALL;
                break;
            }
        }
        prev = rel;
        const double tau = LOW ? fmax(0.5 * eps / rel, 1e-5) : 0.9 * eps / rel;
        // inner MINRES on Ahat y = c, c = S r: y = 0, v_1 = c / b_1
        int iv = 2, ivp = 1, ip1 = 3, ip2 = 4;
        double cc = 0.0, dummy = 0.0;
        for (int e = t; e < N; e += NT) {
            const double cv = ((e % M) < m) ? scs[e] * rs[e] : 0.0;
            V(ivp)[e] = (T)0;
            V(ip1)[e] = (T)0;
            V(ip2)[e] = (T)0;
            yv[e] = (T)0;
            cc += cv * cv;
        }
        wg_sum2_fast<NT>(cc, dummy, slots, phase);
        const double b1 = sqrt(cc);
        if (!(b1 > 0.0)) continue;  // r = 0: the next residual pass decides
        {
            const double inv = 1.0 / b1;
            for (int e = t; e < N; e += NT) V(iv)[e] = (T)(((e % M) < m) ? scs[e] * rs[e] * inv : 0.0);
        }
        double bk = 0.0, hh = b1;
        double c1 = 1.0, s1 = 0.0, c2 = 1.0, s2 = 0.0;
        __syncthreads();
        for (;;) {
            ++it;
            T *v = V(iv), *u = V(ivp);
            // u = Ahat v - b_k v_{k-1} (in the v_{k-1} buffer), a_k = v^T u
            double al = 0.0, vv = 0.0;
            for (int e = t; e < N; e += NT) {
                const int i = e % M, j = e / M;
                double av = 0.0;
                if (i < m) {
                    av = (double)v[e];
                    if (i + 1 < m) av += (double)gT[e] * (double)v[e + 1];
                    if (i > 0) av += (double)gT[e - 1] * (double)v[e - 1];
                    if (j > 0) av += (double)bT[e] * (double)v[e - M];
                    if (j + 1 < m) av += (double)bT[e + M] * (double)v[e + M];
                }
                const double uv = av - bk * (double)u[e];
                u[e] = (T)uv;
                al += (double)v[e] * uv;
            }
            wg_sum2_fast<NT>(al, vv, slots, phase);
            // u -= a_k v, b_{k+1} = ||u||
            double nb = 0.0, d2 = 0.0;
            for (int e = t; e < N; e += NT) {
                const double uv = (double)u[e] - al * (double)v[e];
                u[e] = (T)uv;
                nb += (double)u[e] * (double)u[e];
            }
            wg_sum2_fast<NT>(nb, d2, slots, phase);
            const double bk1 = sqrt(nb);
            // column k of T_k through the previous two rotations, the new rotation
            const double ek = s2 * bk, tt = c2 * bk;
            const double dk = c1 * tt + s1 * al;
            const double gk = c1 * al - s1 * tt;
            const double rk = fmax(sqrt(gk * gk + bk1 * bk1), 1e-300);
            const double ck = gk / rk, sk = bk1 / rk;
            const double step = ck * hh;
            hh = -sk * hh;
            // p_k (into the p_{k-2} buffer), y += step p_k, v_{k+1} = u / b_{k+1} (in place)
            T *p1 = V(ip1), *p2 = V(ip2);
            const double rinv = 1.0 / rk, binv = bk1 > 0.0 ? 1.0 / bk1 : 0.0;
            for (int e = t; e < N; e += NT) {
                const double pv = ((double)v[e] - dk * (double)p1[e] - ek * (double)p2[e]) * rinv;
                p2[e] = (T)pv;
                yv[e] = (T)((double)yv[e] + step * pv);
                u[e] = (T)((double)u[e] * binv);
            }
            // rotate: the p_{k-2} buffer now holds p_k, the v_{k-1} buffer v_{k+1}
            const int tp = ip1;
            ip1 = ip2;
            ip2 = tp;
            const int tv = iv;
            iv = ivp;
            ivp = tv;
            c2 = c1;
            s2 = s1;
            c1 = ck;
            s1 = sk;
            bk = bk1;
            __syncthreads();
            if (fabs(hh) < tau * b1 || !(bk1 > 0.0) || it >= maxit || !isfinite(hh)) break;
        }
        // x += S y (FP64)
        for (int e = t; e < N; e += NT)
            if ((e % M) < m) xs[e] += scs[e] * (double)yv[e];
        __syncthreads();
    }
    if (zero_rhs) {
        rel = 0.0;
        sx = 0.0;
        st |= ST_CONVERGED;
    }
    if (t == 0) {
        state[s] = st | ST_DONE;
        relres[s] = rel;
        q[s] = h * h * sx;
        if (iters) iters[s] = it;
    }
}

template <typename T>
hipError_t launch_minres_t(int n, int S, double fconst, const double *a, const double *sc, const double *gam,
                           const double *beta, double *x, double *r, void *vecs, double eps, int maxit,
                           int max_outer, const int *idx, const int *count, uint32_t *state, double *relres,
                           double *q, int32_t *iters, int disc, hipStream_t st)
{
    if (n >= 64)
        hipLaunchKernelGGL((k_minres_ir<T, 1024>), dim3(S), dim3(1024), 0, st, n, fconst, a, sc, gam, beta, x, r,
                           (T *)vecs, eps, maxit, max_outer, idx, count, state, relres, q, iters, disc);
    else
        hipLaunchKernelGGL((k_minres_ir<T, 256>), dim3(S), dim3(256), 0, st, n, fconst, a, sc, gam, beta, x, r,
                           (T *)vecs, eps, maxit, max_outer, idx, count, state, relres, q, iters, disc);
    return hipGetLastError();
}

hipError_t launch_minres(int n, int S, double fconst, const double *a, const double *sc,
                         const double *gam, const double *beta, double *x, double *r, void *vecs,
                         int low, double eps, int maxit, int max_outer, const int *idx, const int *count,
                         uint32_t *state, double *relres, double *q, int32_t *iters, int disc, hipStream_t st)
{
    if (S == 0) return hipSuccess;
    return low ? launch_minres_t<float>(n, S, fconst, a, sc, gam, beta, x, r, vecs, eps, maxit, max_outer, idx,
                                        count, state, relres, q, iters, disc, st)
               : launch_minres_t<double>(n, S, fconst, a, sc, gam, beta, x, r, vecs, eps, maxit, max_outer, idx,
                                         count, state, relres, q, iters, disc, st);
}

}  // namespace mlmc
