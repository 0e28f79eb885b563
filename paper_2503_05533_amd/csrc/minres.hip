// Batched MINRES (Sec. 2.2: the Krylov solver of the paper's iterative
// experiments, stopped on the relative residual), one workgroup per sample.
//
// MINRES (Paige and Saunders, 1975) runs on the diagonally scaled system
// Ahat xhat = S b, Ahat = S A S, S = diag(A)^(-1/2) (Jacobi preconditioning
// that keeps the operator symmetric).  Ahat is applied matrix-free from the
// scaled couplings gam (right neighbour) and beta (row below) in the padded
// block layout.  The Lanczos vectors, search directions and iterate are
// FP64 vectors in the workspace; dot products are fixed-order workgroup sums.
// The iteration stops when the recurrence estimate of the scaled relative
// residual drops below eps; the true FP64 relative residual of x = S xhat in
// the unscaled system is then computed and the iteration continues (checking
// every 8 iterations) until it is below eps as well, or maxit is reached.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ir_common.h"
#include "kernels.h"

namespace mlmc {

template <int NT>
__global__ __launch_bounds__(NT) void k_minres(int n, double fconst, const double *__restrict__ a,
                                               const double *__restrict__ sc,
                                               const double *__restrict__ gam,
                                               const double *__restrict__ beta,
                                               double *__restrict__ x, double *__restrict__ r,
                                               double *__restrict__ vecs, double eps, int maxit,
                                               uint32_t *__restrict__ state,
                                               double *__restrict__ relres,
                                               double *__restrict__ q, int32_t *__restrict__ iters)
{
    __shared__ double red[NT];
    const int m = n - 1, M = n;
    const int N = m * M;
    const int s = blockIdx.x;
    const size_t vo = (size_t)s * N;
    const double *scs = sc + vo, *gs = gam + vo, *bs = beta + vo;
    double *xs = x + vo, *rsb = r + vo;
    // 7 work vectors per sample: xhat, v, r1, r2, w, w1, w2 (roles rotate by index)
    double *base = vecs + (size_t)s * 7 * N;
    double *xh = base, *v = base + (size_t)N;
    int ir1 = 2, ir2 = 3, iw = 4, iw1 = 5, iw2 = 6;
    auto V = [&](int k) { return base + (size_t)k * N; };
    const double *as = a + (size_t)s * (n + 1) * (n + 1);
    const double h = 1.0 / n, bval = h * h * fconst;
    const int t = threadIdx.x;

    // xhat = 0, r1 = r2 = bhat = S b, w = w1 = w2 = 0
    double bb = 0.0;
    for (int e = t; e < N; e += NT) {
        const double bh = ((e % M) < m) ? scs[e] * bval : 0.0;
        V(ir1)[e] = bh;
        V(ir2)[e] = bh;
        xh[e] = 0.0;
        V(iw)[e] = 0.0;
        V(iw1)[e] = 0.0;
        V(iw2)[e] = 0.0;
        bb += bh * bh;
    }
    bb = wg_sum<NT>(bb, red);
    const double beta1 = sqrt(bb);
    double beta_k = beta1, oldb = 0.0, dbar = 0.0, epsln = 0.0, phibar = beta1;
    double cs = -1.0, sn = 0.0;
    uint32_t st = state[s] & ~(uint32_t)ST_DONE;
    double rel = INFINITY, sx = 0.0;
    int it = 0, next_check = -1;
    bool done = !(beta1 > 0.0);
    while (!done) {
        ++it;
        // Lanczos step: v = r2 / beta; y = Ahat v - (beta/oldb) r1 - (alfa/beta) r2
        double *r1 = V(ir1), *r2 = V(ir2);
        const double sinv = 1.0 / beta_k;
        for (int e = t; e < N; e += NT) v[e] = r2[e] * sinv;
        __syncthreads();
        const double cb = it >= 2 ? beta_k / oldb : 0.0;
        double alfa = 0.0;
        for (int e = t; e < N; e += NT) {
            const int i = e % M, j = e / M;
            double av = v[e];
            if (i < m) {
                if (i + 1 < m) av += gs[e] * v[e + 1];
                if (i > 0) av += gs[e - 1] * v[e - 1];
                if (j > 0) av += bs[e] * v[e - M];
                if (j + 1 < m) av += bs[e + M] * v[e + M];
            }
            const double yv = av - cb * r1[e];
            r1[e] = yv;  // the r1 buffer now holds y
            alfa += v[e] * yv;
        }
        alfa = wg_sum<NT>(alfa, red);
        const double ca = alfa / beta_k;
        double nb = 0.0;
        for (int e = t; e < N; e += NT) {
            const double yv = r1[e] - ca * r2[e];
            r1[e] = yv;
            nb += yv * yv;
        }
        nb = wg_sum<NT>(nb, red);
        // r1 <- r2, r2 <- y
        const int tr = ir1;
        ir1 = ir2;
        ir2 = tr;
        oldb = beta_k;
        beta_k = sqrt(nb);
        // QR update by a plane rotation
        const double oldeps = epsln;
        const double delta = cs * dbar + sn * alfa;
        const double gbar = sn * dbar - cs * alfa;
        epsln = sn * beta_k;
        dbar = -cs * beta_k;
        const double gamma = fmax(sqrt(gbar * gbar + beta_k * beta_k), 1e-300);
        cs = gbar / gamma;
        sn = beta_k / gamma;
        const double phi = cs * phibar;
        phibar = sn * phibar;
        const double dinv = 1.0 / gamma;
        // w1 <- w2, w2 <- w, w = (v - oldeps w1 - delta w2) / gamma, xhat += phi w
        const int tw = iw1;
        iw1 = iw2;
        iw2 = iw;
        iw = tw;
        double *w = V(iw), *w1 = V(iw1), *w2 = V(iw2);
        for (int e = t; e < N; e += NT) {
            const double wn = (v[e] - oldeps * w1[e] - delta * w2[e]) * dinv;
            w[e] = wn;
            xh[e] += phi * wn;
        }
        const bool est_ok = phibar < eps * beta1;
        const bool check = (est_ok && next_check < 0) || (next_check >= 0 && it >= next_check) ||
                           it >= maxit || !(beta_k > 0.0);
        if (check) {
            // true FP64 relative residual of x = S xhat in the unscaled system
            for (int e = t; e < N; e += NT) xs[e] = scs[e] * xh[e];
            __syncthreads();
            const resid_out o = residual_pass<NT>(n, fconst, as, xs, rsb, red);
            rel = sqrt(o.rr) / sqrt(o.bb);
            sx = o.sx;
            if (!isfinite(rel)) {
                st |= ST_NONFINITE;
                done = true;
            } else if (rel < eps) {
                st |= ST_CONVERGED;
                done = true;
            } else if (it >= maxit || !(beta_k > 0.0)) {
                st |= ST_IMAX;
                done = true;
            } else {
                next_check = it + 8;
            }
        }
        __syncthreads();
    }
    if (!(beta1 > 0.0)) {
        for (int e = t; e < N; e += NT) xs[e] = 0.0;
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

hipError_t launch_minres(int n, int S, double fconst, const double *a, const double *sc,
                         const double *gam, const double *beta, double *x, double *r, double *vecs,
                         double eps, int maxit, uint32_t *state, double *relres, double *q,
                         int32_t *iters, hipStream_t st)
{
    if (S == 0) return hipSuccess;
    hipLaunchKernelGGL((k_minres<256>), dim3(S), dim3(256), 0, st, n, fconst, a, sc, gam, beta, x, r,
                       vecs, eps, maxit, state, relres, q, iters);
    return hipGetLastError();
}

}  // namespace mlmc
