// Batched conjugate gradients preconditioned by a geometric multigrid
// V-cycle: a solver whose cost grows like the number of unknowns (gamma = 2
// in the cost model of Sec. 4.4, the regime beta > gamma in which the
// cost-savings corollary predicts its largest gains), in mixed precision:
// CG, its vectors and the operator in FP64, the multigrid preconditioner in
// FP32.  One workgroup per sample.
//
// Vectors live on the (n+1)^2 nodes of a grid (boundary entries 0).  The
// operator is the 5-point matrix of the library's edge rule (node_faces:
// finite volumes or P1 elements), applied matrix-free from the nodal
// coefficient.  Multigrid levels n, n/2, ..., 2 cells per side: level 0
// takes its edge coefficients from the same rule; a coarse edge joins coarse
// nodes two fine cells apart, and gets the harmonic mean of the two fine
// edges it spans (series conduction), averaged with weights 1/4, 1/2, 1/4
// over the fine edge rows (columns) at and beside it.  Smoother: red-black
// Gauss-Seidel, two sweeps red-then-black before the coarse correction and
// two black-then-red after it, so the V-cycle is a symmetric
// preconditioner; restriction by the transpose of bilinear interpolation,
// prolongation bilinear; the 2-cell grid has one unknown, solved exactly by
// one sweep.  CG stops when its recursive residual, and then the true FP64
// residual ||b - A x|| / ||b||, are below eps (strict).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ir_common.h"
#include "kernels.h"

namespace mlmc {

namespace {

constexpr int kMgMaxLevels = 9;  // 256 cells per side down to 2

// Offsets (in floats) of level l's arrays inside a sample's multigrid block:
// x-edges [(nl+1) * nl], y-edges [nl * (nl+1)], u, f, r [(nl+1)^2].
struct mg_level { int n; size_t ex, ey, u, f, r; };

__host__ __device__ inline int mg_levels(int n)
{
    int L = 0;
    while ((n >> L) >= 2) ++L;
    return L;  // levels 0 .. L-1, the last one has 2 cells per side
}

__host__ __device__ inline size_t mg_level_offsets(int n, mg_level *lv)
{
    size_t off = 0;
    const int L = mg_levels(n);
    for (int l = 0; l < L; ++l) {
        const int nl = n >> l, np = nl + 1;
        mg_level d;
        d.n = nl;
        d.ex = off;
        off += (size_t)np * nl;
        d.ey = off;
        off += (size_t)np * nl;
        d.u = off;
        off += (size_t)np * np;
        d.f = off;
        off += (size_t)np * np;
        d.r = off;
        off += (size_t)np * np;
        if (lv) lv[l] = d;
    }
    return (off + 63) & ~(size_t)63;
}

// Fixed-order workgroup sum: xor butterfly per wave, wave partials in order.
template <int NT>
__device__ inline double mg_sum(double v, double (*slots)[NT / 64], int &phase)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) slots[phase][threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) s += slots[phase][k];
    phase ^= 1;
    return s;
}

// One colour of a red-black Gauss-Seidel sweep on level d (colour = parity
// of ix + iy), interior nodes only.
template <int NT>
__device__ inline void mg_sweep(float *base, const mg_level &d, int colour)
{
    const int nl = d.n, np = nl + 1, m = nl - 1;
    const float *ex = base + d.ex, *ey = base + d.ey, *f = base + d.f;
    float *u = base + d.u;
    for (int k = threadIdx.x; k < m * m; k += NT) {
        const int iy = k / m + 1, ix = k % m + 1;
        if (((ix + iy) & 1) != colour) continue;
        const int p = iy * np + ix;
        const float w = ex[iy * nl + ix - 1], e = ex[iy * nl + ix];
        const float s = ey[(iy - 1) * np + ix], nn = ey[iy * np + ix];
        u[p] = (f[p] + w * u[p - 1] + e * u[p + 1] + s * u[p - np] + nn * u[p + np]) / (w + e + s + nn);
    }
    __syncthreads();
}

// r = f - A u on level d (interior nodes; boundary r = 0 is kept from the set-up).
template <int NT>
__device__ inline void mg_residual(float *__restrict__ base, const mg_level &d)
{
    const int nl = d.n, np = nl + 1, m = nl - 1;
    const float *ex = base + d.ex, *ey = base + d.ey, *f = base + d.f, *u = base + d.u;
    float *r = base + d.r;
    for (int k = threadIdx.x; k < m * m; k += NT) {
        const int iy = k / m + 1, ix = k % m + 1;
        const int p = iy * np + ix;
        const float w = ex[iy * nl + ix - 1], e = ex[iy * nl + ix];
        const float s = ey[(iy - 1) * np + ix], nn = ey[iy * np + ix];
        r[p] = f[p] - ((w + e + s + nn) * u[p] - w * u[p - 1] - e * u[p + 1] - s * u[p - np] - nn * u[p + np]);
    }
    __syncthreads();
}

// Coarse right-hand side f_c = P^T r_f (weights 1, 1/2, 1/4 around the
// coincident fine node) and u_c = 0, on the interior coarse nodes.
template <int NT>
__device__ inline void mg_restrict(float *__restrict__ base, const mg_level &fd, const mg_level &cd)
{
    const int npf = fd.n + 1, nc = cd.n, npc = nc + 1, mc = nc - 1;
    const float *r = base + fd.r;
    float *fc = base + cd.f, *uc = base + cd.u;
    for (int k = threadIdx.x; k < mc * mc; k += NT) {
        const int J = k / mc + 1, I = k % mc + 1;
        const int q = (2 * J) * npf + 2 * I;
        const float v = r[q] + 0.5f * (r[q - 1] + r[q + 1] + r[q - npf] + r[q + npf]) +
                        0.25f * (r[q - npf - 1] + r[q - npf + 1] + r[q + npf - 1] + r[q + npf + 1]);
        fc[J * npc + I] = v;
        uc[J * npc + I] = 0.0f;
    }
    __syncthreads();
}

// u_f += P u_c (bilinear), interior fine nodes.
template <int NT>
__device__ inline void mg_prolong(float *__restrict__ base, const mg_level &fd, const mg_level &cd)
{
    const int nf = fd.n, npf = nf + 1, mf = nf - 1, npc = cd.n + 1;
    const float *uc = base + cd.u;
    float *uf = base + fd.u;
    for (int k = threadIdx.x; k < mf * mf; k += NT) {
        const int iy = k / mf + 1, ix = k % mf + 1;
        const int I = ix >> 1, J = iy >> 1;
        const float c00 = uc[J * npc + I];
        float v;
        if (!(ix & 1) && !(iy & 1)) {
            v = c00;
        } else if (ix & 1 && !(iy & 1)) {
            v = 0.5f * (c00 + uc[J * npc + I + 1]);
        } else if (!(ix & 1)) {
            v = 0.5f * (c00 + uc[(J + 1) * npc + I]);
        } else {
            v = 0.25f * (c00 + uc[J * npc + I + 1] + uc[(J + 1) * npc + I] + uc[(J + 1) * npc + I + 1]);
        }
        uf[iy * npf + ix] += v;
    }
    __syncthreads();
}

}  // namespace

size_t mgcg_floats_per_sample(int n) { return mg_level_offsets(n, nullptr); }

template <int NT>
__global__ __launch_bounds__(NT) void k_mgcg(int n, double fconst, const double *__restrict__ a,
                                             double *__restrict__ xout, double *__restrict__ vecs,
                                             float *__restrict__ mg, double eps, int maxit,
                                             uint32_t *__restrict__ state, double *__restrict__ relres,
                                             double *__restrict__ q, int32_t *__restrict__ iters, int disc)
{
    __shared__ double slots[2][NT / 64];
    const int np = n + 1, m = n - 1, M = n, P = np * np;
    const int s = blockIdx.x, t = threadIdx.x;
    const double *as = a + (size_t)s * P;
    double *x = vecs + (size_t)s * 5 * P, *r = x + P, *pv = r + P, *qv = pv + P, *z = qv + P;
    mg_level lv[kMgMaxLevels];
    const size_t per = mg_level_offsets(n, lv);
    const int L = mg_levels(n);
    float *base = mg + (size_t)s * per;
    const double h = 1.0 / n, bval = h * h * fconst;
    int phase = 0;

    // level-0 edges from the edge rule, coarse edges by series and row averages
    {
        const mg_level &d = lv[0];
        for (int k = t; k < np * n; k += NT) {
            const int iy = k / n, ix = k % n;  // x-edge (ix, iy)-(ix+1, iy)
            const bool used = iy >= 1 && iy <= m;
            const int pl = iy * np + ix;
            double v = 0.0;
            if (used) {
                const double aL = as[pl], aR = as[pl + 1];
                v = disc ? face_x(1, aL, aR, as[pl + np + 1], as[pl - np]) : hmean2(aL, aR);
            }
            base[d.ex + iy * n + ix] = (float)v;
        }
        for (int k = t; k < n * np; k += NT) {
            const int iy = k / np, ix = k % np;  // y-edge (ix, iy)-(ix, iy+1)
            const bool used = ix >= 1 && ix <= m;
            const int pb = iy * np + ix;
            double v = 0.0;
            if (used) {
                const double aB = as[pb], aT = as[pb + np];
                v = disc ? face_y(1, aB, aT, as[pb + np + 1], as[pb - 1]) : hmean2(aB, aT);
            }
            base[d.ey + iy * np + ix] = (float)v;
        }
        for (int k = t; k < np * np; k += NT) base[d.r + k] = 0.0f;
        __syncthreads();
    }
    for (int l = 1; l < L; ++l) {
        const mg_level &fd = lv[l - 1], &cd = lv[l];
        const int nf = fd.n, npf = nf + 1, nc = cd.n, npc = nc + 1;
        auto hm = [](float p, float qq) { return (p > 0.0f && qq > 0.0f) ? 2.0f * p * qq / (p + qq) : 0.0f; };
        for (int k = t; k < npc * nc; k += NT) {
            const int J = k / nc, I = k % nc;  // coarse x-edge (I, J)-(I+1, J): fine row 2J, columns 2I, 2I+1
            float v = 0.0f, wsum = 0.0f;
            for (int dr = -1; dr <= 1; ++dr) {
                const int fr = 2 * J + dr;
                if (fr < 0 || fr > nf) continue;
                const float wgt = dr == 0 ? 0.5f : 0.25f;
                v += wgt * hm(base[fd.ex + fr * nf + 2 * I], base[fd.ex + fr * nf + 2 * I + 1]);
                wsum += wgt;
            }
            base[cd.ex + J * nc + I] = (J >= 1 && J < nc) ? v / wsum : 0.0f;
        }
        for (int k = t; k < nc * npc; k += NT) {
            const int J = k / npc, I = k % npc;  // coarse y-edge (I, J)-(I, J+1): fine column 2I, rows 2J, 2J+1
            float v = 0.0f, wsum = 0.0f;
            for (int dc = -1; dc <= 1; ++dc) {
                const int fc = 2 * I + dc;
                if (fc < 0 || fc > nf) continue;
                const float wgt = dc == 0 ? 0.5f : 0.25f;
                v += wgt * hm(base[fd.ey + (2 * J) * npf + fc], base[fd.ey + (2 * J + 1) * npf + fc]);
                wsum += wgt;
            }
            base[cd.ey + J * npc + I] = (I >= 1 && I < nc) ? v / wsum : 0.0f;
        }
        for (int k = t; k < npc * npc; k += NT) {
            base[cd.r + k] = 0.0f;
            base[cd.u + k] = 0.0f;
            base[cd.f + k] = 0.0f;
        }
        __syncthreads();
    }

    // z = M^{-1} r: one V-cycle from u = 0 on the FP32 hierarchy
    auto vcycle = [&]() {
        const mg_level &d0 = lv[0];
        for (int k = t; k < P; k += NT) {
            base[d0.f + k] = (float)r[k];
            base[d0.u + k] = 0.0f;
        }
        __syncthreads();
        for (int l = 0; l + 1 < L; ++l) {
            mg_sweep<NT>(base, lv[l], 0);
            mg_sweep<NT>(base, lv[l], 1);
            mg_sweep<NT>(base, lv[l], 0);
            mg_sweep<NT>(base, lv[l], 1);
            mg_residual<NT>(base, lv[l]);
            mg_restrict<NT>(base, lv[l], lv[l + 1]);
        }
        mg_sweep<NT>(base, lv[L - 1], 0);  // one unknown: exact
        mg_sweep<NT>(base, lv[L - 1], 1);
        for (int l = L - 2; l >= 0; --l) {
            mg_prolong<NT>(base, lv[l], lv[l + 1]);
            mg_sweep<NT>(base, lv[l], 1);
            mg_sweep<NT>(base, lv[l], 0);
            mg_sweep<NT>(base, lv[l], 1);
            mg_sweep<NT>(base, lv[l], 0);
        }
        for (int k = t; k < P; k += NT) z[k] = (double)base[d0.u + k];
        __syncthreads();
    };
    // y = A v (FP64, interior nodes; boundary 0)
    auto apply = [&](const double *v, double *y) {
        for (int k = t; k < P; k += NT) {
            const int iy = k / np, ix = k % np;
            double o = 0.0;
            if (ix >= 1 && ix <= m && iy >= 1 && iy <= m) {
                const faces4 f = node_faces(disc, as, k, np);
                o = (f.w + f.e + f.s + f.n) * v[k] - f.w * v[k - 1] - f.e * v[k + 1] - f.s * v[k - np] -
                    f.n * v[k + np];
            }
            y[k] = o;
        }
        __syncthreads();
    };

    // CG: x = 0, r = b
    double bb = 0.0;
    for (int k = t; k < P; k += NT) {
        const int iy = k / np, ix = k % np;
        const bool in = ix >= 1 && ix <= m && iy >= 1 && iy <= m;
        x[k] = 0.0;
        r[k] = in ? bval : 0.0;
        bb += in ? bval * bval : 0.0;
    }
    bb = mg_sum<NT>(bb, slots, phase);
    __syncthreads();
    uint32_t st = state[s] & ~(uint32_t)ST_DONE;
    double rel = 1.0, target = eps;
    int it = 0;
    if (!(bb > 0.0)) {
        rel = 0.0;
        st |= ST_CONVERGED;
    } else {
        vcycle();
        double rho = 0.0;
        for (int k = t; k < P; k += NT) {
            pv[k] = z[k];
            rho += r[k] * z[k];
        }
        rho = mg_sum<NT>(rho, slots, phase);
        __syncthreads();
        for (;;) {
            ++it;
            apply(pv, qv);
            double pq = 0.0;
            for (int k = t; k < P; k += NT) pq += pv[k] * qv[k];
            pq = mg_sum<NT>(pq, slots, phase);
            const double alpha = rho / pq;
            double rr = 0.0;
            for (int k = t; k < P; k += NT) {
                x[k] += alpha * pv[k];
                r[k] -= alpha * qv[k];
                rr += r[k] * r[k];
            }
            rr = mg_sum<NT>(rr, slots, phase);
            __syncthreads();
            rel = sqrt(rr / bb);
            if (!isfinite(rel)) {
                st |= ST_NONFINITE;
                break;
            }
            if (rel < target) {
                // confirm with the true residual b - A x
                apply(x, qv);
                double tr = 0.0;
                for (int k = t; k < P; k += NT) {
                    const int iy = k / np, ix = k % np;
                    const bool in = ix >= 1 && ix <= m && iy >= 1 && iy <= m;
                    const double d = in ? bval - qv[k] : 0.0;
                    tr += d * d;
                }
                tr = mg_sum<NT>(tr, slots, phase);
                __syncthreads();
                rel = sqrt(tr / bb);
                if (rel < eps) {
                    st |= ST_CONVERGED;
                    break;
                }
                target *= 0.5;  // the recursive residual was optimistic
            }
            if (it >= maxit) {
                st |= ST_IMAX;
                break;
            }
            vcycle();
            double rz = 0.0;
            for (int k = t; k < P; k += NT) rz += r[k] * z[k];
            rz = mg_sum<NT>(rz, slots, phase);
            const double beta = rz / rho;
            rho = rz;
            for (int k = t; k < P; k += NT) pv[k] = z[k] + beta * pv[k];
            __syncthreads();
        }
    }
    // x into the padded unknown layout; Q = h^2 sum x
    double sx = 0.0;
    for (int e = t; e < m * M; e += NT) {
        const int j = e / M, i = e % M;
        const double v = i < m ? x[(j + 1) * np + (i + 1)] : 0.0;
        xout[(size_t)s * m * M + e] = v;
        sx += v;
    }
    sx = mg_sum<NT>(sx, slots, phase);
    if (t == 0) {
        state[s] = st | ST_DONE;
        relres[s] = rel;
        q[s] = h * h * sx;
        if (iters) iters[s] = it;
    }
}

hipError_t launch_mgcg(int n, int S, double fconst, const double *a, double *x, double *vecs, float *mg,
                       double eps, int maxit, uint32_t *state, double *relres, double *q, int32_t *iters, int disc,
                       hipStream_t st)
{
    if (S == 0) return hipSuccess;
    if (mg_levels(n) > kMgMaxLevels) return hipErrorInvalidValue;
    if (n >= 64)
        hipLaunchKernelGGL((k_mgcg<1024>), dim3(S), dim3(1024), 0, st, n, fconst, a, x, vecs, mg, eps, maxit, state,
                           relres, q, iters, disc);
    else
        hipLaunchKernelGGL((k_mgcg<256>), dim3(S), dim3(256), 0, st, n, fconst, a, x, vecs, mg, eps, maxit, state,
                           relres, q, iters, disc);
    return hipGetLastError();
}

}  // namespace mlmc
