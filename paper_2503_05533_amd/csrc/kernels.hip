// HIP kernels (gfx950) of the batched per-level sample solve.
//
// Per grid with n cells per side: m = n-1 unknowns per grid row, the
// unknowns of grid row j form block j (0 <= j < m), and every block is padded
// to M = n entries (entry m is an identity pad).  Internal vectors use that
// padded layout: index j*M + i, i = ix-1, j = iy-1.
//
// The symmetric positive definite system A x = b is block tridiagonal.  With
// the diagonal scaling S = diag(A)^(-1/2) (Ahat = S A S has unit diagonal):
//   Ahat_jj = T_j  (tridiagonal: 1 on the diagonal, gam_j[i] between i, i+1)
//   Ahat_j,j-1 = diag(beta_j)  (coupling to the grid row below)
// Block elimination: Schur complements C_0 = T_0,
//   C_j = T_j - diag(beta_j) C_{j-1}^{-1} diag(beta_j),
// each C_j is inverted in place by the symmetric sweep (Gauss-Jordan) operator
// and -C_j^{-1} is stored as the factor of block j.  Solves are then two
// sweeps of symmetric block mat-vecs (forward: z_j = C_j^{-1}(s r_j -
// beta_j z_{j-1}); back: x_j = z_j - C_j^{-1} beta_{j+1} x_{j+1}).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include "dtypes.h"
#include "kernels.h"
#include "ir_common.h"

namespace mlmc {

// ------------------------------------------------------------------ helpers


// Tile t of the lower block triangle, enumerated row by row: t = I(I+1)/2 + J.
__device__ inline void tile_of(int t, int &I, int &J)
{
    int i = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    I = i;
    J = t - i * (i + 1) / 2;
}

template <int NT>
__device__ inline double block_sum(double v, double *red)
{
    // fixed-order tree reduction (deterministic)
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

// ------------------------------------------------------------------ xi

__device__ inline uint64_t splitmix_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_fill_xi(uint64_t seed, int level, int64_t first, int64_t n, int K, double *xi)
{
    const int npair = (K + 1) / 2;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n * npair) return;
    const int64_t s = g / npair;
    const int p = (int)(g % npair);
    const uint64_t sample = (uint64_t)(first + s);
    const uint64_t base = ((((uint64_t)level << 32) | sample) << 8 | (uint64_t)p) << 1;
    const uint64_t o0 = splitmix_mix(seed + (base + 1ull) * 0x9E3779B97F4A7C15ull);
    const uint64_t o1 = splitmix_mix(seed + ((base | 1ull) + 1ull) * 0x9E3779B97F4A7C15ull);
    const double u1 = ((double)(o0 >> 11) + 1.0) * 0x1.0p-53;
    const double u2 = (double)(o1 >> 11) * 0x1.0p-53;
    const double r = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincos(2.0 * M_PI * u2, &sn, &cs);
    xi[s * K + 2 * p] = r * cs;
    if (2 * p + 1 < K) xi[s * K + 2 * p + 1] = r * sn;
}

// ------------------------------------------------------------------ GEMMs

// C[i][j] = epi(sum_l A[i][l] * B(l, j)), A row-major [R x L];
// B(l,j) = B[l*ldb + j] (BT = false) or B[j*ldb + l] (BT = true).
// 64 x 64 output tile per 256 threads, 4 x 4 per thread, L chunks of 16.
// EPI 0: exp (coefficient field), EPI 1: scale row i by rowscale[i] (or 1).
template <bool BT, int EPI>
__global__ __launch_bounds__(256) void k_gemm64(int R, int Cn, int L, const double *__restrict__ A,
                                                 int lda, const double *__restrict__ B, int ldb,
                                                 double *__restrict__ C, int ldc,
                                                 const double *__restrict__ rowscale)
{
    __shared__ double As[16][64 + 1];
    __shared__ double Bs[16][64 + 1];
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
    double acc[4][4] = {};
    for (int l0 = 0; l0 < L; l0 += 16) {
        for (int e = t; e < 1024; e += 256) {
            int rr = e >> 4, ll = e & 15;
            int gr = r0 + rr, gl = l0 + ll;
            As[ll][rr] = (gr < R && gl < L) ? A[(size_t)gr * lda + gl] : 0.0;
        }
        if (BT) {
            for (int e = t; e < 1024; e += 256) {
                int cc = e >> 4, ll = e & 15;
                int gc = c0 + cc, gl = l0 + ll;
                Bs[ll][cc] = (gc < Cn && gl < L) ? B[(size_t)gc * ldb + gl] : 0.0;
            }
        } else {
            for (int e = t; e < 1024; e += 256) {
                int ll = e >> 6, cc = e & 63;
                int gc = c0 + cc, gl = l0 + ll;
                Bs[ll][cc] = (gc < Cn && gl < L) ? B[(size_t)gl * ldb + gc] : 0.0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int ll = 0; ll < 16; ++ll) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[ll][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[ll][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int gr = r0 + ty * 4 + i;
        if (gr >= R) continue;
        double sc = (EPI == 1 && rowscale) ? rowscale[gr] : 1.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int gc = c0 + tx + 16 * j;
            if (gc < Cn) C[(size_t)gr * ldc + gc] = EPI == 0 ? exp(acc[i][j]) : sc * acc[i][j];
        }
    }
}

// ------------------------------------------------------------------ assembly

// Scaled block coefficients from the nodal coefficient a[(n+1)^2]:
// sc = diag(A)^(-1/2), gam (to the right neighbour), beta (to the row below).
// Diagonal scaling S = diag(A)^(-1/2) of the 5-point operator, one thread per
// padded unknown (x = sample, y = block of unknowns): A_PP is the sum of the
// four edge coefficients around node P (harmonic means, or the P1 rule for
// disc 1: node_faces).
__global__ void k_scale(int n, const double *__restrict__ a, double *__restrict__ sc, int disc)
{
    const int m = n - 1, M = n, np = n + 1;
    const int s = blockIdx.x, e = blockIdx.y * blockDim.x + threadIdx.x;
    if (e >= m * M) return;
    const int j = e / M, i = e % M;
    const size_t o = (size_t)s * m * M + e;
    if (i >= m) {
        sc[o] = 0.0;
        return;
    }
    const double *as = a + (size_t)s * np * np;
    const int p = (j + 1) * np + (i + 1);
    const faces4 f = node_faces(disc, as, p, np);
    sc[o] = 1.0 / sqrt(f.w + f.e + f.s + f.n);
}

// Scaled couplings of S A S: gam to the right neighbour (same grid row), beta
// to the neighbour in the row below; 0 at the grid edge and in the pad.
__global__ void k_coeffs(int n, const double *__restrict__ a, const double *__restrict__ sc,
                         double *__restrict__ gam, double *__restrict__ beta, int disc)
{
    const int m = n - 1, M = n, np = n + 1;
    const int s = blockIdx.x, e = blockIdx.y * blockDim.x + threadIdx.x;
    if (e >= m * M) return;
    const int j = e / M, i = e % M;
    const size_t o = (size_t)s * m * M + e;
    if (i >= m) {
        gam[o] = 0.0;
        beta[o] = 0.0;
        return;
    }
    const double *as = a + (size_t)s * np * np;
    const int p = (j + 1) * np + (i + 1);
    const double sP = sc[o];
    const faces4 f = node_faces(disc, as, p, np);
    gam[o] = (i + 1 < m) ? -f.e * sP * sc[o + 1] : 0.0;
    beta[o] = (j > 0) ? -f.s * sP * sc[o - M] : 0.0;
}

// ------------------------------------------------------------------ factor

// One workgroup per sample.  The M x M working matrix lives in registers as
// TR x TR tiles of the lower block triangle (diagonal tiles full and kept
// symmetric), one tile per thread.  Each sweep pivot k: the owners of
// column k publish it to LDS (double-buffered by parity), one barrier, and
// every tile applies  X_il -= (x_ik / x_kk) x_kl  with the row/column k
// fix-ups of the sweep operator.  After all M pivots the tiles hold -C_j^{-1}.
template <typename Tst, int M, int TR, int NT>
__global__ __launch_bounds__(NT) void k_factor(int S, const double *__restrict__ beta,
                                               const double *__restrict__ gam,
                                               Tst *__restrict__ factor, const int *__restrict__ idx,
                                               const int *__restrict__ count, int64_t slot_base,
                                               uint32_t *__restrict__ state)
{
    using Tac = typename store_traits<Tst>::acc;
    constexpr int Tn = M / TR, T = Tn * (Tn + 1) / 2, E = TR * TR;
    constexpr int m = M - 1;
    __shared__ Tac colbuf[2][M];
    __shared__ Tac bj[M], gj[M];
    __shared__ int bad;
    const int b = blockIdx.x;
    if (count && b >= *count) return;
    const int s = idx ? idx[b] : b;
    const int64_t slot = slot_base + b;
    const int t = threadIdx.x;
    const bool active = t < T;
    int I = 0, J = 0;
    if (active) tile_of(t, I, J);
    const int i0 = I * TR, j0 = J * TR;
    const double *bs = beta + (size_t)s * m * M;
    const double *gs = gam + (size_t)s * m * M;
    Tst *fs = factor + (size_t)slot * m * T * E;
    if (t == 0) bad = 0;
    Tac tile[TR][TR];
#pragma unroll
    for (int r = 0; r < TR; ++r)
#pragma unroll
        for (int c = 0; c < TR; ++c) tile[r][c] = 0;

    for (int j = 0; j < m; ++j) {
        for (int i = t; i < M; i += NT) {
            bj[i] = (Tac)bs[j * M + i];
            gj[i] = (Tac)gs[j * M + i];
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int r = 0; r < TR; ++r)
#pragma unroll
                for (int c = 0; c < TR; ++c) {
                    const int gi = i0 + r, gc = j0 + c;
                    const Tac g_i = gj[gi], g_c = gj[gc];  // unconditional loads keep this branch-free
                    Tac tv = (gi == gc + 1) ? g_c : (Tac)0;
                    tv = (gc == gi + 1) ? g_i : tv;
                    tv = (gi == gc) ? (Tac)1 : tv;
                    tile[r][c] = bj[gi] * tile[r][c] * bj[gc] + tv;
                }
        }
        for (int K = 0; K < Tn; ++K) {
#pragma unroll
            for (int kk = 0; kk < TR; ++kk) {
                const int k = K * TR + kk;
                Tac *buf = colbuf[k & 1];
                if (active) {
                    if (I == K) {
#pragma unroll
                        for (int c = 0; c < TR; ++c) buf[j0 + c] = tile[kk][c];
                    } else if (J == K) {
#pragma unroll
                        for (int r = 0; r < TR; ++r) buf[i0 + r] = tile[r][kk];
                    }
                }
                __syncthreads();
                if (active) {
                    const Tac d = buf[k];
                    const Tac inv = recip(d);
                    Tac v[TR], cc[TR];
#pragma unroll
                    for (int r = 0; r < TR; ++r) v[r] = buf[i0 + r] * inv;
#pragma unroll
                    for (int c = 0; c < TR; ++c) cc[c] = buf[j0 + c];
#pragma unroll
                    for (int r = 0; r < TR; ++r)
#pragma unroll
                        for (int c = 0; c < TR; ++c) tile[r][c] = fma(-v[r], cc[c], tile[r][c]);
                    if (I == K) {
#pragma unroll
                        for (int c = 0; c < TR; ++c) tile[kk][c] = cc[c] * inv;
                    }
                    if (J == K) {
#pragma unroll
                        for (int r = 0; r < TR; ++r) tile[r][kk] = v[r];
                        if (I == K) {
                            tile[kk][kk] = -inv;
                            if (!(d > (Tac)0) || !isfinite(d)) bad = 1;
                        }
                    }
                }
            }
        }
        if (active) {
            Tst *fb = fs + (size_t)j * T * E;
#pragma unroll
            for (int r = 0; r < TR; ++r)
#pragma unroll
                for (int c = 0; c < TR; ++c) fb[(r * TR + c) * T + t] = store_traits<Tst>::store(tile[r][c]);
        }
        __syncthreads();
    }
    if (t == 0 && bad) atomicOr(&state[s], ST_NONFINITE | ST_BREAKDOWN);
}

// ------------------------------------------------------------------ solve

// x (+)= S Ahat^{-1} S rhs for one sample with the tile-layout factor fs
// (all threads of the workgroup call it).  rs == NULL means the constant
// rhs_const.  Arithmetic in Tac (FP64 for the FP64 factor, FP32 otherwise).
// With a single-wave workgroup the LDS atomics below execute in a fixed order.
template <typename Tst, int M, int TR, int NT>
__device__ inline void solve_tile_pass(const double *__restrict__ scs, const double *__restrict__ bs,
                                       const Tst *__restrict__ fs, const double *__restrict__ rs,
                                       double rhs_const, double *__restrict__ xs, int accumulate,
                                       double *__restrict__ zs)
{
    using Tac = typename store_traits<Tst>::acc;
    constexpr int Tn = M / TR, T = Tn * (Tn + 1) / 2, E = TR * TR;
    constexpr int m = M - 1;
    __shared__ Tac g[M], acc[M], xc[M];
    const int t = threadIdx.x;
    const bool active = t < T;
    int I = 0, J = 0;
    if (active) tile_of(t, I, J);
    const int i0 = I * TR, j0 = J * TR;

    auto matvec = [&](int j) {
        // acc[i] += sum_l F_j[i][l] g[l], F_j = stored -C_j^{-1} (symmetric)
        if (!active) return;
        const Tst *fb = fs + (size_t)j * T * E;
        Tac e[TR][TR];
#pragma unroll
        for (int r = 0; r < TR; ++r)
#pragma unroll
            for (int c = 0; c < TR; ++c) e[r][c] = store_traits<Tst>::load(fb[(r * TR + c) * T + t]);
        Tac gr[TR], gc[TR];
#pragma unroll
        for (int r = 0; r < TR; ++r) gr[r] = g[i0 + r];
#pragma unroll
        for (int c = 0; c < TR; ++c) gc[c] = g[j0 + c];
#pragma unroll
        for (int r = 0; r < TR; ++r) {
            Tac sum = 0;
#pragma unroll
            for (int c = 0; c < TR; ++c) sum = fma(e[r][c], gc[c], sum);
            atomicAdd(&acc[i0 + r], sum);
        }
        if (I != J) {
#pragma unroll
            for (int c = 0; c < TR; ++c) {
                Tac sum = 0;
#pragma unroll
                for (int r = 0; r < TR; ++r) sum = fma(e[r][c], gr[r], sum);
                atomicAdd(&acc[j0 + c], sum);
            }
        }
    };

    // forward: z_j = C_j^{-1} (s_j r_j - beta_j z_{j-1}) = -F_j g_j
    for (int i = t; i < M; i += NT) xc[i] = 0;
    __syncthreads();
    for (int j = 0; j < m; ++j) {
        for (int i = t; i < M; i += NT) {
            const double rv = rs ? rs[j * M + i] : (i < m ? rhs_const : 0.0);
            g[i] = (Tac)(scs[j * M + i] * rv) - (Tac)bs[j * M + i] * xc[i];
            acc[i] = 0;
        }
        __syncthreads();
        matvec(j);
        __syncthreads();
        for (int i = t; i < M; i += NT) {
            const Tac z = -acc[i];
            xc[i] = z;
            zs[j * M + i] = (double)z;
        }
        __syncthreads();
    }
    // back: x_{m-1} = z_{m-1}; x_j = z_j - C_j^{-1} beta_{j+1} x_{j+1} = z_j + F_j (beta x)
    for (int i = t; i < M; i += NT) {
        const double d = scs[(m - 1) * M + i] * (double)xc[i];
        xs[(m - 1) * M + i] = accumulate ? xs[(m - 1) * M + i] + d : d;
    }
    for (int j = m - 2; j >= 0; --j) {
        for (int i = t; i < M; i += NT) {
            g[i] = (Tac)bs[(j + 1) * M + i] * xc[i];
            acc[i] = (Tac)zs[j * M + i];
        }
        __syncthreads();
        matvec(j);
        __syncthreads();
        for (int i = t; i < M; i += NT) {
            const Tac xv = acc[i];
            xc[i] = xv;
            const double d = scs[j * M + i] * (double)xv;
            xs[j * M + i] = accumulate ? xs[j * M + i] + d : d;
        }
        __syncthreads();
    }
}


// Algorithm 2.1 for one sample per workgroup (tile-layout factor): x0, then
// {r = b - A x (FP64); stop test; x += solve(r)}; `direct`: residual only.
template <typename Tst, int M, int TR, int NT>
__global__ __launch_bounds__(NT) void k_ir_tile(
    int n, double fconst, const double *__restrict__ a, const double *__restrict__ sc,
    const double *__restrict__ beta, const Tst *__restrict__ factor, double *__restrict__ x,
    double *__restrict__ r, double *__restrict__ zbuf, double eps, int imax, int direct,
    const int *__restrict__ idx, const int *__restrict__ count, int64_t slot_base,
    uint32_t *__restrict__ state, double *__restrict__ relres, double *__restrict__ q,
    int32_t *__restrict__ iters, int disc)
{
    constexpr int Tn = M / TR, T = Tn * (Tn + 1) / 2, E = TR * TR, m = M - 1;
    __shared__ double red[NT];
    const int b = blockIdx.x;
    if (count && b >= *count) return;
    const int s = idx ? idx[b] : b;
    const size_t vo = (size_t)s * m * M;
    const double *scs = sc + vo, *bs = beta + vo;
    const Tst *fs = factor + (size_t)(slot_base + b) * m * T * E;
    double *xs = x + vo, *rsb = r + vo, *zs = zbuf + vo;
    const double *as = a + (size_t)s * (n + 1) * (n + 1);
    const double h = 1.0 / n;
    solve_tile_pass<Tst, M, TR, NT>(scs, bs, fs, nullptr, h * h * fconst, xs, 0, zs);
    uint32_t st = state[s] & ~(uint32_t)ST_DONE;
    double prev = INFINITY, rel = INFINITY, sx = 0.0;
    int trip = 0;
    for (;;) {
        __syncthreads();
        const resid_out o = residual_pass<NT>(n, fconst, as, xs, rsb, red, disc);
        rel = sqrt(o.rr) / sqrt(o.bb);
        sx = o.sx;
        st = ir_decide(st, rel, prev, sx, eps, trip, imax, direct);
        if (st & ST_DONE) break;
        prev = rel;
        __syncthreads();
        solve_tile_pass<Tst, M, TR, NT>(scs, bs, fs, rsb, 0.0, xs, 1, zs);
        ++trip;
    }
    if (threadIdx.x == 0) {
        state[s] = st;
        relres[s] = rel;
        q[s] = h * h * sx;
        if (iters) iters[s] = trip;
    }
}

// ------------------------------------------------------------------ residual


// dQ/dZ at every node for the adjoint gradient: with u and lambda the
// (padded) primal and adjoint solutions (0 on the boundary),
//   gz_e = -sum_{edges f} (lambda_P - lambda_Q)(u_P - u_Q) d w_f / d Z_e,
// Z_e = log a_e, over the edges f = (P, Q) whose coefficient w_f depends on
// a_e.  disc 0: the four edges at e, d w_f / d Z_e = 2 a_o^2 a_e / (a_e + a_o)^2
// (a_o the other end); disc 1: the four edges at e (weight 2/6) and the four
// whose adjacent triangles have e as third vertex (weight 1/6),
// d w_f / d Z_e = weight * a_e.  One thread per node.
__global__ void k_adjoint_gz(int n, int S, const double *__restrict__ a, const double *__restrict__ u,
                             const double *__restrict__ lam, double *__restrict__ gz, int disc)
{
    const int m = n - 1, M = n, np = n + 1;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)S * np * np) return;
    const int s = (int)(g / (np * np));
    const int p = (int)(g % (np * np));
    const int ix = p % np, iy = p / np;
    const double *as = a + (size_t)s * np * np;
    const double *us = u + (size_t)s * m * M, *ls = lam + (size_t)s * m * M;
    auto val = [&](const double *v, int jx, int jy) {
        return (jx >= 1 && jx <= m && jy >= 1 && jy <= m) ? v[(jy - 1) * M + (jx - 1)] : 0.0;
    };
    auto inside = [&](int jx, int jy) { return jx >= 0 && jx <= n && jy >= 0 && jy <= n; };
    // (lambda_P - lambda_Q)(u_P - u_Q) of the edge (px, py) - (qx, qy)
    auto edge = [&](int px, int py, int qx, int qy) {
        if (!inside(px, py) || !inside(qx, qy)) return 0.0;
        return (val(ls, px, py) - val(ls, qx, qy)) * (val(us, px, py) - val(us, qx, qy));
    };
    const double ae = as[p];
    double acc = 0.0;
    if (!disc) {
        const double ue = val(us, ix, iy), le = val(ls, ix, iy);
        const int dx[4] = {1, -1, 0, 0}, dy[4] = {0, 0, 1, -1};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int jx = ix + dx[k], jy = iy + dy[k];
            if (!inside(jx, jy)) continue;
            const double ao = as[jy * np + jx];
            const double du = ue - val(us, jx, jy), dl = le - val(ls, jx, jy);
            const double den = ae + ao;
            acc -= dl * du * 2.0 * ao * ao * ae / (den * den);
        }
    } else {
        // edges with e as an end node
        double s2 = edge(ix, iy, ix + 1, iy) + edge(ix - 1, iy, ix, iy) + edge(ix, iy, ix, iy + 1) +
                    edge(ix, iy - 1, ix, iy);
        // edges whose triangles have e as third vertex: e north of the right
        // node or south of the left node of an x-edge; east of the top node or
        // west of the bottom node of a y-edge
        double s1 = edge(ix - 1, iy - 1, ix, iy - 1) + edge(ix, iy + 1, ix + 1, iy + 1) +
                    edge(ix - 1, iy - 1, ix - 1, iy) + edge(ix + 1, iy, ix + 1, iy + 1);
        acc = -ae * (2.0 * s2 + s1) / 6.0;
    }
    gz[g] = acc;
}

// Copy the padded solution to the caller's unpadded [S][(n-1)^2] layout.
__global__ void k_unpad(int n, int S, const double *__restrict__ x, double *__restrict__ u)
{
    const int m = n - 1, M = n;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)S * m * m) return;
    const int s = (int)(g / (m * m));
    const int P = (int)(g % (m * m));
    u[(size_t)s * m * m + P] = x[(size_t)s * m * M + (P / m) * M + P % m];
}

// Scatter per-sample results of a compact subset back (promotion).
__global__ void k_init_state(int S, uint32_t *state, double *relres)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    state[s] = 0;
    relres[s] = INFINITY;
}

// Reset the refinement state of the samples in idx (for a promoted re-solve).
__global__ void k_reset_subset(int P, const int *__restrict__ idx, const int *__restrict__ count,
                               uint32_t *state, double *relres)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P || (count && p >= *count)) return;
    const int s = idx[p];
    state[s] = ST_PROMOTED;
    relres[s] = INFINITY;
}

// Zero n ints (a kernel rather than a memset node, so captured graphs replay it).
__global__ void k_zero_int(int *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Collect samples that need promotion (not converged) into idx; count in *cnt.
__global__ void k_collect(int S, const uint32_t *__restrict__ state, int *__restrict__ idx,
                          int *__restrict__ cnt)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    if (!(state[s] & ST_CONVERGED)) {
        const int p = atomicAdd(cnt, 1);
        idx[p] = s;
    }
}

// ------------------------------------------------------------------ pairing and level sums

// Y = Qf - Qc (Qc may be NULL), combined status, and the FP64 level sums
// [sum Y, sum Y^2, sum Qf, sum Qc, n_promoted, n_noconv, sum iters] in a fixed
// order (per-thread strided partial sums, then a tree).
__global__ __launch_bounds__(1024) void k_pair_sums(int S, const double *__restrict__ qf,
                                                    const double *__restrict__ qc,
                                                    const uint32_t *__restrict__ stf,
                                                    const uint32_t *__restrict__ stc,
                                                    const int32_t *__restrict__ itf,
                                                    const int32_t *__restrict__ itc,
                                                    double *__restrict__ y,
                                                    uint8_t *__restrict__ status,
                                                    double *__restrict__ sums)
{
    __shared__ double part[16][8];
    double sy = 0, sy2 = 0, sf = 0, scc = 0, npro = 0, nnc = 0, sit = 0, sitc = 0;
    for (int s = threadIdx.x; s < S; s += 1024) {
        const double f = qf[s], c = qc ? qc[s] : 0.0;
        const double yv = f - c;
        if (y) y[s] = yv;
        sy += yv;
        sy2 += yv * yv;
        sf += f;
        scc += c;
        const uint32_t a = stf[s], bcs = stc ? stc[s] : (uint32_t)ST_CONVERGED;
        if (status) status[s] = (uint8_t)((a & 15u) | ((bcs & 15u) << 4));
        npro += ((a | bcs) & ST_PROMOTED) ? 1.0 : 0.0;
        nnc += (!(a & ST_CONVERGED) || !(bcs & ST_CONVERGED)) ? 1.0 : 0.0;
        sit += itf ? (double)itf[s] : 0.0;
        sitc += itc ? (double)itc[s] : 0.0;
    }
    // fixed-order reductions: a butterfly inside each wave, then the 16 wave
    // partials in wave order (deterministic)
    double v[8] = {sy, sy2, sf, scc, npro, nnc, sit, sitc};
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) part[wv][q] = v[q];
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        double r = 0.0;
        for (int w = 0; w < 16; ++w) r += part[w][threadIdx.x];
        sums[threadIdx.x] = r;
    }
}

}  // namespace mlmc

// ------------------------------------------------------------------ launchers

using namespace mlmc;

namespace {
template <typename Tst, int M, int TR>
constexpr int nthreads()
{
    constexpr int Tn = M / TR, T = Tn * (Tn + 1) / 2;
    return ((T + 63) / 64) * 64;
}

template <int M>
struct tile_cfg;
template <> struct tile_cfg<4> { static constexpr int TR = 2; };
template <> struct tile_cfg<8> { static constexpr int TR = 2; };
template <> struct tile_cfg<16> { static constexpr int TR = 2; };
template <> struct tile_cfg<32> { static constexpr int TR = 4; };

template <typename Tst, int M>
hipError_t launch_factor_t(int nblocks, const double *beta, const double *gam, void *factor,
                           const int *idx, const int *count, int64_t slot_base, uint32_t *state,
                           hipStream_t st)
{
    constexpr int TR = tile_cfg<M>::TR, NT = nthreads<Tst, M, TR>();
    hipLaunchKernelGGL((k_factor<Tst, M, TR, NT>), dim3(nblocks), dim3(NT), 0, st, nblocks, beta,
                       gam, (Tst *)factor, idx, count, slot_base, state);
    return hipGetLastError();
}

template <typename Tst, int M>
hipError_t launch_ir_t(const ir_args &g, hipStream_t st)
{
    constexpr int TR = tile_cfg<M>::TR, NT = nthreads<Tst, M, TR>();
    hipLaunchKernelGGL((k_ir_tile<Tst, M, TR, NT>), dim3(g.nblocks), dim3(NT), 0, st, g.n, g.fconst,
                       g.a, g.sc, g.beta, (const Tst *)g.factor, g.x, g.r, g.z, g.eps, g.imax,
                       g.direct, g.idx, g.count, g.slot_base, g.state, g.relres, g.q, g.iters, g.disc);
    return hipGetLastError();
}

template <typename Tst>
hipError_t launch_ir_m(const ir_args &g, hipStream_t st)
{
    switch (g.n) {
    case 4: return launch_ir_t<Tst, 4>(g, st);
    case 8: return launch_ir_t<Tst, 8>(g, st);
    case 16: return launch_ir_t<Tst, 16>(g, st);
    case 32: return launch_ir_t<Tst, 32>(g, st);
    }
    return hipErrorInvalidValue;
}


// FP8 storage: the grids below 16 only (the tile kernels)
hipError_t launch_factor_fp8(int M, int nb, const double *beta, const double *gam, void *factor,
                             const int *idx, const int *count, int64_t slot_base, uint32_t *state,
                             hipStream_t st)
{
    switch (M) {
    case 4: return launch_factor_t<fp8e4m3, 4>(nb, beta, gam, factor, idx, count, slot_base, state, st);
    case 8: return launch_factor_t<fp8e4m3, 8>(nb, beta, gam, factor, idx, count, slot_base, state, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_ir_fp8(const ir_args &g, hipStream_t st)
{
    switch (g.n) {
    case 4: return launch_ir_t<fp8e4m3, 4>(g, st);
    case 8: return launch_ir_t<fp8e4m3, 8>(g, st);
    }
    return hipErrorInvalidValue;
}

template <typename Tst>
hipError_t launch_factor_m(int M, int nb, const double *beta, const double *gam, void *factor,
                           const int *idx, const int *count, int64_t slot_base, uint32_t *state,
                           hipStream_t st)
{
    switch (M) {
    case 4: return launch_factor_t<Tst, 4>(nb, beta, gam, factor, idx, count, slot_base, state, st);
    case 8: return launch_factor_t<Tst, 8>(nb, beta, gam, factor, idx, count, slot_base, state, st);
    case 16: return launch_factor_t<Tst, 16>(nb, beta, gam, factor, idx, count, slot_base, state, st);
    case 32: return launch_factor_t<Tst, 32>(nb, beta, gam, factor, idx, count, slot_base, state, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

namespace mlmc {

size_t factor_entries_per_sample(int dtype, int n)
{
    const int M = n;
    if (use_blk(dtype, n)) {
        const int NB = M / 16;
        return (size_t)(n - 1) * (NB * (NB + 1) / 2) * 256;
    }
    int TR = M <= 16 ? 2 : (M <= 32 ? 4 : 8);
    const int Tn = M / TR, T = Tn * (Tn + 1) / 2;
    return (size_t)(n - 1) * T * TR * TR;
}

hipError_t launch_fill_xi(uint64_t seed, int level, int64_t first, int64_t n, int K, double *xi,
                          hipStream_t st)
{
    const int64_t tot = n * ((K + 1) / 2);
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_xi, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, seed, level,
                       first, n, K, xi);
    return hipGetLastError();
}

hipError_t launch_field(int S, int K, int P, const double *xi, const double *phit, double *a,
                        hipStream_t st)
{
    return launch_field_mfma(S, K, P, xi, phit, a, st);
}

hipError_t launch_grad_gemm(int S, int K, int P, const double *gz, const double *phit,
                            const double *gq, double *grad, hipStream_t st)
{
    dim3 grid((K + 63) / 64, (S + 63) / 64);
    hipLaunchKernelGGL((k_gemm64<true, 1>), grid, dim3(256), 0, st, S, K, P, gz, P, phit, P, grad, K,
                       gq);
    return hipGetLastError();
}

hipError_t launch_coeffs(int n, int S, const double *a, double *sc, double *gam, double *beta, int disc,
                         hipStream_t st)
{
    if (S == 0) return hipSuccess;
    const dim3 grid((unsigned)S, (unsigned)(((n - 1) * n + 255) / 256));
    hipLaunchKernelGGL(k_scale, grid, dim3(256), 0, st, n, a, sc, disc);
    hipLaunchKernelGGL(k_coeffs, grid, dim3(256), 0, st, n, a, sc, gam, beta, disc);
    return hipGetLastError();
}

hipError_t launch_factor(int dtype, int n, int nblocks, const double *a, double *sc, double *beta,
                         const double *gam, void *factor, const int *idx, const int *count,
                         int64_t slot_base, uint32_t *state, double frhs, double *fz, double *x0,
                         int disc, int variant, hipStream_t st)
{
    if (nblocks == 0) return hipSuccess;
    if (fz && !factor_fuses_forward(dtype, n)) return hipErrorInvalidValue;
    if (x0 && (!fz || idx || !factor_solves_initial(dtype, n))) return hipErrorInvalidValue;
    if (use_blk(dtype, n))
        return launch_factor_blk(dtype, n, nblocks, a, sc, beta, gam, factor, idx, count, slot_base, state,
                                 frhs, fz, x0, disc, variant, st);
    switch (dtype) {
    case 0: return launch_factor_m<double>(n, nblocks, beta, gam, factor, idx, count, slot_base, state, st);
    case 1: return launch_factor_m<float>(n, nblocks, beta, gam, factor, idx, count, slot_base, state, st);
    case 2: return launch_factor_m<__hip_bfloat16>(n, nblocks, beta, gam, factor, idx, count, slot_base, state, st);
    case 3: return launch_factor_m<__half>(n, nblocks, beta, gam, factor, idx, count, slot_base, state, st);
    case 4: return launch_factor_fp8(n, nblocks, beta, gam, factor, idx, count, slot_base, state, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_ir(int dtype, const ir_args &g, hipStream_t st)
{
    if (g.nblocks == 0) return hipSuccess;
    if (use_blk(dtype, g.n)) return launch_ir_blk(dtype, g, st);
    switch (dtype) {
    case 0: return launch_ir_m<double>(g, st);
    case 1: return launch_ir_m<float>(g, st);
    case 2: return launch_ir_m<__hip_bfloat16>(g, st);
    case 3: return launch_ir_m<__half>(g, st);
    case 4: return launch_ir_fp8(g, st);
    }
    return hipErrorInvalidValue;
}


hipError_t launch_adjoint_gz(int n, int S, const double *a, const double *u, const double *lam,
                             double *gz, int disc, hipStream_t st)
{
    const int64_t tot = (int64_t)S * (n + 1) * (n + 1);
    hipLaunchKernelGGL(k_adjoint_gz, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, S, a, u,
                       lam, gz, disc);
    return hipGetLastError();
}

hipError_t launch_unpad(int n, int S, const double *x, double *u, hipStream_t st)
{
    const int64_t N = (int64_t)S * (n - 1) * (n - 1);
    hipLaunchKernelGGL(k_unpad, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, n, S, x, u);
    return hipGetLastError();
}

hipError_t launch_init_state(int S, uint32_t *state, double *relres, hipStream_t st)
{
    hipLaunchKernelGGL(k_init_state, dim3((S + 255) / 256), dim3(256), 0, st, S, state, relres);
    return hipGetLastError();
}

hipError_t launch_reset_subset(int P, const int *idx, const int *count, uint32_t *state,
                               double *relres, hipStream_t st)
{
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reset_subset, dim3((P + 255) / 256), dim3(256), 0, st, P, idx, count, state,
                       relres);
    return hipGetLastError();
}

hipError_t launch_zero_int(int *p, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_int, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_collect(int S, const uint32_t *state, int *idx, int *cnt, hipStream_t st)
{
    hipLaunchKernelGGL(k_collect, dim3((S + 255) / 256), dim3(256), 0, st, S, state, idx, cnt);
    return hipGetLastError();
}

hipError_t launch_pair_sums(int S, const double *qf, const double *qc, const uint32_t *stf,
                            const uint32_t *stc, const int32_t *itf, const int32_t *itc, double *y,
                            uint8_t *status, double *sums, hipStream_t st)
{
    hipLaunchKernelGGL(k_pair_sums, dim3(1), dim3(1024), 0, st, S, qf, qc, stf, stc, itf, itc, y,
                       status, sums);
    return hipGetLastError();
}

}  // namespace mlmc
