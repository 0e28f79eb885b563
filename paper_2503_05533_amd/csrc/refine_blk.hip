// Algorithm 2.1 with the block-layout factor of factor_mfma.hip: the
// refinement kernels for M >= 32 (one sample per workgroup, the triangular
// passes over the stored blocks on the MFMA layout, the FP64 residual
// matrix-free) and the one-row-per-lane kernel for the n = 16 grid.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "blk_common.h"
#include "dtypes.h"
#include "ir_common.h"
#include "kernels.h"

namespace mlmc {

// Waves per SIMD the n = 16 refinement kernel is held to: four with FP32
// arithmetic (128 registers), three in FP64, whose z, x and two factor rows
// in flight take 124 registers by themselves.
template <typename Tst> constexpr int ir_rows_waves() { return sizeof(typename store_traits<Tst>::acc) == 4 ? 4 : 3; }

// Algorithm 2.1 on the n = 16 grid with the factor of k_factor_rows16: 16
// lanes per sample (lane i owns the unknowns (i, j) of every grid row j and
// row i of every stored F_j, the entries its factorisation lane stored), 16
// samples per workgroup, no LDS.  The solution x and the forward-sweep
// result z stay in registers; F_j is applied row by row with the vector it
// multiplies broadcast along the 16-lane row.  The FP64 residual takes its
// east and west neighbours by DPP row shifts and forms each face coefficient
// once (the east face is the west face of the next lane, the south face the
// north face of the row before); the per-sample sums are fixed-order DPP
// reductions.  A correction recomputes the residual row by row inside its
// forward sweep instead of storing it.  The arguments and outputs of
// k_ir_blk, with the sample count S in place of n and no residual buffer;
// every factor type.  D: the edge rule, as in k_factor_rows16.
template <typename Tst, bool STRIDE, int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ir_rows_waves<Tst>()))) void k_ir_rows16(
    int S, double fconst, const double *__restrict__ a, const double *__restrict__ sc,
    const double *__restrict__ beta, const Tst *__restrict__ factor, double *__restrict__ x,
    const double *__restrict__ zbuf, double eps, int imax, int direct, const int *__restrict__ idx,
    const int *__restrict__ count, int64_t slot_base, uint32_t *__restrict__ state,
    double *__restrict__ relres, double *__restrict__ q, int32_t *__restrict__ iters, int fwd_done)
{
    using Tac = typename store_traits<Tst>::acc;
    constexpr int M = 16, m = M - 1, NP = M + 1, disc = D;
    const int i = threadIdx.x & 15;
    for (int b = blockIdx.x * 16 + (threadIdx.x >> 4);; b += gridDim.x * 16) {
        // whole 16-lane rows leave together, so no DPP source lane of a live row is idle
        if (b >= S || (count && b >= *count)) return;
        const int s = idx ? idx[b] : b;
        const size_t vo = (size_t)s * m * M + i;
        const double *scs = sc + vo, *bs = beta + vo;
        double *xs = x + vo;
        const Tst *fs = factor + (size_t)(slot_base + b) * m * 256 + i * 4;  // row i: 4 entries at g * 64
        const double *ac = a + (size_t)s * NP * NP + (i + 1);                // node column i + 1
        const double h = 1.0 / M, bval = h * h * fconst;
        const bool in = i < m;  // lane m is the identity pad

        // Loads in the sweeps and residual passes take an offset the compiler cannot
        // see through (opaque): without it, the addresses of all 60 factor loads and
        // the loop-invariant coefficient loads of every row are hoisted out of the
        // refinement loop and held in registers.
        auto opaque = [](int v) {
            asm volatile("" : "+v"(v));
            return v;
        };
        auto ldq = [&](int j, quad<Tst> (&dst)[4]) {
            const Tst *fb = fs + opaque(j * 256);
#pragma unroll
            for (int g = 0; g < 4; ++g) dst[g] = *(const quad<Tst> *)(fb + g * 64);
        };
        auto row_of = [&](const quad<Tst> (&src)[4], Tac (&f)[16]) {
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
                for (int c = 0; c < 4; ++c) f[drow<Tac>(g, c)] = store_traits<Tst>::load(src[g].v[c]);
        };

        Tac z[m];      // z_j, entry i
        double xv[m];  // x_j, entry i
        // Every step uses operands loaded one step earlier and first requests the
        // next step's (loads complete in order, so a wait for a late request would
        // also wait for the prefetch in front of it).
        quad<Tst> fq[2][4];
        double scp[2], bp[2];

        // Forward sweep z_j = -F_j (s_j r_j - beta_j z_{j-1}); rj(j) gives r_j and
        // runs before the step's arithmetic (it may issue loads of its own).
        auto forward = [&](auto &&rj) {
            const int o = opaque(0);
            const double *scq = scs + o, *bq = bs + o;
            ldq(0, fq[0]);
            scp[0] = scq[0];
            bp[0] = 0.0;
#pragma unroll
            for (int j = 0; j < m; ++j) {
                if (j + 1 < m) {
                    ldq(j + 1, fq[(j + 1) & 1]);
                    scp[(j + 1) & 1] = scq[(j + 1) * M];
                    bp[(j + 1) & 1] = bq[(j + 1) * M];
                }
                const double r = rj(j);
                const Tac gv0 = (Tac)(scp[j & 1] * r);
                const Tac gv = j > 0 ? gv0 - (Tac)bp[j & 1] * z[j - 1] : gv0;
                Tac f[16];
                row_of(fq[j & 1], f);
                z[j] = -dot16_colbcast(f, gv, (Tac)0);
                __builtin_amdgcn_sched_barrier(0);  // one grid row at a time: bounds the registers in flight
            }
        };
        // back: x_{m-1} = s z_{m-1}; x_j = s_j (z_j + F_j (beta_{j+1} x~_{j+1})),
        // x~ the unscaled iterate; accumulate adds to x
        auto back = [&](bool accumulate) {
            const int o = opaque(0);
            const double *scq = scs + o, *bq = bs + o;
            ldq(m - 2, fq[(m - 2) & 1]);
            scp[(m - 2) & 1] = scq[(m - 2) * M];
            bp[(m - 2) & 1] = bq[(m - 1) * M];
            Tac xc = z[m - 1];
            {
                const double d = scq[(m - 1) * M] * (double)xc;
                xv[m - 1] = accumulate ? xv[m - 1] + d : d;
                xs[(m - 1) * M] = xv[m - 1];
            }
#pragma unroll
            for (int j = m - 2; j >= 0; --j) {
                if (j > 0) {
                    ldq(j - 1, fq[(j - 1) & 1]);
                    scp[(j - 1) & 1] = scq[(j - 1) * M];
                    bp[(j - 1) & 1] = bq[j * M];
                }
                const Tac gv = (Tac)bp[j & 1] * xc;
                Tac f[16];
                row_of(fq[j & 1], f);
                xc = z[j] + dot16_colbcast(f, gv, (Tac)0);
                const double d = scp[j & 1] * (double)xc;
                xv[j] = accumulate ? xv[j] + d : d;
                xs[j * M] = xv[j];
                __builtin_amdgcn_sched_barrier(0);
            }
        };
        // Residual r = b - A x row by row (entry i; 0 on the pad): the object keeps
        // the carried face and the prefetched node values of the next row.
        struct resid_rows {
            const double *ac;
            double c, aS, cN, w;  // centre of row j, its south face, prefetched north and west nodes
            double wS;            // the node south of the west node (P1 faces)
        };
        auto resid_start = [&]() {
            resid_rows R;
            R.ac = ac + opaque(0);  // face coefficients are formed anew in every pass
            R.c = R.ac[NP];
            R.aS = disc ? face_y(1, R.ac[0], R.c, dpp_f64<0x101>(R.c), R.ac[-1]) : hmean2(R.c, R.ac[0]);
            R.cN = R.ac[2 * NP];
            R.w = R.ac[NP - 1];
            R.wS = R.ac[-1];
            return R;
        };
        auto resid_row = [&](resid_rows &R, int j) {
            const double cN = R.cN, w = R.w;
            if (j + 1 < m) {
                R.cN = R.ac[(j + 3) * NP];
                R.w = R.ac[(j + 2) * NP - 1];
            }
            double aw, an;
            if (disc) {
                aw = face_x(1, w, R.c, cN, R.wS);
                an = face_y(1, R.c, cN, dpp_f64<0x101>(cN), w);
            } else {
                aw = hmean2(R.c, w);
                an = hmean2(R.c, cN);
            }
            R.wS = w;
            const double ae = dpp_f64<0x101>(aw);  // the next lane's west face
            const double xw = dpp_f64<0x111>(xv[j]), xe = dpp_f64<0x101>(xv[j]);
            double ax = (aw + ae + R.aS + an) * xv[j];
            ax -= i > 0 ? aw * xw : 0.0;
            ax -= i + 1 < m ? ae * xe : 0.0;
            if (j > 0) ax -= R.aS * xv[j - 1];
            if (j + 1 < m) ax -= an * xv[j + 1];
            R.c = cN;
            R.aS = an;
            return in ? bval - ax : 0.0;
        };

        // initial solve (fwd_done: the factorisation ran it and x holds x0)
        if (fwd_done) {
#pragma unroll
            for (int j = 0; j < m; ++j) xv[j] = xs[j * M];
        } else {
            forward([&](int) { return in ? bval : 0.0; });
            back(false);
        }

        uint32_t st = state[s] & ~(uint32_t)ST_DONE;
        double prev = INFINITY, rel = INFINITY, sx = 0.0;
        int trip = 0;
        for (;;) {
            double rr = 0.0, bb = 0.0, sxl = 0.0;
            {
                resid_rows R = resid_start();
#pragma unroll
                for (int j = 0; j < m; ++j) {
                    const double rv = resid_row(R, j);
                    rr += rv * rv;
                    bb += in ? bval * bval : 0.0;
                    sxl += in ? xv[j] : 0.0;
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            rr = rowbcast<15>(row16_total(rr));
            bb = rowbcast<15>(row16_total(bb));
            sx = rowbcast<15>(row16_total(sxl));
            rel = sqrt(rr) / sqrt(bb);
            st = ir_decide(st, rel, prev, sx, eps, trip, imax, direct);
            if (st & ST_DONE) break;
            prev = rel;
            {
                resid_rows R = resid_start();
                forward([&](int j) { return resid_row(R, j); });
            }
            back(true);
            ++trip;
        }
        if (i == 0) {
            state[s] = st;
            relres[s] = rel;
            q[s] = h * h * sx;
            if (iters) iters[s] = trip;
        }
        if constexpr (!STRIDE) return;
    }
}

// ------------------------------------------------------------------ block solve

// The solve with the twisted factor (blk_common.h): with k = (m - 1) / 2,
// F_j = -C_j^{-1} (j < k), -D_j^{-1} (j > k) and -E_k^{-1}, the forward
// sweeps of both chains and the middle,
//   z_j = -F_j (g_j - beta_j z_{j-1})          j = 0 .. k-1
//   w_j = -F_j (g_j - beta_{j+1} w_{j+1})      j = m-1 .. k+1
//   x_k = -F_k (g_k - beta_k z_{k-1} - beta_{k+1} w_{k+1}),
// then the back sweeps outwards from the middle,
//   x_j = z_j + F_j beta_{j+1} x_{j+1}         j = k-1 .. 0
//   x_j = w_j + F_j beta_j x_{j-1}             j = k+1 .. m-1,
// one block after the other (2m - 1 steps, as the one-sided solve).  zs
// keeps z, x_k and w at their block rows (the factorisation's forward sweep
// leaves the same).  Step s visits block row tw_row(s): s < 2k the two
// forward chains, s = 2k the middle, s > 2k the two back chains.
template <int m> __device__ __forceinline__ int tw_row(int s)
{
    constexpr int k = (m - 1) / 2;
    // independent selects (no branch chain)
    int r = k + 1 + (s - m - k);
    r = s < m + k ? k - 1 - (s - m) : r;
    r = s == 2 * k ? k : r;
    r = s < 2 * k ? m - 1 + k - s : r;
    r = s < k ? s : r;
    return r;
}
template <typename Tst, int M, int DEPTH, typename Tac, typename Buf, typename LoadF, typename ApplyF,
          typename GatherF>
__device__ __forceinline__ void solve_twisted(const double *__restrict__ scs, const double *__restrict__ bs,
                                              const double *__restrict__ rs, double rhs_const,
                                              double *__restrict__ xs, int accumulate, double *__restrict__ zs,
                                              bool fwd_done, bool own, int t, Tac *g, Buf &bA, Buf &bB, Buf &bC,
                                              LoadF &load, ApplyF &apply, GatherF &gather)
{
    constexpr int m = M - 1, k = (m - 1) / 2, NS = 2 * m - 1, NF = 2 * k;
    const double rc = t < m ? rhs_const : 0.0;
    // Steps [s0, s1) with the rotation of solve_blk_pass: step s applies its
    // block while the block of step s + DEPTH (clamped to s1 - 1; a redundant
    // load is harmless) streams in; upd(s) is the owner threads' update.
    auto run = [&](int s0, int s1, auto &&upd) {
        auto step = [&](int s, Buf &use, Buf &fill) {
            if constexpr (DEPTH > 0) {
                load(tw_row<m>(s + DEPTH < s1 ? s + DEPTH : s1 - 1), fill);
                apply(use);
            } else {
                load(tw_row<m>(s), bA);
                apply(bA);
            }
            __syncthreads();
            if (own) upd(s);
            __syncthreads();
        };
        if constexpr (DEPTH >= 1) load(tw_row<m>(s0), bA);
        if constexpr (DEPTH == 2) load(tw_row<m>(s0 + 1 < s1 ? s0 + 1 : s0), bB);
        __syncthreads();
        int s = s0;
        if constexpr (DEPTH == 2) {
            for (; s + 3 <= s1; s += 3) {
                step(s, bA, bC);
                step(s + 1, bB, bA);
                step(s + 2, bC, bB);
            }
            if (s < s1) step(s++, bA, bC);
            if (s < s1) step(s++, bB, bA);
        } else if constexpr (DEPTH == 1) {
            for (; s + 2 <= s1; s += 2) {
                step(s, bA, bB);
                step(s + 1, bB, bA);
            }
            if (s < s1) step(s++, bA, bB);
        } else {
            for (; s < s1; ++s) step(s, bA, bA);
        }
    };
    // The inputs of an update are read one step ahead and combined only when
    // used (an operation on a value in flight would wait for it, and with it
    // for the block loads issued before).
    double l_sc = 0.0, l_r = 0.0, l_b = 0.0, l_z = 0.0, l_x = 0.0;
    double b_k = 0.0, b_k1 = 0.0;
    if (own) {
        b_k = bs[k * M + t];
        b_k1 = bs[(k + 1) * M + t];
    }
    Tac sav = 0;  // z_{k-1}, then x_k
    // inputs of back step q: z (or w), scaling and old x of its row, and the
    // beta that couples the next back step's row to it
    auto fetch_b = [&](int q) {
        q = q < NS ? q : NS - 1;
        const int j = tw_row<m>(q);
        const int ib0 = q + 1 < m + k ? j : j + 1;
        l_z = zs[j * M + t];
        l_sc = scs[j * M + t];
        l_x = accumulate ? xs[j * M + t] : 0.0;
        l_b = bs[(ib0 < m ? ib0 : m - 1) * M + t];
    };
    if (!fwd_done) {
        // inputs of forward step q's right-hand side: the scaled rhs of its
        // row and the beta coupling it to the step before (beta_q on the top
        // chain, beta_{j+1} on the bottom one, beta_{k+1} at the middle; none
        // at the first bottom step)
        auto fetch_f = [&](int q) {
            q = q < NF ? q : NF;
            const int j = tw_row<m>(q);
            l_sc = scs[j * M + t];
            l_r = rs ? rs[j * M + t] : rc;
            l_b = bs[(q <= k ? j : j + 1) * M + t];
        };
        if (own) {
            g[t] = (Tac)(scs[t] * (rs ? rs[t] : rc));
            fetch_f(1);
        }
        run(0, NF, [&](int s) {
            const Tac v = -gather(t);
            zs[tw_row<m>(s) * M + t] = (double)v;
            sav = s == k - 1 ? v : sav;
            // g of step s + 1; the middle also takes -beta_k z_{k-1}
            const Tac cb = s + 1 == k ? (Tac)0 : -(Tac)l_b;
            const Tac cm = s + 1 == NF ? -(Tac)b_k * sav : (Tac)0;
            g[t] = (Tac)(l_sc * l_r) + cb * v + cm;
            fetch_f(s + 2);
        });
        // the middle block row
        double m_sc = 0.0, m_x = 0.0;
        if (own) {
            m_sc = scs[k * M + t];
            m_x = accumulate ? xs[k * M + t] : 0.0;
        }
        load(k, bA);
        apply(bA);
        __syncthreads();
        if (own) {
            sav = -gather(t);
            zs[k * M + t] = (double)sav;
            xs[k * M + t] = m_x + m_sc * (double)sav;
            g[t] = (Tac)b_k * sav;
            fetch_b(m);
        }
        __syncthreads();
    } else if (own) {
        // the factorisation left z, x_k and w: the back sweeps start at once
        sav = (Tac)zs[k * M + t];
        const double d = scs[k * M + t] * (double)sav;
        xs[k * M + t] = accumulate ? xs[k * M + t] + d : d;
        g[t] = (Tac)b_k * sav;
        fetch_b(m);
    }
    run(m, NS, [&](int s) {
        const Tac v = (Tac)l_z + gather(t);
        const double d = l_sc * (double)v;
        xs[tw_row<m>(s) * M + t] = accumulate ? l_x + d : d;
        // g of step s + 1: beta x of the row before; the first bottom step
        // takes beta_{k+1} x_k
        g[t] = s + 1 == m + k ? (Tac)b_k1 * sav : (Tac)l_b * v;
        fetch_b(s + 1);
    });
}

// x (+)= S Ahat^{-1} S rhs for one sample with the block-layout factor fs
// (all threads of the workgroup call it).  Wave w holds the blocks of its
// row pair; per Schur block it forms its share of F g: row sums of its
// blocks accumulate in registers and are reduced across each 16-lane row by
// DPP, the transposed (column) contributions of off-diagonal blocks are
// reduced across the four lane rows and stored once per block.  Every
// partial has its own LDS slot, so the sum over waves (one thread per vector
// entry) is in a fixed order.  Two barriers per Schur block; the next block's
// factor entries are loaded while the current one is applied.  rs == NULL
// means the constant rhs_const.
template <typename Tst, int M, int G, bool PREF>
__device__ __forceinline__ void solve_blk_pass(const double *__restrict__ scs, const double *__restrict__ bs,
                                      const Tst *__restrict__ fs, const double *__restrict__ rs,
                                      double rhs_const, double *__restrict__ xs, int accumulate,
                                      double *__restrict__ zs, bool fwd_done = false)
{
    using Tac = typename store_traits<Tst>::acc;
    constexpr int NB = M / 16, NBL = NB * (NB + 1) / 2, W = blk_waves<M, G>(), SPW = blk_slots<M, G>();
    constexpr int m = M - 1, NT = 64 * W;
    static_assert(NT >= M, "one vector entry per thread");
    __shared__ Tac g[M];
    __shared__ Tac partR[W][M];     // row sums of the wave's two block rows (other entries 0)
    __shared__ Tac partC[W][2][M];  // column sums of the off-diagonal blocks of each row (others 0)
    const int t = threadIdx.x, l = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int pr = w / G;  // the wave's row pair (pr, NB-1-pr)
    const int lr = l >> 4, lc = l & 15;

    for (int i = l; i < M; i += 64) {
        partR[w][i] = 0;
        partC[w][0][i] = 0;
        partC[w][1][i] = 0;
    }

    // Blocks in flight while one is applied (PREF): two, or one where three
    // rotating buffers would not fit the registers of a 1024-thread workgroup.
    constexpr int DEPTH = !PREF ? 0 : (M >= 256 ? 1 : 2);
    Tst bA[SPW][4], bB[SPW][4], bC[SPW][4];
    auto load = [&](int j, Tst (&dst)[SPW][4]) {
        int wq = w;
        asm volatile("" : "+s"(wq));
        const Tst *fb = fs + (size_t)j * NBL * 256;
#pragma unroll
        for (int q = 0; q < SPW; ++q) {
            int I, J;
            const bool valid = slot_blk<NB, G>(wq, q, I, J);
            if constexpr (G > 1) {
                if (!valid) continue;
            }
            const int bb = I * (I + 1) / 2 + J;
            const quad<Tst> qv = *(const quad<Tst> *)(fb + ((size_t)bb * 64 + l) * 4);
#pragma unroll
            for (int r = 0; r < 4; ++r) dst[q][r] = qv.v[r];
        }
    };
    // this wave's partials of F g for the block held in `cur`
    auto apply = [&](const Tst (&cur)[SPW][4]) {
        int wq = w;
        asm volatile("" : "+s"(wq));
        Tac ra0[4] = {0, 0, 0, 0}, ra1[4] = {0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < SPW; ++q) {
            int I, J;
            const bool valid = slot_blk<NB, G>(wq, q, I, J);
            if constexpr (G > 1) {
                if (!valid) continue;
            }
            Tac f[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) f[r] = store_traits<Tst>::load(cur[q][r]);
            const Tac gj = g[16 * J + lc];
            const bool first = (I == pr);  // wave-uniform: which of the two block rows
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (first)
                    ra0[r] = fma(f[r], gj, ra0[r]);
                else
                    ra1[r] = fma(f[r], gj, ra1[r]);
            }
            if (I != J) {
                Tac c = 0;
#pragma unroll
                for (int r = 0; r < 4; ++r) c = fma(f[r], g[16 * I + drow<Tac>(lr, r)], c);
                c = rows4_total(c);
                if (lr == 0) partC[wq][first ? 0 : 1][16 * J + lc] = c;
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const Tac v0 = row16_total(ra0[r]);
            const Tac v1 = row16_total(ra1[r]);
            if (lc == 15) {
                partR[wq][16 * pr + drow<Tac>(lr, r)] = v0;
                if (NB > 1) partR[wq][16 * (NB - 1 - pr) + drow<Tac>(lr, r)] = v1;
            }
        }
    };
    auto gather = [&](int i) {
        Tac v = 0;
#pragma unroll
        for (int ww = 0; ww < W; ++ww) v += partR[ww][i] + partC[ww][0][i] + partC[ww][1][i];
        return v;
    };

    // Thread t < M owns vector entry t of every block; its inputs of the next
    // block are loaded one block ahead.
    const bool own = t < M;
    if constexpr (twisted<Tac, M>()) {
        solve_twisted<Tst, M, DEPTH>(scs, bs, rs, rhs_const, xs, accumulate, zs, fwd_done, own, t, g, bA, bB, bC,
                                     load, apply, gather);
        return;
    }
    // forward: z_j = -F_j (s_j r_j - beta_j z_{j-1})
    Tac xc = 0;
    double v_sc = 0.0, v_b = 0.0, v_r = 0.0;
    if (fwd_done) {
        // the factorisation ran the forward sweep for this right-hand side
        if (own) xc = (Tac)zs[(m - 1) * M + t];
    } else {
        if (own) {
            const double r0 = rs ? rs[t] : (t < m ? rhs_const : 0.0);
            g[t] = (Tac)(scs[t] * r0);
            if (m > 1) {
                v_sc = scs[M + t];
                v_b = bs[M + t];
                v_r = rs ? rs[M + t] : (t < m ? rhs_const : 0.0);
            }
        }
        // One block of the forward pass: apply block j (in `use`) while block
        // j + DEPTH (clamped; a redundant load of the last block is harmless)
        // streams into `fill`.
        auto fwd = [&](int j, const Tst (&use)[SPW][4], Tst (&fill)[SPW][4]) {
            if constexpr (PREF) {
                load(j + DEPTH < m ? j + DEPTH : m - 1, fill);
                apply(use);
            } else {
                load(j, bA);
                apply(bA);
            }
            __syncthreads();
            if (own) {
                xc = -gather(t);
                zs[j * M + t] = (double)xc;
                g[t] = (Tac)(v_sc * v_r) - (Tac)v_b * xc;
                const int jn = j + 2 < m ? j + 2 : m - 1;
                v_sc = scs[jn * M + t];
                v_b = bs[jn * M + t];
                v_r = rs ? rs[jn * M + t] : (t < m ? rhs_const : 0.0);
            }
            __syncthreads();
        };
        if constexpr (DEPTH >= 1) load(0, bA);
        if constexpr (DEPTH == 2) load(m > 1 ? 1 : 0, bB);
        __syncthreads();
        // The loop bodies are kept free of data-dependent branches so that waits
        // for a block's factor entries do not also wait for the blocks behind it;
        // the buffers rotate by unrolling, never by register copies (a copy would
        // wait for the load in flight).
        {
            int j = 0;
            if constexpr (DEPTH == 2) {
                for (; j + 3 <= m; j += 3) {
                    fwd(j, bA, bC);
                    fwd(j + 1, bB, bA);
                    fwd(j + 2, bC, bB);
                }
                if (j < m) fwd(j++, bA, bC);
                if (j < m) fwd(j++, bB, bA);
            } else if constexpr (DEPTH == 1) {
                for (; j + 2 <= m; j += 2) {
                    fwd(j, bA, bB);
                    fwd(j + 1, bB, bA);
                }
                if (j < m) fwd(j++, bA, bB);
            } else {
                for (; j < m; ++j) fwd(j, bA, bA);
            }
        }
    }
    // back: x_{m-1} = z_{m-1}; x_j = z_j + F_j (beta_{j+1} x_{j+1})
    double v_z = 0.0, v_x = 0.0;
    if (own) {
        const double d = scs[(m - 1) * M + t] * (double)xc;
        xs[(m - 1) * M + t] = accumulate ? xs[(m - 1) * M + t] + d : d;
        if (m >= 2) {
            g[t] = (Tac)bs[(m - 1) * M + t] * xc;
            v_z = zs[(m - 2) * M + t];
            v_sc = scs[(m - 2) * M + t];
            v_x = accumulate ? xs[(m - 2) * M + t] : 0.0;
            v_b = (m >= 3) ? bs[(m - 2) * M + t] : 0.0;
        }
    }
    // One block of the back pass: apply block j while block j - DEPTH (clamped
    // at 0) streams in.
    auto back = [&](int j, const Tst (&use)[SPW][4], Tst (&fill)[SPW][4]) {
        if constexpr (PREF) {
            load(j >= DEPTH ? j - DEPTH : 0, fill);
            apply(use);
        } else {
            load(j, bA);
            apply(bA);
        }
        __syncthreads();
        if (own) {
            xc = (Tac)v_z + gather(t);
            const double d = v_sc * (double)xc;
            xs[j * M + t] = accumulate ? v_x + d : d;
            g[t] = (Tac)v_b * xc;
            const int jp = j > 0 ? j - 1 : 0;
            v_z = zs[jp * M + t];
            v_sc = scs[jp * M + t];
            v_x = accumulate ? xs[jp * M + t] : 0.0;
            v_b = bs[jp * M + t];
        }
        __syncthreads();
    };
    if constexpr (DEPTH >= 1) {
        if (m >= 2) load(m - 2, bA);
    }
    if constexpr (DEPTH == 2) {
        if (m >= 3) load(m - 3, bB);
    }
    __syncthreads();
    {
        int j = m - 2;
        if constexpr (DEPTH == 2) {
            for (; j - 2 >= 0; j -= 3) {
                back(j, bA, bC);
                back(j - 1, bB, bA);
                back(j - 2, bC, bB);
            }
            if (j >= 0) back(j--, bA, bC);
            if (j >= 0) back(j--, bB, bA);
        } else if constexpr (DEPTH == 1) {
            for (; j - 1 >= 0; j -= 2) {
                back(j, bA, bB);
                back(j - 1, bB, bA);
            }
            if (j >= 0) back(j--, bA, bB);
        } else {
            for (; j >= 0; --j) back(j, bA, bA);
        }
    }
}


// Algorithm 2.1 for one sample per workgroup, after the factorisation:
// x0 = S Ahat^{-1} S b, then {r = b - A x (FP64); stop test; x += solve(r)}.
// With `direct` the first residual only yields Q and the relative residual.
// Workgroups b >= *count (when count is given) exit at once.
// Two workgroups of the n = 128 low-precision refinement share a CU (>= 4
// waves per SIMD), so that a batch of up to 512 samples runs in one round.
template <typename Tst, int M, int G> constexpr int ir_min_waves()
{
    return (M == 128 && G == 2 && sizeof(Tst) <= 4) ? 4 : 1;
}
template <typename Tst, int M, int G, bool PREF, int D>
__global__ __launch_bounds__((64 * blk_waves<M, G>())) __attribute__((amdgpu_waves_per_eu(ir_min_waves<Tst, M, G>()))) void k_ir_blk(
    int n, double fconst, const double *__restrict__ a, const double *__restrict__ sc,
    const double *__restrict__ beta, const Tst *__restrict__ factor, double *__restrict__ x,
    double *__restrict__ r, double *__restrict__ zbuf, double eps, int imax, int direct,
    const int *__restrict__ idx, const int *__restrict__ count, int64_t slot_base,
    uint32_t *__restrict__ state, double *__restrict__ relres, double *__restrict__ q,
    int32_t *__restrict__ iters, int fwd_done)
{
    constexpr int NB = M / 16, NBL = NB * (NB + 1) / 2, m = M - 1, NT = 64 * blk_waves<M, G>();
    __shared__ double red[3 * NT];
    const int b = blockIdx.x;
    if (count && b >= *count) return;
    const int s = idx ? idx[b] : b;
    const size_t vo = (size_t)s * m * M;
    const double *scs = sc + vo, *bs = beta + vo;
    const Tst *fs = factor + (size_t)(slot_base + b) * m * NBL * 256;
    double *xs = x + vo, *rsb = r + vo, *zs = zbuf + vo;
    const double *as = a + (size_t)s * (n + 1) * (n + 1);
    const double h = 1.0 / n;
    // fwd_done 2: the factorisation ran the whole initial solve (x0 in x)
    if (fwd_done != 2) solve_blk_pass<Tst, M, G, PREF>(scs, bs, fs, nullptr, h * h * fconst, xs, 0, zs, fwd_done != 0);
    uint32_t st = state[s] & ~(uint32_t)ST_DONE;
    double prev = INFINITY, rel = INFINITY, sx = 0.0;
    int trip = 0;
    for (;;) {
        __syncthreads();
        const resid_out o = residual_pass_m<NT, M, D>(fconst, as, xs, rsb, red);
        rel = sqrt(o.rr) / sqrt(o.bb);
        sx = o.sx;
        st = ir_decide(st, rel, prev, sx, eps, trip, imax, direct);
        if (st & ST_DONE) break;
        prev = rel;
        __syncthreads();
        solve_blk_pass<Tst, M, G, PREF>(scs, bs, fs, rsb, 0.0, xs, 1, zs);
        ++trip;
    }
    if (threadIdx.x == 0) {
        state[s] = st;
        relres[s] = rel;
        q[s] = h * h * sx;
        if (iters) iters[s] = trip;
    }
}

// ------------------------------------------------------------------ launchers

namespace {

// Default waves per block-row pair (G) of the refinement kernel, within the
// register budget (the autotuner may choose the other one).
template <typename Tst, int M> struct solve_cfg { static constexpr int G = 1; };
template <typename Tst> struct solve_cfg<Tst, 128> { static constexpr int G = 2; };
template <typename Tst> struct solve_cfg<Tst, 256> { static constexpr int G = 2; };
template <> struct solve_cfg<double, 64> { static constexpr int G = 2; };
template <> struct solve_cfg<double, 128> { static constexpr int G = 2; };
template <> struct solve_cfg<double, 256> { static constexpr int G = 1; };

// Refinement kernel variants: G waves per block-row pair (1 or 2); the FP64
// n = 256 variant keeps no register double-buffer (register budget).
template <typename Tst, int M, int G> struct ir_pref { static constexpr bool v = true; };
template <int G> struct ir_pref<double, 256, G> { static constexpr bool v = false; };

template <typename Tst, int M, int G, int D>
hipError_t li_g(const ir_args &g, hipStream_t st)
{
    constexpr bool PREF = ir_pref<Tst, M, G>::v;
    hipLaunchKernelGGL((k_ir_blk<Tst, M, G, PREF, D>), dim3(g.nblocks), dim3(64 * blk_waves<M, G>()), 0, st, g.n,
                       g.fconst, g.a, g.sc, g.beta, (const Tst *)g.factor, g.x, g.r, g.z, g.eps,
                       g.imax, g.direct, g.idx, g.count, g.slot_base, g.state, g.relres, g.q, g.iters,
                       g.fwd_done);
    return hipGetLastError();
}

template <typename Tst, bool STRIDE, int D>
void li_rows16(const ir_args &g, dim3 grid, hipStream_t st)
{
    hipLaunchKernelGGL((k_ir_rows16<Tst, STRIDE, D>), grid, dim3(256), 0, st, g.nblocks, g.fconst, g.a, g.sc,
                       g.beta, (const Tst *)g.factor, g.x, g.z, g.eps, g.imax, g.direct, g.idx, g.count,
                       g.slot_base, g.state, g.relres, g.q, g.iters, g.fwd_done);
}

template <typename Tst, int M>
hipError_t li(const ir_args &g, hipStream_t st)
{
    if constexpr (M == 16) {
        if (g.nblocks == 0) return hipSuccess;
        const unsigned grid = (unsigned)((g.nblocks + 15) / 16);
        const dim3 gr(g.idx && grid > 1024 ? 1024 : grid);
        if (g.idx && g.disc) li_rows16<Tst, true, 1>(g, gr, st);
        else if (g.idx) li_rows16<Tst, true, 0>(g, gr, st);
        else if (g.disc) li_rows16<Tst, false, 1>(g, gr, st);
        else li_rows16<Tst, false, 0>(g, gr, st);
        return hipGetLastError();
    } else {
        const int G = g.variant > 0 ? g.variant : solve_cfg<Tst, M>::G;
        if (g.disc) return G == 2 ? li_g<Tst, M, 2, 1>(g, st) : li_g<Tst, M, 1, 1>(g, st);
        return G == 2 ? li_g<Tst, M, 2, 0>(g, st) : li_g<Tst, M, 1, 0>(g, st);
    }
}

template <typename Tst>
hipError_t li_m(const ir_args &g, hipStream_t st)
{
    switch (g.n) {
    case 16: return li<Tst, 16>(g, st);
    case 32: return li<Tst, 32>(g, st);
    case 64: return li<Tst, 64>(g, st);
    case 128: return li<Tst, 128>(g, st);
    case 256: return li<Tst, 256>(g, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_ir_blk(int dtype, const ir_args &g, hipStream_t st)
{
    switch (dtype) {
    case 0: return li_m<double>(g, st);
    case 1: return li_m<float>(g, st);
    case 2: return li_m<__hip_bfloat16>(g, st);
    case 3: return li_m<__half>(g, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace mlmc
