// Block-layout factorisations (M = n, the padded block size): the MFMA
// kernels for M >= 32 (every such grid for the FP32/BF16/FP16 factors,
// n >= 64 for the FP64 factor), the one-row-per-lane kernel for the n = 16
// grid (every factor type), and the KL field on MFMA.  The refinement
// kernels that apply the stored factor are in refine_blk.hip.
//
// Each Schur complement C_j (M x M, SPD) is inverted in place by the sweep
// operator applied to 16-pivot panels: with V = C[:, K] (the panel columns,
// M x 16) and P = C[K, K],
//   C[K, K] <- -P^{-1},  C[I, K] <- V_I P^{-1},  C[R, R] <- C[R, R] - V_R P^{-1} V_R^T,
// which equals sweeping the 16 pivots one at a time.  The lower-triangle
// 16 x 16 blocks of C live in MFMA accumulator registers (one wave owns every
// W-th block); the rank-16 trailing update runs on v_mfma 16x16x4 (FP32 for
// the FP32/BF16/FP16 factors, FP64 for the FP64 factor); -P^{-1} is formed
// by one wave of the group in 16 broadcast sweep steps and shared through LDS.
//
// Stored factor: per Schur block j, NBL = NB(NB+1)/2 lower blocks b (row by
// row), each in the MFMA result layout: entry (row drow(l/16, r), col l%16) of
// block b at offset (b*64 + l)*4 + r, so that a lane's four entries of a block
// are one contiguous vector access.
//
// Where twisted<Tac, M>() holds (blk_common.h) the workgroup has two wave
// groups: the first forms C_0 .. C_{k-1} from the top, the second
// D_{m-1} .. D_{k+1} from the bottom (D_{m-1} = T_{m-1},
// D_j = T_j - B_{j+1} D_{j+1}^{-1} B_{j+1}), both at once, and the middle
// block E_k = T_k - B_k C_{k-1}^{-1} B_k - B_{k+1} D_{k+1}^{-1} B_{k+1} is
// summed from the two groups' registers and inverted by the first.  Block row
// j of the stored factor holds -C_j^{-1}, -E_k^{-1} or -D_j^{-1}; the solve
// (refine_blk.hip) runs the matching sweeps.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "blk_common.h"
#include "dtypes.h"
#include "ir_common.h"
#include "kernels.h"

namespace mlmc {

// Whether the factorisation also runs the forward sweep of the initial solve
// (z_j = -F_j (s_j rhs - beta_j z_{j-1}) with each F_j as it is formed), so
// that the solve starts with the back sweep (or, where the twisted layout's
// factorisation runs that too, with the residual): the FP32/BF16/FP16 factors.  In
// FP64 the partial sums would add 12-50 KB of LDS to a workgroup that already
// holds 36-130 KB, crowding out the kernels of the other levels that share
// its CU in the multi-level step (measured: slower and erratic steps).
template <typename Tac, int M> constexpr bool factor_fwd_ok() { return sizeof(Tac) == 4; }

// H16: for the FP16/BF16 factors, form the products in the storage format
// (one 16x16x16 MFMA per block product); false: four FP32 16x16x4 products
// (the autotuner chooses per grid, as the faster factorisation can cost more
// corrections).  Where twisted<Tac, M>() holds, two wave groups eliminate
// from both ends (blk_common.h): the chain of one sample is half as long.
template <typename Tst, int M> constexpr int factor_groups()
{
    return twisted<typename store_traits<Tst>::acc, M>() ? 2 : 1;
}
template <typename Tst, int M, bool H16 = true>
__global__ __launch_bounds__((64 * blk_waves<M, 1>() * factor_groups<Tst, M>())) void k_factor_mfma(int S, const double *__restrict__ beta,
                                                             const double *__restrict__ gam,
                                                             Tst *__restrict__ factor,
                                                             const int *__restrict__ idx,
                                                             const int *__restrict__ count,
                                                             int64_t slot_base,
                                                             uint32_t *__restrict__ state,
                                                             const double *__restrict__ fsc, double frhs,
                                                             double *__restrict__ fz, double *__restrict__ x0)
{
    using Tac = typename store_traits<Tst>::acc;
    using V4 = typename vec4_of<Tac>::type;
    constexpr int NB = M / 16, NBL = NB * (NB + 1) / 2, W = blk_waves<M, 1>(), SPW = blk_slots<M, 1>();
    constexpr int m = M - 1, LD = 17, NT = 64 * W;
    constexpr bool FWD = factor_fwd_ok<Tac, M>();
    constexpr bool TW = twisted<Tac, M>();
    constexpr int NG = TW ? 2 : 1, KM = (m - 1) / 2, STEPS = TW ? KM + 1 : m;
    // per wave group (the twisted elimination's two chains; one group otherwise)
    __shared__ Tac Vb_[NG][2][M * LD];      // panel columns C[:, K], double-buffered
    __shared__ Tac Pw_[NG][16 * LD];        // -P^{-1} of the group's panel
    __shared__ Tac Uw_[NG][W][2][16 * LD];  // per wave: U of its two block rows
    __shared__ Tac bj_[NG][2][M], gj_[NG][2][M];
    // forward sweep (fz != NULL): right-hand side of the block, and per wave
    // its row sums and column partials, each in its own slot (fixed-order sum)
    __shared__ Tac gfw_[NG][FWD ? M : 1];
    __shared__ Tac partR_[NG][FWD ? W : 1][FWD ? M : 1];
    __shared__ Tac partC_[NG][FWD ? W : 1][2][FWD ? M : 1];
    __shared__ Tac xk_[(FWD && TW) ? M : 1];  // x_k, passed to the bottom group's back sweep
    __shared__ int bad;
    const int b = blockIdx.x;
    if (count && b >= *count) return;
    const int s = idx ? idx[b] : b;
    const int64_t slot = slot_base + b;
    // group 0 walks the block rows from the top, group 1 (twisted) from the
    // bottom: chain step j is row rowof(j), coupled to the previous step's row
    // by the beta stored at row brow(j) (j >= 1)
    const int grp = TW ? __builtin_amdgcn_readfirstlane((int)threadIdx.x / NT) : 0;
    auto &Vb = Vb_[grp];
    auto &Pw = Pw_[grp];
    auto &Uw = Uw_[grp];
    auto &bj = bj_[grp];
    auto &gj = gj_[grp];
    auto &gfw = gfw_[grp];
    auto &partR = partR_[grp];
    auto &partC = partC_[grp];
    auto rowof = [&](int jj) { return grp ? m - 1 - jj : jj; };
    auto brow = [&](int jj) { return grp ? m - jj : jj; };
    const int t = (int)threadIdx.x - grp * NT, l = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int lr = l >> 4, lc = l & 15;
    const double *bs = beta + (size_t)s * m * M;
    const double *gs = gam + (size_t)s * m * M;
    Tst *fs = factor + (size_t)slot * m * NBL * 256;
    if (threadIdx.x == 0) bad = 0;
    const bool fwd = FWD && fz != nullptr;
    const double *fscs = fwd ? fsc + (size_t)s * m * M : nullptr;
    double *fzs = fwd ? fz + (size_t)s * m * M : nullptr;
    if constexpr (FWD) {
        for (int i = l; i < M; i += 64) {
            partR[w][i] = 0;
            partC[w][0][i] = 0;
            partC[w][1][i] = 0;
        }
    }
    Tac zc = 0;  // z_{j-1}, entry t (t < M)
    V4 acc[SPW];
#pragma unroll
    for (int q = 0; q < SPW; ++q) acc[q] = V4{0, 0, 0, 0};
    // coefficients of block 0 now, of block j+1 prefetched during block j
    double pb = 0.0, pg = 0.0;
    if (t < M) {
        pb = grp ? 0.0 : bs[t];
        pg = gs[rowof(0) * M + t];
    }
    bool okw = true, okc = true;
    // The wave's partials of F g (g in gfw, entries of F by fval(slot, r)):
    // row sums of its tiles reduced across 16-lane rows, transposed
    // contributions of the off-diagonal tiles across the four lane rows, each
    // in its own slot (the solve's fixed-order scheme).
    auto partials = [&](int wj, auto &&fval) {
        Tac ra0[4] = {0, 0, 0, 0}, ra1[4] = {0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < SPW; ++q) {
            int I, J;
            slot_blk<NB, 1>(wj, q, I, J);
            Tac f[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) f[r] = fval(q, r);
            const Tac gjv = gfw[16 * J + lc];
            const bool first = (I == wj);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (first)
                    ra0[r] = fma(f[r], gjv, ra0[r]);
                else
                    ra1[r] = fma(f[r], gjv, ra1[r]);
            }
            if (I != J) {
                Tac c = 0;
#pragma unroll
                for (int r = 0; r < 4; ++r) c = fma(f[r], gfw[16 * I + drow<Tac>(lr, r)], c);
                c = rows4_total(c);
                if (lr == 0) partC[wj][first ? 0 : 1][16 * J + lc] = c;
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const Tac v0 = row16_total(ra0[r]);
            const Tac v1 = row16_total(ra1[r]);
            if (lc == 15) {
                partR[wj][16 * wj + drow<Tac>(lr, r)] = v0;
                if (NB > 1) partR[wj][16 * (NB - 1 - wj) + drow<Tac>(lr, r)] = v1;
            }
        }
    };
    auto gathered = [&](auto i) {
        Tac v = 0;
#pragma unroll
        for (int ww = 0; ww < W; ++ww) v += partR[ww][i] + partC[ww][0][i] + partC[ww][1][i];
        return v;
    };

    for (int j = 0; j < STEPS; ++j) {
        const int jb = j & 1, row = rowof(j);
        // the middle block row (twisted): the top group forms T + B F B, the
        // bottom group B G B, their sum is E_k; only the top group's result
        // (and flags) count
        const bool mid = TW && j == KM, skipT = mid && grp == 1;
        if (mid) okc = okw;
        if (t < M) {
            bj[jb][t] = (Tac)pb;
            gj[jb][t] = (Tac)pg;
            if (j + 1 < STEPS) {
                pb = bs[brow(j + 1) * M + t];
                pg = gs[rowof(j + 1) * M + t];
            }
        }
        __syncthreads();
        int wj = w;
        asm volatile("" : "+s"(wj));  // keep per-slot addresses out of registers across iterations
        // C_j = T_j + diag(beta_j) (-C_{j-1}^{-1}) diag(beta_j)
#pragma unroll
        for (int q = 0; q < SPW; ++q) {
            int I, J;
            slot_blk<NB, 1>(wj, q, I, J);
            const int C = 16 * J + lc;
            const Tac bc = bj[jb][C], gc = gj[jb][C];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int R = 16 * I + drow<Tac>(lr, r);
                const Tac gr = gj[jb][R];  // unconditional loads keep the update branch-free
                Tac tv = (R == C + 1) ? gc : (Tac)0;
                tv = (C == R + 1) ? gr : tv;
                tv = (R == C) ? (Tac)1 : tv;
                acc[q][r] = bj[jb][R] * acc[q][r] * bc + (skipT ? (Tac)0 : tv);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (TW) {
            if (mid) {
                // E_k = (T + B F B) + (B G B), passed four slots per wave at a
                // time through the bottom group's panel buffer (idle until its
                // panel loop); both groups then run the panel loop, the bottom
                // one on its own part (its results are not used)
                Tac *XB = &Vb_[1][0][0];
                static_assert(4 * W * 256 <= 2 * M * LD, "exchange buffer");
#pragma unroll
                for (int q0 = 0; q0 < SPW; q0 += 4) {
                    if (grp == 1)
#pragma unroll
                        for (int q = q0; q < q0 + 4 && q < SPW; ++q)
#pragma unroll
                            for (int r = 0; r < 4; ++r) XB[(w * 4 + (q - q0)) * 256 + l * 4 + r] = acc[q][r];
                    __syncthreads();
                    if (grp == 0)
#pragma unroll
                        for (int q = q0; q < q0 + 4 && q < SPW; ++q)
#pragma unroll
                            for (int r = 0; r < 4; ++r) acc[q][r] += XB[(w * 4 + (q - q0)) * 256 + l * 4 + r];
                    __syncthreads();
                }
            }
        }
        for (int K = 0; K < NB; ++K) {
            int wk = w;
            asm volatile("" : "+s"(wk));
            Tac *V = Vb[K & 1];
            // publish the panel columns C[:, K]
#pragma unroll
            for (int q = 0; q < SPW; ++q) {
                int I, J;
                slot_blk<NB, 1>(wk, q, I, J);
                if (J == K) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) V[(16 * I + drow<Tac>(lr, r)) * LD + lc] = acc[q][r];
                } else if (I == K) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) V[(16 * J + lc) * LD + drow<Tac>(lr, r)] = acc[q][r];
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            __syncthreads();
            asm volatile("" : "+s"(wk));
            // one wave of the group forms -P^{-1} (the sweeping wave rotates over
            // the SIMDs with K, the two groups' on different SIMDs; the others
            // wait at the barrier rather than repeat the sweep: the kernel is
            // issue-bound where two workgroups share a CU), then every wave
            // forms U for its two block rows
            Tac *P = Pw;
            if (W == 1 || wk == (K + 2 * grp) % W) {
                Tac p[4];  // lane 16 g + i: P[i][4g .. 4g+3]
#pragma unroll
                for (int c = 0; c < 4; ++c) p[c] = V[(16 * K + lc) * LD + 4 * lr + c];
                okw = sweep16(p, l) && okw;
#pragma unroll
                for (int c = 0; c < 4; ++c) P[lc * LD + 4 * lr + c] = p[c];
            }
            if constexpr (W > 1)
                __syncthreads();
            else
                wave_lds_sync();
            // -P^{-1}[4kc+lr][lc] (= [lc][4kc+lr] by symmetry) is the B operand of U and
            // the A operand of row K; U rows are re-read in the A layout per block below
            // (operands are re-read from LDS rather than held, to bound registers).
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                const int row = x ? NB - 1 - wk : wk;
                V4 u = V4{0, 0, 0, 0};
                if constexpr (H16 && mfma_in_storage<Tst>()) {
                    float av[4], bv[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        av[c] = V[(16 * row + lc) * LD + 4 * lr + c];
                        bv[c] = P[(4 * lr + c) * LD + lc];
                    }
                    u = mfma16<Tst>(av, bv, u);
                } else {
#pragma unroll
                    for (int kc = 0; kc < 4; ++kc)
                        u = mfma4(V[(16 * row + lc) * LD + 4 * kc + lr], P[(4 * kc + lr) * LD + lc], u);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) Uw[wk][x][drow<Tac>(lr, r) * LD + lc] = u[r];
            }
            wave_lds_sync();
#pragma unroll
            for (int q = 0; q < SPW; ++q) {
                int I, J;
                slot_blk<NB, 1>(wk, q, I, J);
                const Tac *U = Uw[wk][(q <= wk) ? 0 : 1];  // which of the wave's two rows
                if (I != K && J != K) {
                    // C[I,J] += U_I V_J^T
                    Tac av[4], bv[4];
                    if constexpr (H16 && mfma_in_storage<Tst>()) {
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            av[c] = U[lc * LD + 4 * lr + c];
                            bv[c] = V[(16 * J + lc) * LD + 4 * lr + c];
                        }
                        acc[q] = mfma16<Tst>(av, bv, acc[q]);
                    } else {
#pragma unroll
                        for (int kc = 0; kc < 4; ++kc) {
                            av[kc] = U[lc * LD + 4 * kc + lr];
                            bv[kc] = V[(16 * J + lc) * LD + 4 * kc + lr];
                        }
#pragma unroll
                        for (int kc = 0; kc < 4; ++kc) acc[q] = mfma4(av[kc], bv[kc], acc[q]);
                    }
                } else if (I == K && J == K) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[q][r] = P[drow<Tac>(lr, r) * LD + lc];
                } else if (J == K) {
                    // C[I,K] = V_I P^{-1} = -U_I
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[q][r] = -U[drow<Tac>(lr, r) * LD + lc];
                } else {
                    // C[K,J] = (V_J P^{-1})^T = P^{-1} V_J^T = -((-P^{-1}) V_J^T)
                    V4 z = V4{0, 0, 0, 0};
                    if constexpr (H16 && mfma_in_storage<Tst>()) {
                        float av[4], bv[4];
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            av[c] = P[(4 * lr + c) * LD + lc];
                            bv[c] = V[(16 * J + lc) * LD + 4 * lr + c];
                        }
                        z = mfma16<Tst>(av, bv, z);
                    } else {
#pragma unroll
                        for (int kc = 0; kc < 4; ++kc)
                            z = mfma4(P[(4 * kc + lr) * LD + lc], V[(16 * J + lc) * LD + 4 * kc + lr], z);
                    }
                    acc[q] = -z;
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        // store -C_j^{-1}
        asm volatile("" : "+s"(wj));
        Tst *fb = fs + (size_t)row * NBL * 256;
        const bool keep = !(mid && grp == 1);
#pragma unroll
        for (int q = 0; q < SPW; ++q) {
            int I, J;
            slot_blk<NB, 1>(wj, q, I, J);
            const int bb = I * (I + 1) / 2 + J;
            quad<Tst> qv;
#pragma unroll
            for (int r = 0; r < 4; ++r) qv.v[r] = store_traits<Tst>::store(acc[q][r]);
            if (keep) *(quad<Tst> *)(fb + ((size_t)bb * 64 + l) * 4) = qv;
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (FWD) {
            if (fwd) {
                // z_j = -F_j g_j with F_j as stored (rounded to Tst), the same
                // sums as the solve's forward sweep: row sums of the wave's tiles
                // reduced across 16-lane rows, transposed contributions of the
                // off-diagonal tiles across the four lane rows
                if (t < M) {
                    const Tac gv = (Tac)(fscs[row * M + t] * (t < m ? frhs : 0.0));
                    // the bottom group's part of the middle row: -beta_{k+1} w_{k+1}
                    gfw[t] = skipT ? -(Tac)bs[brow(j) * M + t] * zc
                                   : (j > 0 ? gv - (Tac)bs[brow(j) * M + t] * zc : gv);
                }
                __syncthreads();
                if constexpr (TW) {
                    if (mid) {
                        // g_k - beta_k z_{k-1} - beta_{k+1} w_{k+1}
                        if (grp == 0 && t < M) gfw[t] += gfw_[1][t];
                        __syncthreads();
                    }
                }
                asm volatile("" : "+s"(wj));
                partials(wj, [&](int q, int r) {
                    return store_traits<Tst>::load(store_traits<Tst>::store(acc[q][r]));
                });
                __syncthreads();
                if (t < M) {
                    zc = -gathered(t);
                    if (keep) fzs[row * M + t] = (double)zc;
                }
            }
        }
    }
    if constexpr (TW && FWD) {
        if (fwd && x0) {
            // The back sweeps of the initial solve, both chains at once, from
            // the middle outwards with the blocks as stored (each wave reads back
            // the tiles it wrote): x_j = z_j + F_j beta_{j+1} x_{j+1} (top),
            // x_j = w_j + F_j beta_j x_{j-1} (bottom); x0 = S x.
            double *xs0 = x0 + (size_t)s * m * M;
            if (grp == 0 && t < M) {
                xk_[t] = zc;
                xs0[KM * M + t] = fscs[KM * M + t] * (double)zc;
            }
            __syncthreads();
            Tac xp = t < M ? xk_[t] : (Tac)0;
            // step jj: block row KM - 1 - jj (top) or KM + 1 + jj (bottom); the
            // next step's tiles load while this one is applied (two buffers that
            // rotate by unrolling)
            auto brow_of = [&](int jj) { return grp ? KM + 1 + jj : KM - 1 - jj; };
            auto ld = [&](int jj, quad<Tst> (&dst)[SPW]) {
                int wq = w;
                asm volatile("" : "+s"(wq));
                const Tst *fb = fs + (size_t)brow_of(jj) * NBL * 256;
#pragma unroll
                for (int q = 0; q < SPW; ++q) {
                    int I, J;
                    slot_blk<NB, 1>(wq, q, I, J);
                    dst[q] = *(const quad<Tst> *)(fb + ((size_t)(I * (I + 1) / 2 + J) * 64 + l) * 4);
                }
            };
            auto bstep = [&](int jj, quad<Tst> (&use)[SPW], quad<Tst> (&fill)[SPW]) {
                const int row = brow_of(jj);
                const int bi = grp ? row : row + 1;
                ld(jj + 1 < KM ? jj + 1 : KM - 1, fill);  // a redundant last load is harmless
                if (t < M) gfw[t] = (Tac)bs[bi * M + t] * xp;
                __syncthreads();
                int wj = w;
                asm volatile("" : "+s"(wj));
                partials(wj, [&](int q, int r) { return store_traits<Tst>::load(use[q].v[r]); });
                __syncthreads();
                if (t < M) {
                    xp = (Tac)fzs[row * M + t] + gathered(t);
                    xs0[row * M + t] = fscs[row * M + t] * (double)xp;
                }
            };
            quad<Tst> tA[SPW], tB[SPW];
            ld(0, tA);
            int jj = 0;
            for (; jj + 2 <= KM; jj += 2) {
                bstep(jj, tA, tB);
                bstep(jj + 1, tB, tA);
            }
            if (jj < KM) bstep(jj, tA, tB);
        }
    }
    if (TW && grp == 1) okw = okc;
    if (!okw) bad = 1;
    __syncthreads();
    if (threadIdx.x == 0 && bad) atomicOr(&state[s], ST_NONFINITE | ST_BREAKDOWN);
}

// Factorisation of one sample per 16 lanes, 16 samples per workgroup: the
// stored layout of k_factor_mfma at M = 16, and the forward sweep of the
// initial solve for every factor type.  It reads the nodal coefficient a and
// forms the scaled operator itself (the assembly pass is not run for this
// grid), writing the scaling and the row couplings the refinement uses.  The
// stored block keeps the entry (row drow(g, c), column r) of MFMA lane
// l = 16 g + r at offset
// l * 4 + c; by symmetry that is entry drow(g, c) of row r, so each lane
// stores four 4-entry vectors and the 16 lanes of a sample cover every
// 256-entry block contiguously.  The solves read each lane's vectors back as
// its row.  With x0 != NULL it also runs the back sweep of the initial solve
// and writes x0 there (z goes to fz on the way), so the refinement starts
// with the residual.
// STRIDE: a pass over promoted samples, launched with a capped grid (its
// device-side count is usually zero); its workgroups step through the slots
// by the grid.  D: the edge rule (0 finite volumes, 1 P1 elements), fixed at
// compile time so that each rule's kernel holds only its own registers.
template <typename Tst, bool STRIDE, int D>
__global__ __launch_bounds__(256) void k_factor_rows16(int S, const double *__restrict__ a,
                                                       double *__restrict__ sc, double *__restrict__ beta,
                                                       Tst *__restrict__ factor,
                                                       const int *__restrict__ idx,
                                                       const int *__restrict__ count,
                                                       int64_t slot_base, uint32_t *__restrict__ state,
                                                       double frhs, double *__restrict__ fz,
                                                       double *__restrict__ x0)
{
    constexpr int disc = D;
    using Tac = typename store_traits<Tst>::acc;
    constexpr int M = 16, m = M - 1, NP = M + 1;
    const int i = threadIdx.x & 15;
    for (int b = blockIdx.x * 16 + (threadIdx.x >> 4);; b += gridDim.x * 16) {
        // whole 16-lane rows leave together, so no DPP source lane of a live row is idle
        if (b >= S || (count && b >= *count)) return;
        const int s = idx ? idx[b] : b;
        const int64_t slot = slot_base + b;
        const size_t vo = (size_t)s * m * M + i;
        const double *ac = a + (size_t)s * NP * NP + (i + 1);  // node column i + 1
        // the first pass over a batch writes the scaling and the row couplings for
        // the refinement; a pass over promoted samples (idx) forms the same values
        const bool wr = idx == nullptr;
        double *scs = sc + vo, *bs = beta + vo;
        Tst *fs = factor + (size_t)slot * m * 256;
        const bool fwd = fz != nullptr;
        double *fzs = fwd ? fz + vo : nullptr;
        const bool in = i < m;  // lane m is the identity pad

        Tac a16[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) a16[c] = 0;
        Tac zc = 0;  // z_{j-1}, entry i
        // Scaled operator S A S of grid row j from the nodal coefficient, with the
        // assembly's operations in its order: the four face coefficients (the east
        // face is the next lane's west face, the south face the row before's
        // north face), s = 1/sqrt(their sum), gamma to the east neighbour and
        // beta to the row below; 0 in the pad.  Row j + 1's values are formed
        // while row j is swept (independent work for the sweep's latency gaps),
        // and the nodes they need were requested one row before that.
        // (disc 1, P1 faces: also the node south of the west node, carried in
        // wS, and the node east of the north node, the next lane's cN)
        double c = ac[NP], cN = ac[2 * NP], w = ac[NP - 1], wS = ac[-1];
        double aS = disc ? face_y(1, ac[0], c, dpp_f64<0x101>(c), ac[-1]) : hmean2(c, ac[0]), sS = 0.0;
        auto coeffs = [&](int j, double &sj, double &bj, double &gj) {
            double cNN = 0.0, wN = 0.0;
            if (j + 1 < m) {
                cNN = ac[(j + 3) * NP];
                wN = ac[(j + 2) * NP - 1];
            }
            double aw, an;
            if (disc) {
                aw = face_x(1, w, c, cN, wS);
                an = face_y(1, c, cN, dpp_f64<0x101>(cN), w);
            } else {
                aw = hmean2(c, w);
                an = hmean2(c, cN);
            }
            const double ae = dpp_f64<0x101>(aw);
            sj = in ? 1.0 / sqrt(aw + ae + aS + an) : 0.0;
            const double sE = dpp_f64<0x101>(sj);
            gj = (i + 1 < m) ? -ae * sj * sE : 0.0;
            bj = (in && j > 0) ? -aS * sj * sS : 0.0;
            if (wr) {
                scs[j * M] = sj;
                bs[j * M] = bj;
            }
            aS = an;
            sS = sj;
            c = cN;
            cN = cNN;
            wS = w;
            w = wN;
        };
        double sjn, bjn, gjn;
        coeffs(0, sjn, bjn, gjn);
        bool ok = true;

        for (int j = 0; j < m; ++j) {
            const double sj = sjn, bj = bjn, gj = gjn;
            if (j + 1 < m) coeffs(j + 1, sjn, bjn, gjn);
            const Tac bf = (Tac)bj, gf = (Tac)gj;
            const Tac gl = row_shr1(gf);  // gamma_j[i-1] (0 in lane 0)
            form_schur16(a16, bf, gf, gl, i);
            ok = sweep16_rows(a16, i) && ok;
            // store -C_j^{-1}
            Tst *fb = fs + (size_t)j * 256;
            Tac fr[16];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                quad<Tst> qv;
#pragma unroll
                for (int cc = 0; cc < 4; ++cc) {
                    qv.v[cc] = store_traits<Tst>::store(a16[drow<Tac>(g, cc)]);
                    fr[drow<Tac>(g, cc)] = store_traits<Tst>::load(qv.v[cc]);
                }
                *(quad<Tst> *)(fb + (16 * g + i) * 4) = qv;
            }
            if (fwd) {
                // z_j = -F_j (s_j rhs - beta_j z_{j-1}) with F_j as stored
                const Tac gv0 = (Tac)(sj * (in ? frhs : 0.0));
                const Tac gv = j > 0 ? gv0 - bf * zc : gv0;
                zc = -dot16_colbcast(fr, gv, (Tac)0);
                fzs[j * M] = (double)zc;
            }
        }
        if (fwd && x0 && wr) {
            // The back sweep of the initial solve, right after the factorisation, so
            // that the refinement only forms the residual when no correction is
            // needed: x_{m-1} = s z_{m-1}; x_j = s_j (z_j + F_j (beta_{j+1} x~_{j+1}))
            // with the arithmetic of the refinement kernel's back sweep.  Every
            // operand was stored by this lane above; each step requests the next
            // step's first.
            double *x0s = x0 + vo;
            quad<Tst> fq[2][4];
            double zp[2], sp[2], bp[2];
            auto req = [&](int j) {
#pragma unroll
                for (int g = 0; g < 4; ++g) fq[j & 1][g] = *(const quad<Tst> *)(fs + (size_t)j * 256 + (16 * g + i) * 4);
                zp[j & 1] = fzs[j * M];
                sp[j & 1] = scs[j * M];
                bp[j & 1] = bs[(j + 1) * M];
            };
            req(m - 2);
            Tac xc = (Tac)fzs[(m - 1) * M];
            x0s[(m - 1) * M] = scs[(m - 1) * M] * (double)xc;
#pragma unroll
            for (int j = m - 2; j >= 0; --j) {
                if (j > 0) req(j - 1);
                const Tac gv = (Tac)bp[j & 1] * xc;
                Tac f[16];
#pragma unroll
                for (int g = 0; g < 4; ++g)
#pragma unroll
                    for (int cc = 0; cc < 4; ++cc) f[drow<Tac>(g, cc)] = store_traits<Tst>::load(fq[j & 1][g].v[cc]);
                xc = (Tac)zp[j & 1] + dot16_colbcast(f, gv, (Tac)0);
                x0s[j * M] = sp[j & 1] * (double)xc;
            }
        }
        if (!ok && i == 0) atomicOr(&state[s], ST_NONFINITE | ST_BREAKDOWN);
        if constexpr (!STRIDE) return;
    }
}

// ------------------------------------------------------------------ KL field

// Z = xi Phi^T on all (n+1)^2 nodes and a = exp(Z), FP64 on v_mfma 16x16x4.
// A workgroup computes 64 samples x 64 nodes, wave w the 32 x 32 quarter
// (w / 2, w % 2) as 2 x 2 result tiles.  The contraction over the K modes
// runs in chunks of 16; in slice kk of a chunk the lane row lr stands for
// mode c0 + 4 lr + kk, so each lane reads four consecutive entries of a xi
// row (staged through LDS per chunk, read from global memory as whole
// 16-mode rows) and four rows of Phi^T (coalesced over the 16 nodes of a
// lane row).  Modes beyond K contribute zero; rows and nodes beyond S and P
// are not stored (their loads are clamped in bounds).
__global__ __launch_bounds__(256) void k_field_mfma(int S, int K, int P, const double *__restrict__ xi,
                                                    const double *__restrict__ phit,
                                                    double *__restrict__ a)
{
    const int t = threadIdx.x, l = t & 63, w = t >> 6, lr = l >> 4, lc = l & 15;
    const int s0 = blockIdx.y * 64 + 32 * (w >> 1), p0 = blockIdx.x * 64 + 32 * (w & 1);
    f64x4 acc[2][2];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = f64x4{0, 0, 0, 0};
    int rowc[2], colc[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        rowc[q] = min(s0 + 16 * q + lc, S - 1);
        colc[q] = min(p0 + 16 * q + lc, P - 1);
    }
    // xi[64 samples][16 modes] of the chunk, staged through LDS: the global
    // reads are then 128-byte rows (16 consecutive modes of a sample) instead
    // of one sample per lane
    __shared__ double xs[64][17];
    const int xr = t >> 2, xq = (t & 3) * 4;  // thread t stages sample row xr, modes xq .. xq + 3
    const int xrow = min(blockIdx.y * 64 + xr, S - 1);
    for (int c0 = 0; c0 < K; c0 += 16) {
        __syncthreads();  // the previous chunk's reads of xs are done
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = c0 + xq + e;
            xs[xr][xq + e] = k < K ? xi[(size_t)xrow * K + k] : 0.0;
        }
        __syncthreads();
        double av[2][4], bv[2][4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int k = c0 + 4 * lr + kk;
            const bool in = k < K;
            const int kc = in ? k : K - 1;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const double ph = phit[(size_t)kc * P + colc[q]];
                av[q][kk] = xs[32 * (w >> 1) + 16 * q + lc][4 * lr + kk];
                bv[q][kk] = in ? ph : 0.0;
            }
        }
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = mfma4(av[ti][kk], bv[tj][kk], acc[ti][tj]);
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = s0 + 16 * ti + drow<double>(lr, r), col = p0 + 16 * tj + lc;
                if (row < S && col < P) a[(size_t)row * P + col] = exp(acc[ti][tj][r]);
            }
}

// ------------------------------------------------------------------ launchers

namespace {

template <typename Tst, int M>
hipError_t lf(int nb, const double *a, double *sc, double *beta, const double *gam, void *factor,
              const int *idx, const int *count, int64_t slot_base, uint32_t *state, double frhs,
              double *fz, double *x0, int disc, int variant, hipStream_t st)
{
    if constexpr (M == 16) {
        if (nb == 0) return hipSuccess;
        const unsigned grid = (unsigned)((nb + 15) / 16);
        const dim3 gr(idx && grid > 1024 ? 1024 : grid);
        if (idx && disc)
            hipLaunchKernelGGL((k_factor_rows16<Tst, true, 1>), gr, dim3(256), 0, st, nb, a, sc, beta,
                               (Tst *)factor, idx, count, slot_base, state, frhs, fz, x0);
        else if (idx)
            hipLaunchKernelGGL((k_factor_rows16<Tst, true, 0>), gr, dim3(256), 0, st, nb, a, sc, beta,
                               (Tst *)factor, idx, count, slot_base, state, frhs, fz, x0);
        else if (disc)
            hipLaunchKernelGGL((k_factor_rows16<Tst, false, 1>), gr, dim3(256), 0, st, nb, a, sc, beta,
                               (Tst *)factor, idx, count, slot_base, state, frhs, fz, x0);
        else
            hipLaunchKernelGGL((k_factor_rows16<Tst, false, 0>), gr, dim3(256), 0, st, nb, a, sc, beta,
                               (Tst *)factor, idx, count, slot_base, state, frhs, fz, x0);
    } else {
        const dim3 block(64 * blk_waves<M, 1>() * factor_groups<Tst, M>());
        if (variant == 1 && mfma_in_storage<Tst>())
            hipLaunchKernelGGL((k_factor_mfma<Tst, M, false>), dim3(nb), block, 0, st, nb, beta, gam,
                               (Tst *)factor, idx, count, slot_base, state, sc, frhs, fz, x0);
        else
            hipLaunchKernelGGL((k_factor_mfma<Tst, M>), dim3(nb), block, 0, st, nb, beta, gam, (Tst *)factor, idx,
                               count, slot_base, state, sc, frhs, fz, x0);
    }
    return hipGetLastError();
}

template <typename Tst>
hipError_t lf_m(int M, int nb, const double *a, double *sc, double *beta, const double *gam, void *factor,
                const int *idx, const int *count, int64_t slot_base, uint32_t *state, double frhs,
                double *fz, double *x0, int disc, int variant, hipStream_t st)
{
    switch (M) {
    case 16: return lf<Tst, 16>(nb, a, sc, beta, gam, factor, idx, count, slot_base, state, frhs, fz, x0, disc, variant, st);
    case 32: return lf<Tst, 32>(nb, a, sc, beta, gam, factor, idx, count, slot_base, state, frhs, fz, x0, disc, variant, st);
    case 64: return lf<Tst, 64>(nb, a, sc, beta, gam, factor, idx, count, slot_base, state, frhs, fz, x0, disc, variant, st);
    case 128: return lf<Tst, 128>(nb, a, sc, beta, gam, factor, idx, count, slot_base, state, frhs, fz, x0, disc, variant, st);
    case 256: return lf<Tst, 256>(nb, a, sc, beta, gam, factor, idx, count, slot_base, state, frhs, fz, x0, disc, variant, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_field_mfma(int S, int K, int P, const double *xi, const double *phit, double *a,
                             hipStream_t st)
{
    if (S == 0) return hipSuccess;
    const dim3 grid((unsigned)((P + 63) / 64), (unsigned)((S + 63) / 64));
    hipLaunchKernelGGL(k_field_mfma, grid, dim3(256), 0, st, S, K, P, xi, phit, a);
    return hipGetLastError();
}

hipError_t launch_factor_blk(int dtype, int n, int nblocks, const double *a, double *sc, double *beta,
                             const double *gam, void *factor, const int *idx, const int *count,
                             int64_t slot_base, uint32_t *state, double frhs, double *fz, double *x0,
                             int disc, int variant, hipStream_t st)
{
    switch (dtype) {
    case 0: return lf_m<double>(n, nblocks, a, sc, beta, gam, factor, idx, count, slot_base, state, frhs, fz, x0, disc, variant, st);
    case 1: return lf_m<float>(n, nblocks, a, sc, beta, gam, factor, idx, count, slot_base, state, frhs, fz, x0, disc, variant, st);
    case 2: return lf_m<__hip_bfloat16>(n, nblocks, a, sc, beta, gam, factor, idx, count, slot_base, state, frhs, fz, x0, disc, variant, st);
    case 3: return lf_m<__half>(n, nblocks, a, sc, beta, gam, factor, idx, count, slot_base, state, frhs, fz, x0, disc, variant, st);
    }
    return hipErrorInvalidValue;
}

bool factor_fuses_forward(int dtype, int n)
{
    return use_blk(dtype, n) && (dtype != 0 || n == 16);
}

bool factor_solves_initial(int dtype, int n)
{
    if (n == 16) return true;
    if (!factor_fuses_forward(dtype, n)) return false;
    switch (n) {
    case 32: return twisted<float, 32>();
    case 64: return twisted<float, 64>();
    case 128: return twisted<float, 128>();
    }
    return false;
}

}  // namespace mlmc
