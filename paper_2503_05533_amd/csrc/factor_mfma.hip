// Block-layout factorisations and refinement (M = n, the padded block size):
// the MFMA kernels for M >= 32 (every such grid for the FP32/BF16/FP16
// factors, n >= 64 for the FP64 factor), and one-row-per-lane kernels for
// the n = 16 grid (every factor type), further below.
//
// Each Schur complement C_j (M x M, SPD) is inverted in place by the sweep
// operator applied to 16-pivot panels: with V = C[:, K] (the panel columns,
// M x 16) and P = C[K, K],
//   C[K, K] <- -P^{-1},  C[I, K] <- V_I P^{-1},  C[R, R] <- C[R, R] - V_R P^{-1} V_R^T,
// which equals sweeping the 16 pivots one at a time.  The lower-triangle
// 16 x 16 blocks of C live in MFMA accumulator registers (one wave owns every
// W-th block); the rank-16 trailing update runs on v_mfma 16x16x4 (FP32 for
// the FP32/BF16/FP16 factors, FP64 for the FP64 factor); -P^{-1} is formed
// inside every wave by 16 broadcast sweep steps.
//
// Stored factor: per Schur block j, NBL = NB(NB+1)/2 lower blocks b (row by
// row), each in the MFMA result layout: entry (row drow(l/16, r), col l%16) of
// block b at offset (b*64 + l)*4 + r, so that a lane's four entries of a block
// are one contiguous vector access.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dtypes.h"
#include "kernels.h"
#include "ir_common.h"

namespace mlmc {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
// Four consecutive stored entries, accessed as one vector load or store.
template <typename T> struct alignas(4 * sizeof(T)) quad { T v[4]; };

template <typename T> struct vec4_of;
template <> struct vec4_of<float> { using type = f32x4; };
template <> struct vec4_of<double> { using type = f64x4; };

__device__ inline f32x4 mfma4(float a, float b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline f64x4 mfma4(double a, double b, f64x4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// The FP16 and BF16 factors form their products in their own precision with
// FP32 accumulation: a rank-16 product of 16 x 16 blocks is one
// v_mfma_f32_16x16x16_{f16,bf16} whose operands are rounded to the storage
// type (lane l = 16 lr + lc holds A[lc][4 lr .. 4 lr + 3] and
// B[4 lr .. 4 lr + 3][lc]; the result has the layout of the FP32 16x16x4
// product).  The FP32 factor keeps four FP32 16x16x4 products.
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
template <typename Tst> constexpr bool mfma_in_storage() { return false; }
template <> constexpr bool mfma_in_storage<__half>() { return true; }
template <> constexpr bool mfma_in_storage<__hip_bfloat16>() { return true; }

template <typename Tst> __device__ inline f32x4 mfma16(const float a[4], const float b[4], f32x4 c);
template <> __device__ inline f32x4 mfma16<__half>(const float a[4], const float b[4], f32x4 c)
{
    const f16x4 av = {(_Float16)a[0], (_Float16)a[1], (_Float16)a[2], (_Float16)a[3]};
    const f16x4 bv = {(_Float16)b[0], (_Float16)b[1], (_Float16)b[2], (_Float16)b[3]};
    return __builtin_amdgcn_mfma_f32_16x16x16f16(av, bv, c, 0, 0, 0);
}
template <> __device__ inline f32x4 mfma16<__hip_bfloat16>(const float a[4], const float b[4], f32x4 c)
{
    const bf16x4 av = {(__bf16)a[0], (__bf16)a[1], (__bf16)a[2], (__bf16)a[3]};
    const bf16x4 bv = {(__bf16)b[0], (__bf16)b[1], (__bf16)b[2], (__bf16)b[3]};
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s16x4, av),
                                                      __builtin_bit_cast(s16x4, bv), c, 0, 0, 0);
}

// Row (within a 16 x 16 block) of result register r in lane group lr = l/16:
// FP32 16x16x4 puts D[4 lr + r][l%16] in register r, FP64 16x16x4 puts
// D[4 r + lr][l%16] there.
template <typename T> __device__ constexpr int drow(int lr, int r);
template <> __device__ constexpr int drow<float>(int lr, int r) { return 4 * lr + r; }
template <> __device__ constexpr int drow<double>(int lr, int r) { return 4 * r + lr; }

// Waves per sample and block slots per wave for block size M with G waves
// per row pair; a single block row (M = 16) is one wave with one block.
template <int M, int G> constexpr int blk_waves() { return M >= 32 ? G * (M / 16) / 2 : 1; }
template <int M, int G> constexpr int blk_slots() { return M >= 32 ? (M / 16 + G) / G : 1; }

// Block ownership: the NB block rows are paired (p, NB-1-p), which together
// hold NB+1 lower blocks; G waves share a pair, wave w = G p + h taking the
// pair's blocks h, h+G, h+2G, ...  Returns false for an empty slot.
template <int NB, int G>
__device__ inline bool slot_blk(int w, int q, int &I, int &J)
{
    const int p = w / G, qq = w % G + G * q;
    if (qq > NB) return false;
    if (qq <= p) {
        I = p;
        J = qq;
    } else {
        I = NB - 1 - p;
        J = qq - p - 1;
    }
    return true;
}

// Lane-`lane` value of a wave-uniform broadcast (readlane) and the DPP
// broadcast of lane k of every 16-lane row to the whole row (row_newbcast).
template <typename T> __device__ inline T bcast(T v, int lane);
template <> __device__ inline float bcast<float>(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
template <> __device__ inline double bcast<double>(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int K> __device__ inline float rowbcast(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x150 + K, 0xF, 0xF, false));
}
template <int K> __device__ inline double rowbcast(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x150 + K, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x150 + K, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Lane swaps across the four 16-lane rows of a wave (gfx950):
// permlane32_swap(x, y) yields ([x0 x1 y0 y1], [x2 x3 y2 y3]) and
// permlane16_swap(x, y) yields ([x0 y0 x2 y2], [x1 y1 x3 y3]) (rows of 16).
// Sum over the four rows of the lanes with the same l % 16, ((r0 + r2) + (r1 + r3)),
// returned in every lane.
__device__ inline float rows4_total(float v)
{
    const unsigned u = __float_as_uint(v);
    const auto a = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    const float s = __uint_as_float(a[0]) + __uint_as_float(a[1]);
    const unsigned us = __float_as_uint(s);
    const auto b = __builtin_amdgcn_permlane16_swap(us, us, false, false);
    return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}
__device__ inline double swap32_lo_hi(double v, int which)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    return __longlong_as_double(
        (long long)(((unsigned long long)(which ? hi[1] : hi[0]) << 32) | (which ? lo[1] : lo[0])));
}
__device__ inline double swap16_lo_hi(double v, int which)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    return __longlong_as_double(
        (long long)(((unsigned long long)(which ? hi[1] : hi[0]) << 32) | (which ? lo[1] : lo[0])));
}
__device__ inline double rows4_total(double v)
{
    const double s = swap32_lo_hi(v, 0) + swap32_lo_hi(v, 1);
    return swap16_lo_hi(s, 0) + swap16_lo_hi(s, 1);
}

// p[c] += P[K][4g+c] * me for c = 0..3, with P[K][4g+c] the value of p[c] in
// lane K of the 16-lane row: the row broadcast is the DPP operand of the
// FMA.  One wait pair covers a VALU write of p just before; within the block
// no instruction reads a register written by the one before it.
template <int K> __device__ inline void fmac4_rowbcast(float p[4], float me)
{
    asm volatile("s_nop 1\n\t"
                 "v_fmac_f32_dpp %0, %0, %4 row_newbcast:%c5 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %1, %1, %4 row_newbcast:%c5 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %2, %2, %4 row_newbcast:%c5 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %3, %3, %4 row_newbcast:%c5 row_mask:0xf bank_mask:0xf"
                 : "+v"(p[0]), "+v"(p[1]), "+v"(p[2]), "+v"(p[3])
                 : "v"(me), "i"(K));
}
template <int K> __device__ inline void fmac4_rowbcast(double p[4], double me)
{
#pragma unroll
    for (int c = 0; c < 4; ++c) p[c] = fma(rowbcast<K>(p[c]), me, p[c]);
}

template <typename T, int K>
__device__ inline void sweep_step(T p[4], int i, int g, bool &ok)
{
    const T pik = __shfl(p[K & 3], 16 * (K >> 2) + i, 64);                 // P[i][K]
    const T d = bcast(p[K & 3], 16 * (K >> 2) + K);                        // P[K][K]
    ok = ok && (d > (T)0) && isfinite(d);
    const T inv = recip(d), f = pik * inv;
    const bool piv = (i == K);
    // rows i != K: P[i][c] - f P[K][c]; row K (whose lanes hold p == rk):
    // P[K][c] / d, written P[K][c] + (1/d - 1) P[K][c] so one FMA serves both.
    // The pivots of the scaled SPD blocks are at most 1, so 1/d - 1 >= 0 up to
    // rounding and the form is accurate to rounding.  The multiplier is
    // formed with its sign so that the row broadcast folds into the FMA as
    // its DPP operand.
    const T me = piv ? inv - (T)1 : -f;
    fmac4_rowbcast<K>(p, me);  // p[c] += P[K][4g+c] me
    // column K sits in register K & 3 of lane row K >> 2: f there, -1/d at (K, K)
    constexpr int cK = K & 3;
    p[cK] = (g == (K >> 2)) ? (piv ? -inv : f) : p[cK];
}

// -P^{-1} of a 16 x 16 SPD matrix by the sweep operator inside one wave.
// Lane l = 16 g + i holds P[i][4g .. 4g+3] in p[0..3]; pivot row K reaches
// each 16-lane row by DPP row broadcast, the pivot column entry P[i][K] by
// one cross-lane permute.  Returns false if a pivot was not positive and finite.
template <typename T>
__device__ inline bool sweep16(T p[4], int l)
{
    const int i = l & 15, g = l >> 4;
    bool ok = true;
    sweep_step<T, 0>(p, i, g, ok);
    sweep_step<T, 1>(p, i, g, ok);
    sweep_step<T, 2>(p, i, g, ok);
    sweep_step<T, 3>(p, i, g, ok);
    sweep_step<T, 4>(p, i, g, ok);
    sweep_step<T, 5>(p, i, g, ok);
    sweep_step<T, 6>(p, i, g, ok);
    sweep_step<T, 7>(p, i, g, ok);
    sweep_step<T, 8>(p, i, g, ok);
    sweep_step<T, 9>(p, i, g, ok);
    sweep_step<T, 10>(p, i, g, ok);
    sweep_step<T, 11>(p, i, g, ok);
    sweep_step<T, 12>(p, i, g, ok);
    sweep_step<T, 13>(p, i, g, ok);
    sweep_step<T, 14>(p, i, g, ok);
    sweep_step<T, 15>(p, i, g, ok);
    return ok;
}

// Inclusive scan over the 16 lanes of a DPP row: lane 15 of each row ends
// with the row total.
template <int CTRL>
__device__ inline float dpp_f32(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_f64(double v)
{
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(bits & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline float row16_total(float v)
{
    v += dpp_f32<0x111>(v);
    v += dpp_f32<0x112>(v);
    v += dpp_f32<0x114>(v);
    v += dpp_f32<0x118>(v);
    return v;
}
__device__ inline double row16_total(double v)
{
    v += dpp_f64<0x111>(v);
    v += dpp_f64<0x112>(v);
    v += dpp_f64<0x114>(v);
    v += dpp_f64<0x118>(v);
    return v;
}

// Wave-scope ordering of LDS accesses between lanes of one wave.
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Whether the factorisation also runs the forward sweep of the initial solve
// (z_j = -F_j (s_j rhs - beta_j z_{j-1}) with each F_j as it is formed), so
// that the solve starts with the back sweep: the FP32/BF16/FP16 factors.  In
// FP64 the partial sums would add 12-50 KB of LDS to a workgroup that already
// holds 36-130 KB, crowding out the kernels of the other levels that share
// its CU in the multi-level step (measured: slower and erratic steps).
template <typename Tac, int M> constexpr bool factor_fwd_ok() { return sizeof(Tac) == 4; }

// H16: for the FP16/BF16 factors, form the products in the storage format
// (one 16x16x16 MFMA per block product); false: four FP32 16x16x4 products
// (the autotuner chooses per grid, as the faster factorisation can cost more
// corrections).
template <typename Tst, int M, bool H16 = true>
__global__ __launch_bounds__((64 * blk_waves<M, 1>())) void k_factor_mfma(int S, const double *__restrict__ beta,
                                                             const double *__restrict__ gam,
                                                             Tst *__restrict__ factor,
                                                             const int *__restrict__ idx,
                                                             const int *__restrict__ count,
                                                             int64_t slot_base,
                                                             uint32_t *__restrict__ state,
                                                             const double *__restrict__ fsc, double frhs,
                                                             double *__restrict__ fz)
{
    using Tac = typename store_traits<Tst>::acc;
    using V4 = typename vec4_of<Tac>::type;
    constexpr int NB = M / 16, NBL = NB * (NB + 1) / 2, W = blk_waves<M, 1>(), SPW = blk_slots<M, 1>();
    constexpr int m = M - 1, LD = 17, NT = 64 * W;
    constexpr bool FWD = factor_fwd_ok<Tac, M>();
    __shared__ Tac Vb[2][M * LD];      // panel columns C[:, K], double-buffered
    __shared__ Tac Pw[W][16 * LD];     // per wave: -P^{-1}
    __shared__ Tac Uw[W][2][16 * LD];  // per wave: U of its two block rows
    __shared__ Tac bj[2][M], gj[2][M];
    // forward sweep (fz != NULL): right-hand side of the block, and per wave
    // its row sums and column partials, each in its own slot (fixed-order sum)
    __shared__ Tac gfw[FWD ? M : 1];
    __shared__ Tac partR[FWD ? W : 1][FWD ? M : 1];
    __shared__ Tac partC[FWD ? W : 1][2][FWD ? M : 1];
    __shared__ int bad;
    const int b = blockIdx.x;
    if (count && b >= *count) return;
    const int s = idx ? idx[b] : b;
    const int64_t slot = slot_base + b;
    const int t = threadIdx.x, l = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int lr = l >> 4, lc = l & 15;
    const double *bs = beta + (size_t)s * m * M;
    const double *gs = gam + (size_t)s * m * M;
    Tst *fs = factor + (size_t)slot * m * NBL * 256;
    if (t == 0) bad = 0;
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
        pb = bs[t];
        pg = gs[t];
    }
    bool okw = true;

    for (int j = 0; j < m; ++j) {
        const int jb = j & 1;
        if (t < M) {
            bj[jb][t] = (Tac)pb;
            gj[jb][t] = (Tac)pg;
            if (j + 1 < m) {
                pb = bs[(j + 1) * M + t];
                pg = gs[(j + 1) * M + t];
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
                acc[q][r] = bj[jb][R] * acc[q][r] * bc + tv;
            }
            __builtin_amdgcn_sched_barrier(0);
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
            // every wave: -P^{-1} (redundantly), then U for its two block rows
            Tac *P = Pw[wk];
            {
                Tac p[4];  // lane 16 g + i: P[i][4g .. 4g+3]
#pragma unroll
                for (int c = 0; c < 4; ++c) p[c] = V[(16 * K + lc) * LD + 4 * lr + c];
                okw = sweep16(p, l) && okw;
#pragma unroll
                for (int c = 0; c < 4; ++c) P[lc * LD + 4 * lr + c] = p[c];
            }
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
        Tst *fb = fs + (size_t)j * NBL * 256;
#pragma unroll
        for (int q = 0; q < SPW; ++q) {
            int I, J;
            slot_blk<NB, 1>(wj, q, I, J);
            const int bb = I * (I + 1) / 2 + J;
            quad<Tst> qv;
#pragma unroll
            for (int r = 0; r < 4; ++r) qv.v[r] = store_traits<Tst>::store(acc[q][r]);
            *(quad<Tst> *)(fb + ((size_t)bb * 64 + l) * 4) = qv;
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (FWD) {
            if (fwd) {
                // z_j = -F_j g_j with F_j as stored (rounded to Tst), the same
                // sums as the solve's forward sweep: row sums of the wave's tiles
                // reduced across 16-lane rows, transposed contributions of the
                // off-diagonal tiles across the four lane rows
                if (t < M) {
                    const Tac gv = (Tac)(fscs[j * M + t] * (t < m ? frhs : 0.0));
                    gfw[t] = j > 0 ? gv - (Tac)bs[j * M + t] * zc : gv;
                }
                __syncthreads();
                asm volatile("" : "+s"(wj));
                Tac ra0[4] = {0, 0, 0, 0}, ra1[4] = {0, 0, 0, 0};
#pragma unroll
                for (int q = 0; q < SPW; ++q) {
                    int I, J;
                    slot_blk<NB, 1>(wj, q, I, J);
                    Tac f[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) f[r] = store_traits<Tst>::load(store_traits<Tst>::store(acc[q][r]));
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
                __syncthreads();
                if (t < M) {
                    Tac v = 0;
#pragma unroll
                    for (int ww = 0; ww < W; ++ww) v += partR[ww][t] + partC[ww][0][t] + partC[ww][1][t];
                    zc = -v;
                    fzs[j * M + t] = (double)zc;
                }
            }
        }
    }
    if (!okw) bad = 1;
    __syncthreads();
    if (t == 0 && bad) atomicOr(&state[s], ST_NONFINITE | ST_BREAKDOWN);
}

// ------------------------------------------------- single-block grids (M = 16)
//
// For M = 16 every Schur block is one 16 x 16 tile, and a wave factors four
// samples at once (FP32 arithmetic for the FP32/BF16/FP16 factors, FP64 for
// the FP64 factor): lane l works on sample l / 16 and holds row i = l % 16 of
// the current block in 16 registers (register c = column c).
// Pivot row K is the value of register c in lane K of the same 16-lane row,
// the DPP row-broadcast operand of one FMA per register; pivot column K is the
// lane's own register K.  No LDS and no barrier: samples never share lanes.

// One wait pair before a DPP read of a register that a VALU wrote just before;
// the DPP source of each line below is not written by the line before it.
template <int K> __device__ inline float rowbcast_w(float v)
{
    float r;
    asm volatile("s_nop 1\n\tv_mov_b32_dpp %0, %1 row_newbcast:%c2 row_mask:0xf bank_mask:0xf"
                 : "=v"(r)
                 : "v"(v), "i"(K));
    return r;
}

// a[c] += P[K][c] me for all 16 registers (P[K][c] = a[c] in lane K).
template <int K> __device__ inline void fmac16_rowbcast(float a[16], float me)
{
    asm volatile("s_nop 1\n\t"
                 "v_fmac_f32_dpp %0, %0, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %1, %1, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %2, %2, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %3, %3, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %4, %4, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %5, %5, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %6, %6, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %7, %7, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %8, %8, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %9, %9, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %10, %10, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %11, %11, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %12, %12, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %13, %13, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %14, %14, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %15, %15, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf"
                 : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5]), "+v"(a[6]), "+v"(a[7]),
                   "+v"(a[8]), "+v"(a[9]), "+v"(a[10]), "+v"(a[11]), "+v"(a[12]), "+v"(a[13]), "+v"(a[14]), "+v"(a[15])
                 : "v"(me), "i"(K));
}

// a[c] *= bv_c, with bv_c the value of bv in lane c of the 16-lane row.
__device__ inline void scale16_colbcast(float a[16], float bv)
{
    asm volatile("s_nop 1\n\t"
                 "v_mul_f32_dpp %0, %16, %0 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\t"
                 "v_mul_f32_dpp %1, %16, %1 row_newbcast:1 row_mask:0xf bank_mask:0xf\n\t"
                 "v_mul_f32_dpp %2, %16, %2 row_newbcast:2 row_mask:0xf bank_mask:0xf\n\t"
                 "v_mul_f32_dpp %3, %16, %3 row_newbcast:3 row_mask:0xf bank_mask:0xf\n\t"
                 "v_mul_f32_dpp %4, %16, %4 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
                 "v_mul_f32_dpp %5, %16, %5 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\t"
                 "v_mul_f32_dpp %6, %16, %6 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\t"
                 "v_mul_f32_dpp %7, %16, %7 row_newbcast:7 row_mask:0xf bank_mask:0xf\n\t"
                 "v_mul_f32_dpp %8, %16, %8 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\t"
                 "v_mul_f32_dpp %9, %16, %9 row_newbcast:9 row_mask:0xf bank_mask:0xf\n\t"
                 "v_mul_f32_dpp %10, %16, %10 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\t"
                 "v_mul_f32_dpp %11, %16, %11 row_newbcast:11 row_mask:0xf bank_mask:0xf\n\t"
                 "v_mul_f32_dpp %12, %16, %12 row_newbcast:12 row_mask:0xf bank_mask:0xf\n\t"
                 "v_mul_f32_dpp %13, %16, %13 row_newbcast:13 row_mask:0xf bank_mask:0xf\n\t"
                 "v_mul_f32_dpp %14, %16, %14 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\t"
                 "v_mul_f32_dpp %15, %16, %15 row_newbcast:15 row_mask:0xf bank_mask:0xf"
                 : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5]), "+v"(a[6]), "+v"(a[7]),
                   "+v"(a[8]), "+v"(a[9]), "+v"(a[10]), "+v"(a[11]), "+v"(a[12]), "+v"(a[13]), "+v"(a[14]), "+v"(a[15])
                 : "v"(bv));
}

// acc + sum_c f[c] gv_c, with gv_c the value of gv in lane c of the 16-lane
// row (the sum in column order; operand 0 is acc, 1..16 are f, 17 is gv).
__device__ inline float dot16_colbcast(const float f[16], float gv, float acc)
{
    asm volatile("s_nop 1\n\t"
                 "v_fmac_f32_dpp %0, %17, %1 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %0, %17, %2 row_newbcast:1 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %0, %17, %3 row_newbcast:2 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %0, %17, %4 row_newbcast:3 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %0, %17, %5 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %0, %17, %6 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %0, %17, %7 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %0, %17, %8 row_newbcast:7 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %0, %17, %9 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %0, %17, %10 row_newbcast:9 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %0, %17, %11 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %0, %17, %12 row_newbcast:11 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %0, %17, %13 row_newbcast:12 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %0, %17, %14 row_newbcast:13 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %0, %17, %15 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f32_dpp %0, %17, %16 row_newbcast:15 row_mask:0xf bank_mask:0xf"
                 : "+v"(acc)
                 : "v"(f[0]), "v"(f[1]), "v"(f[2]), "v"(f[3]), "v"(f[4]), "v"(f[5]), "v"(f[6]), "v"(f[7]),
                   "v"(f[8]), "v"(f[9]), "v"(f[10]), "v"(f[11]), "v"(f[12]), "v"(f[13]), "v"(f[14]), "v"(f[15]),
                   "v"(gv));
    return acc;
}

// FP64 forms of the row helpers: v_fmac_f64 takes the row broadcast as its DPP
// operand; the 64-bit multiply has no DPP form, so the column scaling of the
// Schur complement is folded into an FMA (see form_schur16).
template <int K> __device__ inline double rowbcast_w(double v)
{
    double r;
    asm volatile("s_nop 1\n\tv_mov_b64_dpp %0, %1 row_newbcast:%c2 row_mask:0xf bank_mask:0xf"
                 : "=v"(r)
                 : "v"(v), "i"(K));
    return r;
}
template <int K> __device__ inline void fmac16_rowbcast(double a[16], double me)
{
    asm volatile("s_nop 1\n\t"
                 "v_fmac_f64_dpp %0, %0, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %1, %1, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %2, %2, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %3, %3, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %4, %4, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %5, %5, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %6, %6, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %7, %7, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %8, %8, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %9, %9, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %10, %10, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %11, %11, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %12, %12, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %13, %13, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %14, %14, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %15, %15, %16 row_newbcast:%c17 row_mask:0xf bank_mask:0xf"
                 : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5]), "+v"(a[6]), "+v"(a[7]),
                   "+v"(a[8]), "+v"(a[9]), "+v"(a[10]), "+v"(a[11]), "+v"(a[12]), "+v"(a[13]), "+v"(a[14]), "+v"(a[15])
                 : "v"(me), "i"(K));
}
__device__ inline double dot16_colbcast(const double f[16], double gv, double acc)
{
    asm volatile("s_nop 1\n\t"
                 "v_fmac_f64_dpp %0, %17, %1 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %0, %17, %2 row_newbcast:1 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %0, %17, %3 row_newbcast:2 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %0, %17, %4 row_newbcast:3 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %0, %17, %5 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %0, %17, %6 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %0, %17, %7 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %0, %17, %8 row_newbcast:7 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %0, %17, %9 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %0, %17, %10 row_newbcast:9 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %0, %17, %11 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %0, %17, %12 row_newbcast:11 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %0, %17, %13 row_newbcast:12 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %0, %17, %14 row_newbcast:13 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %0, %17, %15 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %0, %17, %16 row_newbcast:15 row_mask:0xf bank_mask:0xf"
                 : "+v"(acc)
                 : "v"(f[0]), "v"(f[1]), "v"(f[2]), "v"(f[3]), "v"(f[4]), "v"(f[5]), "v"(f[6]), "v"(f[7]),
                   "v"(f[8]), "v"(f[9]), "v"(f[10]), "v"(f[11]), "v"(f[12]), "v"(f[13]), "v"(f[14]), "v"(f[15]),
                   "v"(gv));
    return acc;
}
// t[c] += bv_c u[c] for c in [8 H, 8 H + 8), bv_c the value of bv in lane c of
// the 16-lane row (operands: t 0..7, bv 16, u 8..15)
__device__ inline void fma8_colbcast_lo(double t[8], const double u[8], double bv)
{
    asm volatile("s_nop 1\n\t"
                 "v_fmac_f64_dpp %0, %16, %8 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %1, %16, %9 row_newbcast:1 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %2, %16, %10 row_newbcast:2 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %3, %16, %11 row_newbcast:3 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %4, %16, %12 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %5, %16, %13 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %6, %16, %14 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %7, %16, %15 row_newbcast:7 row_mask:0xf bank_mask:0xf"
                 : "+v"(t[0]), "+v"(t[1]), "+v"(t[2]), "+v"(t[3]), "+v"(t[4]), "+v"(t[5]), "+v"(t[6]), "+v"(t[7])
                 : "v"(u[0]), "v"(u[1]), "v"(u[2]), "v"(u[3]), "v"(u[4]), "v"(u[5]), "v"(u[6]), "v"(u[7]),
                   "v"(bv));
}
__device__ inline void fma8_colbcast_hi(double t[8], const double u[8], double bv)
{
    asm volatile("s_nop 1\n\t"
                 "v_fmac_f64_dpp %0, %16, %8 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %1, %16, %9 row_newbcast:9 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %2, %16, %10 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %3, %16, %11 row_newbcast:11 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %4, %16, %12 row_newbcast:12 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %5, %16, %13 row_newbcast:13 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %6, %16, %14 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\t"
                 "v_fmac_f64_dpp %7, %16, %15 row_newbcast:15 row_mask:0xf bank_mask:0xf"
                 : "+v"(t[0]), "+v"(t[1]), "+v"(t[2]), "+v"(t[3]), "+v"(t[4]), "+v"(t[5]), "+v"(t[6]), "+v"(t[7])
                 : "v"(u[0]), "v"(u[1]), "v"(u[2]), "v"(u[3]), "v"(u[4]), "v"(u[5]), "v"(u[6]), "v"(u[7]),
                   "v"(bv));
}

// Entry c of row i of T_j (unit diagonal, gamma_j[c] at (c + 1, c) and
// (c, c + 1)): gf = gamma_j[i], gl = gamma_j[i - 1].
template <typename T>
__device__ inline T tri_entry(int c, int i, T gf, T gl)
{
    T tv = (c == i + 1) ? gf : (T)0;
    tv = (c + 1 == i) ? gl : tv;
    return (c == i) ? (T)1 : tv;
}
// C_j = T_j + diag(beta_j) (-C_{j-1}^{-1}) diag(beta_j), row i per lane.
__device__ inline void form_schur16(float a[16], float bf, float gf, float gl, int i)
{
    scale16_colbcast(a, bf);
#pragma unroll
    for (int c = 0; c < 16; ++c) a[c] = fmaf(bf, a[c], tri_entry(c, i, gf, gl));
}
__device__ inline void form_schur16(double a[16], double bf, double gf, double gl, int i)
{
    double t[16], u[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        t[c] = tri_entry(c, i, gf, gl);
        u[c] = bf * a[c];
    }
    fma8_colbcast_lo(t, u, bf);
    fma8_colbcast_hi(t + 8, u + 8, bf);
#pragma unroll
    for (int c = 0; c < 16; ++c) a[c] = t[c];
}

template <typename T, int K>
__device__ inline void sweep_row_step(T a[16], int i, bool &ok)
{
    const T d = rowbcast_w<K>(a[K]);  // P[K][K]
    ok = ok && (d > (T)0) && isfinite(d);
    const T inv = recip(d), f = a[K] * inv;
    const bool piv = (i == K);
    // rows i != K: P[i][c] - f P[K][c]; row K: P[K][c] / d (as in sweep_step)
    const T me = piv ? inv - (T)1 : -f;
    const T colK = piv ? -inv : f;
    fmac16_rowbcast<K>(a, me);
    a[K] = colK;
}

// -P^{-1} of the 16 x 16 SPD block held one row per lane (see above).
template <typename T>
__device__ inline bool sweep16_rows(T a[16], int i)
{
    bool ok = true;
    sweep_row_step<T, 0>(a, i, ok);
    sweep_row_step<T, 1>(a, i, ok);
    sweep_row_step<T, 2>(a, i, ok);
    sweep_row_step<T, 3>(a, i, ok);
    sweep_row_step<T, 4>(a, i, ok);
    sweep_row_step<T, 5>(a, i, ok);
    sweep_row_step<T, 6>(a, i, ok);
    sweep_row_step<T, 7>(a, i, ok);
    sweep_row_step<T, 8>(a, i, ok);
    sweep_row_step<T, 9>(a, i, ok);
    sweep_row_step<T, 10>(a, i, ok);
    sweep_row_step<T, 11>(a, i, ok);
    sweep_row_step<T, 12>(a, i, ok);
    sweep_row_step<T, 13>(a, i, ok);
    sweep_row_step<T, 14>(a, i, ok);
    sweep_row_step<T, 15>(a, i, ok);
    return ok;
}

// Value of lane i - 1 of the 16-lane row (0 in lane 0).
__device__ inline float row_shr1(float v) { return dpp_f32<0x111>(v); }
__device__ inline double row_shr1(double v) { return dpp_f64<0x111>(v); }

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
// by the grid.
template <typename Tst, bool STRIDE>
__global__ __launch_bounds__(256) void k_factor_rows16(int S, const double *__restrict__ a,
                                                       double *__restrict__ sc, double *__restrict__ beta,
                                                       Tst *__restrict__ factor,
                                                       const int *__restrict__ idx,
                                                       const int *__restrict__ count,
                                                       int64_t slot_base, uint32_t *__restrict__ state,
                                                       double frhs, double *__restrict__ fz,
                                                       double *__restrict__ x0, int disc)
{
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
// every factor type.
template <typename Tst, bool STRIDE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ir_rows_waves<Tst>()))) void k_ir_rows16(
    int S, double fconst, const double *__restrict__ a, const double *__restrict__ sc,
    const double *__restrict__ beta, const Tst *__restrict__ factor, double *__restrict__ x,
    const double *__restrict__ zbuf, double eps, int imax, int direct, const int *__restrict__ idx,
    const int *__restrict__ count, int64_t slot_base, uint32_t *__restrict__ state,
    double *__restrict__ relres, double *__restrict__ q, int32_t *__restrict__ iters, int fwd_done, int disc)
{
    using Tac = typename store_traits<Tst>::acc;
    constexpr int M = 16, m = M - 1, NP = M + 1;
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
template <typename Tst, int M, int G, bool PREF>
__global__ __launch_bounds__((64 * blk_waves<M, G>())) __attribute__((amdgpu_waves_per_eu(ir_min_waves<Tst, M, G>()))) void k_ir_blk(
    int n, double fconst, const double *__restrict__ a, const double *__restrict__ sc,
    const double *__restrict__ beta, const Tst *__restrict__ factor, double *__restrict__ x,
    double *__restrict__ r, double *__restrict__ zbuf, double eps, int imax, int direct,
    const int *__restrict__ idx, const int *__restrict__ count, int64_t slot_base,
    uint32_t *__restrict__ state, double *__restrict__ relres, double *__restrict__ q,
    int32_t *__restrict__ iters, int fwd_done, int disc)
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
    solve_blk_pass<Tst, M, G, PREF>(scs, bs, fs, nullptr, h * h * fconst, xs, 0, zs, fwd_done != 0);
    uint32_t st = state[s] & ~(uint32_t)ST_DONE;
    double prev = INFINITY, rel = INFINITY, sx = 0.0;
    int trip = 0;
    for (;;) {
        __syncthreads();
        const resid_out o = residual_pass_m<NT, M>(fconst, as, xs, rsb, red, disc);
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
// Solve configuration: waves per row pair (G) and register double-buffering
// of the next Schur block (PREF), within the register budget.
template <typename Tst, int M> struct solve_cfg { static constexpr int G = 1; static constexpr bool PREF = true; };
template <typename Tst> struct solve_cfg<Tst, 128> { static constexpr int G = 2; static constexpr bool PREF = true; };
template <typename Tst> struct solve_cfg<Tst, 256> { static constexpr int G = 2; static constexpr bool PREF = true; };
template <> struct solve_cfg<double, 64> { static constexpr int G = 2; static constexpr bool PREF = true; };
template <> struct solve_cfg<double, 128> { static constexpr int G = 2; static constexpr bool PREF = true; };
template <> struct solve_cfg<double, 256> { static constexpr int G = 1; static constexpr bool PREF = false; };

template <typename Tst, int M>
hipError_t lf(int nb, const double *a, double *sc, double *beta, const double *gam, void *factor,
              const int *idx, const int *count, int64_t slot_base, uint32_t *state, double frhs,
              double *fz, double *x0, int disc, int variant, hipStream_t st)
{
    if constexpr (M == 16) {
        if (nb == 0) return hipSuccess;
        const unsigned grid = (unsigned)((nb + 15) / 16);
        if (idx)
            hipLaunchKernelGGL((k_factor_rows16<Tst, true>), dim3(grid < 1024 ? grid : 1024), dim3(256), 0, st, nb,
                               a, sc, beta, (Tst *)factor, idx, count, slot_base, state, frhs, fz, x0, disc);
        else
            hipLaunchKernelGGL((k_factor_rows16<Tst, false>), dim3(grid), dim3(256), 0, st, nb, a, sc, beta,
                               (Tst *)factor, idx, count, slot_base, state, frhs, fz, x0, disc);
    } else if (variant == 1 && mfma_in_storage<Tst>()) {
        hipLaunchKernelGGL((k_factor_mfma<Tst, M, false>), dim3(nb), dim3(64 * blk_waves<M, 1>()), 0, st, nb, beta,
                           gam, (Tst *)factor, idx, count, slot_base, state, sc, frhs, fz);
    } else {
        hipLaunchKernelGGL((k_factor_mfma<Tst, M>), dim3(nb), dim3(64 * blk_waves<M, 1>()), 0, st, nb, beta, gam,
                           (Tst *)factor, idx, count, slot_base, state, sc, frhs, fz);
    }
    return hipGetLastError();
}


// Refinement kernel variants: G waves per block-row pair (1 or 2); the FP64
// n = 256 variant keeps no register double-buffer (register budget).
template <typename Tst, int M, int G> struct ir_pref { static constexpr bool v = true; };
template <int G> struct ir_pref<double, 256, G> { static constexpr bool v = false; };

template <typename Tst, int M, int G>
hipError_t li_g(const ir_args &g, hipStream_t st)
{
    constexpr bool PREF = ir_pref<Tst, M, G>::v;
    hipLaunchKernelGGL((k_ir_blk<Tst, M, G, PREF>), dim3(g.nblocks), dim3(64 * blk_waves<M, G>()), 0, st, g.n,
                       g.fconst, g.a, g.sc, g.beta, (const Tst *)g.factor, g.x, g.r, g.z, g.eps,
                       g.imax, g.direct, g.idx, g.count, g.slot_base, g.state, g.relres, g.q, g.iters,
                       g.fwd_done, g.disc);
    return hipGetLastError();
}

template <typename Tst, int M>
hipError_t li(const ir_args &g, hipStream_t st)
{
    if constexpr (M == 16) {
        if (g.nblocks == 0) return hipSuccess;
        const unsigned grid = (unsigned)((g.nblocks + 15) / 16);
        if (g.idx)
            hipLaunchKernelGGL((k_ir_rows16<Tst, true>), dim3(grid < 1024 ? grid : 1024), dim3(256), 0, st,
                               g.nblocks, g.fconst, g.a, g.sc, g.beta, (const Tst *)g.factor, g.x, g.z, g.eps,
                               g.imax, g.direct, g.idx, g.count, g.slot_base, g.state, g.relres, g.q, g.iters,
                               g.fwd_done, g.disc);
        else
            hipLaunchKernelGGL((k_ir_rows16<Tst, false>), dim3(grid), dim3(256), 0, st,
                               g.nblocks, g.fconst, g.a, g.sc, g.beta, (const Tst *)g.factor, g.x, g.z, g.eps,
                               g.imax, g.direct, g.idx, g.count, g.slot_base, g.state, g.relres, g.q, g.iters,
                               g.fwd_done, g.disc);
        return hipGetLastError();
    } else {
        int G = g.variant > 0 ? g.variant : solve_cfg<Tst, M>::G;
        return G == 2 ? li_g<Tst, M, 2>(g, st) : li_g<Tst, M, 1>(g, st);
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
