// Device helpers of the block-layout factorisation and refinement kernels:
// MFMA wrappers, the stored-block layout, the slot map of blocks to waves,
// lane broadcasts and reductions, the 16-pivot sweep steps, and the
// one-row-per-lane pieces of the n = 16 kernels.
//
// Stored factor: per Schur block j, NBL = NB(NB+1)/2 lower blocks b (row by
// row), each in the MFMA result layout: entry (row drow(l/16, r), col l%16) of
// block b at offset (b*64 + l)*4 + r, so that a lane's four entries of a block
// are one contiguous vector access.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dtypes.h"
#include "kernels.h"

namespace mlmc {

#ifndef TWISTED_ON
#define TWISTED_ON 1
#endif

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

// Twisted (both-ends) elimination of the block layout: the block rows
// 0 .. k-1 are eliminated top-down and m-1 .. k+1 bottom-up (m = M - 1 is odd,
// k = (m - 1) / 2), each by a group of waves of one workgroup, and the middle
// block row k last; the stored block of row j is the inverse Schur
// complement of its chain (-C_j^{-1} above k, -D_j^{-1} below k) and of the
// middle, -E_k^{-1}.  Used where the two groups' LDS still lets two
// workgroups share a CU: the FP32-arithmetic factors up to M = 128, FP64 at
// M = 64 (Tac: the arithmetic type).
template <typename Tac, int M> constexpr bool twisted()
{
    return TWISTED_ON && M >= 32 && (sizeof(Tac) == 4 ? M <= 128 : M == 64);
}
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

}  // namespace mlmc
