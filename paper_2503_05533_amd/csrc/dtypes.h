// Storage-type traits for the factor: FP64, FP32, BF16, FP16, FP8 (E4M3).
// Loads and stores convert to the arithmetic type: FP64 for the FP64 factor,
// FP32 for the others (the MFMA kernels multiply FP16/BF16 operands in
// their own precision, with FP32 accumulation).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace mlmc {

template <typename S> struct store_traits;

template <> struct store_traits<double> {
    using acc = double;
    __device__ static inline double load(double v) { return v; }
    __device__ static inline double store(double v) { return v; }
};
template <> struct store_traits<float> {
    using acc = float;
    __device__ static inline float load(float v) { return v; }
    __device__ static inline float store(float v) { return v; }
};
template <> struct store_traits<__hip_bfloat16> {
    using acc = float;
    __device__ static inline float load(__hip_bfloat16 v) { return __bfloat162float(v); }
    __device__ static inline __hip_bfloat16 store(float v) { return __float2bfloat16(v); }
};
template <> struct store_traits<__half> {
    using acc = float;
    __device__ static inline float load(__half v) { return __half2float(v); }
    __device__ static inline __half store(float v) { return __float2half(v); }
};

// FP8 E4M3 storage (sign, 4 exponent bits, 3 significand bits: the
// quarter-precision format q43 of Sec. 2.1, unit roundoff 2^-4, largest
// finite value 448), converted by the hardware with round to nearest even.
struct fp8e4m3 { uint8_t bits; };
template <> struct store_traits<fp8e4m3> {
    using acc = float;
    __device__ static inline float load(fp8e4m3 v) { return __builtin_amdgcn_cvt_f32_fp8((int)v.bits, 0); }
    __device__ static inline fp8e4m3 store(float v)
    {
        return fp8e4m3{(uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false) & 0xff)};
    }
};

// 1/d from the hardware reciprocal refined by Newton steps (one for FP32,
// two for FP64: relative error at the unit roundoff).
__device__ inline float recip(float d)
{
    float r = __builtin_amdgcn_rcpf(d);
    return fmaf(r, fmaf(-d, r, 1.0f), r);
}
__device__ inline double recip(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    return fma(r, fma(-d, r, 1.0), r);
}

}  // namespace mlmc
