// Storage-type traits for the factor: FP64, FP32, BF16, FP16.
// Arithmetic is FP64 for the FP64 factor and FP32 for the others.
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
