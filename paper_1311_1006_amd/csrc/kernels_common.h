// kernels_common.h -- small device helpers shared by the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace fmm {

constexpr int kBinomStride = 64;   // binomial table C(n, k), n, k < 64, row-major

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <class T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

}  // namespace fmm
