// kernels_common.h -- small device helpers shared by the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace fmm {

constexpr int kBinomStride = 64;   // binomial table C(n, k), k < 64, row-major
constexpr int kBinomRows = 128;    // n < 128: M2L reads C(k + l, k) with k, l < p <= 64

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Workgroups are handed to the 8 XCDs of the chip in turn (workgroup b to
// XCD b mod 8).  This maps them so that each XCD runs one contiguous range of
// the launch: neighbouring work items (nearby boxes) then share that XCD's L2.
__device__ __forceinline__ int xcd_block()
{
    const int G = (int)gridDim.x, b = (int)blockIdx.x;
    const int x = b & 7, i = b >> 3, full = G >> 3, rem = G & 7;
    return x < rem ? x * (full + 1) + i : rem * (full + 1) + (x - rem) * full + i;
}

// orders the LDS accesses of one wavefront (no workgroup barrier)
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

// Sum v[0..V) over the NL lanes of each aligned lane group (lanes that
// differ in bits [0, log2 NL)), halving the values a lane keeps at every
// step: afterwards lane l holds the totals of the value indices
// treduce_base<V, NL>(l) + i, i < max(V / NL, 1).  When V < NL the last
// steps are plain sums, and NL / V lanes (differing in their low bits) hold
// the same total.

// one step with lane mask M while NV values are live (compile-time indices)
template <class T, int V, int NV, int M>
struct TStep {
    static __device__ __forceinline__ void run(T (&v)[V], int lane)
    {
        if (NV > 1) {
            constexpr int H = NV > 1 ? NV / 2 : 1;
            const bool hi = (lane & M) != 0;
#pragma unroll
            for (int i = 0; i < H; ++i) {
                const T keep = hi ? v[i + H] : v[i];
                const T send = hi ? v[i] : v[i + H];
                v[i] = keep + __shfl_xor(send, M, 64);
            }
        } else {
            v[0] += __shfl_xor(v[0], M, 64);
        }
        TStep<T, V, (NV > 1 ? NV / 2 : 1), M / 2>::run(v, lane);
    }
};
template <class T, int V, int NV>
struct TStep<T, V, NV, 0> {
    static __device__ __forceinline__ void run(T (&)[V], int) {}
};

template <int V, int NL, class T>
__device__ __forceinline__ void treduce(T (&v)[V], int lane)
{
    TStep<T, V, V, NL / 2>::run(v, lane);
}

template <int V, int NL>
__device__ __forceinline__ int treduce_base(int lane)
{
    int base = 0, nv = V;
#pragma unroll
    for (int m = NL / 2; m >= 1; m >>= 1) {
        if (nv > 1) {
            nv /= 2;
            if (lane & m) base += nv;
        }
    }
    return base;
}

}  // namespace fmm
