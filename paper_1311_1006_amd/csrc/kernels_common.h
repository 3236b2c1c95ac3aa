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

// ---- exchanges inside a wavefront without LDS: DPP lane permutations
// inside rows of 16 lanes, and the gfx950 row swaps between rows
constexpr int kDppXor1 = 0xB1;        // lane ^ 1 (quad permutation 1, 0, 3, 2)
constexpr int kDppXor2 = 0x4E;        // lane ^ 2 (quad permutation 2, 3, 0, 1)
constexpr int kDppHalfMirror = 0x141; // lane 7 - l inside each half row
constexpr int kDppMirror = 0x140;     // lane 15 - l inside each row
constexpr int kDppShr1 = 0x111, kDppShr2 = 0x112, kDppShr4 = 0x114, kDppShr8 = 0x118;   // lane l - k in the row

// the value of the lane CTRL names; 0 where that lane lies outside the row
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// The row swaps of a double: rows 0 and 1 (2 and 3) exchanged, or rows 0, 1
// and 2, 3.  With both operands the value itself, the first result holds
// the value of the lower row of each pair in both rows, the second that of
// the upper row, so combining the two results combines the row pair.
__device__ __forceinline__ void row_swap16(double x, double& a, double& b)
{
    const long long v = __double_as_longlong(x);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(v >> 32), (unsigned)(v >> 32), false, false);
    a = __longlong_as_double(((long long)hi[0] << 32) | lo[0]);
    b = __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
}
__device__ __forceinline__ void row_swap32(double x, double& a, double& b)
{
    const long long v = __double_as_longlong(x);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(v >> 32), (unsigned)(v >> 32), false, false);
    a = __longlong_as_double(((long long)hi[0] << 32) | lo[0]);
    b = __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
}

// minimum / maximum of x over each half of the wavefront (lanes 0-31 and
// 32-63), in every lane of that half; fmin / fmax ignore a NaN operand
__device__ __forceinline__ double half_wave_min(double x)
{
    x = fmin(x, dpp_f64<kDppXor1>(x));
    x = fmin(x, dpp_f64<kDppXor2>(x));
    x = fmin(x, dpp_f64<kDppHalfMirror>(x));
    x = fmin(x, dpp_f64<kDppMirror>(x));
    double a, b;
    row_swap16(x, a, b);
    return fmin(a, b);
}
__device__ __forceinline__ double half_wave_max(double x)
{
    x = fmax(x, dpp_f64<kDppXor1>(x));
    x = fmax(x, dpp_f64<kDppXor2>(x));
    x = fmax(x, dpp_f64<kDppHalfMirror>(x));
    x = fmax(x, dpp_f64<kDppMirror>(x));
    double a, b;
    row_swap16(x, a, b);
    return fmax(a, b);
}
// minimum / maximum of x over the wavefront, in every lane
__device__ __forceinline__ double wave_min(double x)
{
    double a, b;
    row_swap32(half_wave_min(x), a, b);
    return fmin(a, b);
}
__device__ __forceinline__ double wave_max(double x)
{
    double a, b;
    row_swap32(half_wave_max(x), a, b);
    return fmax(a, b);
}

__device__ __forceinline__ void row_swap16(int x, int& a, int& b)
{
    const auto r = __builtin_amdgcn_permlane16_swap((unsigned)x, (unsigned)x, false, false);
    a = (int)r[0];
    b = (int)r[1];
}
__device__ __forceinline__ void row_swap32(int x, int& a, int& b)
{
    const auto r = __builtin_amdgcn_permlane32_swap((unsigned)x, (unsigned)x, false, false);
    a = (int)r[0];
    b = (int)r[1];
}
__device__ __forceinline__ void row_swap16(float x, float& a, float& b)
{
    int ia, ib;
    row_swap16(__float_as_int(x), ia, ib);
    a = __int_as_float(ia);
    b = __int_as_float(ib);
}
__device__ __forceinline__ void row_swap32(float x, float& a, float& b)
{
    int ia, ib;
    row_swap32(__float_as_int(x), ia, ib);
    a = __int_as_float(ia);
    b = __int_as_float(ib);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_any(double x) { return dpp_f64<CTRL>(x); }
template <int CTRL>
__device__ __forceinline__ float dpp_any(float x) { return dpp_f32<CTRL>(x); }
template <int CTRL>
__device__ __forceinline__ int dpp_any(int x) { return dpp_i32<CTRL>(x); }

// The value of a partner lane whose bit M differs from this lane's and
// whose higher bits agree (its lower bits may differ): lane ^ 1, lane ^ 2,
// the half-row mirror (lane ^ 7), the row mirror (lane ^ 15), the other row
// of a row pair (lane ^ 16) and the other half wavefront (lane ^ 32).
// Butterflies over such partners combine every lane of an aligned group of
// 2M lanes exactly once.
template <int M, class T>
__device__ __forceinline__ T partner(T x)
{
    static_assert(M == 1 || M == 2 || M == 4 || M == 8 || M == 16 || M == 32, "lane distance");
    if constexpr (M == 1) return dpp_any<kDppXor1>(x);
    else if constexpr (M == 2) return dpp_any<kDppXor2>(x);
    else if constexpr (M == 4) return dpp_any<kDppHalfMirror>(x);
    else if constexpr (M == 8) return dpp_any<kDppMirror>(x);
    else {
        T a, b;
        if constexpr (M == 16) row_swap16(x, a, b);
        else row_swap32(x, a, b);
        return (threadIdx.x & M) ? a : b;
    }
}

// maximum of x over the wavefront, in every lane
__device__ __forceinline__ int wave_max_i32(int x)
{
    x = max(x, partner<1>(x));
    x = max(x, partner<2>(x));
    x = max(x, partner<4>(x));
    x = max(x, partner<8>(x));
    int a, b;
    row_swap16(x, a, b);
    x = max(a, b);
    row_swap32(x, a, b);
    return max(a, b);
}

// Segmented inclusive scan over the wavefront of pairs (h, v): a lane's h
// says a segment starts in it; (h1, v1) followed by (h2, v2) combine to
// (h1 | h2, h2 ? v2 : v1 + v2).  Shifts by 1, 2, 4, 8 inside every row, then
// each row takes the combination of the rows before it.  eh, ev receive the
// exclusive values (those of the previous lane; (0, 0) in lane 0).
__device__ __forceinline__ void seg_combine(int hp, int vp, int& h, int& v)
{
    v = h ? v : vp + v;
    h |= hp;
}
__device__ __forceinline__ void wave_seg_scan(int& h, int& v, int& eh, int& ev)
{
    seg_combine(dpp_i32<kDppShr1>(h), dpp_i32<kDppShr1>(v), h, v);
    seg_combine(dpp_i32<kDppShr2>(h), dpp_i32<kDppShr2>(v), h, v);
    seg_combine(dpp_i32<kDppShr4>(h), dpp_i32<kDppShr4>(v), h, v);
    seg_combine(dpp_i32<kDppShr8>(h), dpp_i32<kDppShr8>(v), h, v);
    const int h0 = __builtin_amdgcn_readlane(h, 15), v0 = __builtin_amdgcn_readlane(v, 15);
    const int h1 = __builtin_amdgcn_readlane(h, 31), v1 = __builtin_amdgcn_readlane(v, 31);
    const int h2 = __builtin_amdgcn_readlane(h, 47), v2 = __builtin_amdgcn_readlane(v, 47);
    // the rows before row 1, 2, 3 combined
    int ch1 = h0, cv1 = v0;
    int ch2 = h1, cv2 = v1;
    seg_combine(ch1, cv1, ch2, cv2);
    int ch3 = h2, cv3 = v2;
    seg_combine(ch2, cv2, ch3, cv3);
    const int row = (int)(threadIdx.x & 63) >> 4;
    const int ch = row == 0 ? 0 : row == 1 ? ch1 : row == 2 ? ch2 : ch3;
    const int cv = row == 0 ? 0 : row == 1 ? cv1 : row == 2 ? cv2 : cv3;
    if (row > 0) seg_combine(ch, cv, h, v);
    // the previous lane's inclusive values; the first lane of a row takes
    // the combination of the rows before it
    eh = __builtin_amdgcn_update_dpp(ch, h, kDppShr1, 0xF, 0xF, false);
    ev = __builtin_amdgcn_update_dpp(cv, v, kDppShr1, 0xF, 0xF, false);
}

// inclusive prefix sum of x over the lanes of the wavefront: shifts by 1,
// 2, 4, 8 inside every row, then each row adds the totals of the rows
// before it (read from lanes 15, 31, 47)
__device__ __forceinline__ int wave_incl_scan(int x)
{
    x += dpp_i32<kDppShr1>(x);
    x += dpp_i32<kDppShr2>(x);
    x += dpp_i32<kDppShr4>(x);
    x += dpp_i32<kDppShr8>(x);
    const int t0 = __builtin_amdgcn_readlane(x, 15);
    const int t1 = __builtin_amdgcn_readlane(x, 31);
    const int t2 = __builtin_amdgcn_readlane(x, 47);
    const int row = (int)(threadIdx.x & 63) >> 4;
    return x + (row == 0 ? 0 : row == 1 ? t0 : row == 2 ? t0 + t1 : t0 + t1 + t2);
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
                v[i] = keep + partner<M>(send);
            }
        } else {
            v[0] += partner<M>(v[0]);
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
