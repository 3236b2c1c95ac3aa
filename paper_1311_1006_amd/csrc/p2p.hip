// p2p.hip -- near-field direct sums over the finest-level strong lists
// (Sec. 2.1: pairs not accounted for by M2L shifts are evaluated directly;
// Sec. 3.1: both G(x_i,x_j) and G(x_j,x_i) are computed, so there is no
// write conflict and the result is deterministic).
//
//     phi_i += sum_{S in strong(leaf(i))} sum_{j in S, z_j != z_i} m_j / (z_i - z_j)
//
// One wavefront per work item (a leaf, or a chunk of a large leaf's targets).
// The 64 lanes are TW = 64/NS target slots times NS source splits: lane
// (t, s) owns targets t, t+TW, ... (R of them in registers) and the sources
// j = s, s+NS, ... of every leaf in the strong list; a butterfly over the NS
// splits combines the partial sums.  Leaves at the optimum hold 15-60 points,
// fewer than 64 lanes, hence the source split.  Exclusion by position: a pair
// with z_j = z_i has r^2 = 0 and its reciprocal is clamped to the largest
// finite value, which multiplies an exact zero.
//   FP64:  dz in FP64, 1/r^2 by v_rcp_f64 and two Newton steps.
//   mixed: positions stored as FP32 hi + lo, dz = (hi_i - hi_j) + (lo_i - lo_j),
//          everything else in FP32, FP32 accumulation.
#include <cfloat>

#include "fmm_internal.h"

namespace fmm {

struct P2PItem {
    int32_t leaf, t0, tn, pad;
};

__device__ __forceinline__ void pair64(double xi, double yi, const double4& s, double& ar, double& ai)
{
    double dx = xi - s.x, dy = yi - s.y;
    double r2 = fma(dx, dx, dy * dy);
    double y = __builtin_amdgcn_rcp(r2);
    double e = fma(-r2, y, 1.0);
    y = fma(y, e, y);
    e = fma(-r2, y, 1.0);
    y = fma(y, e, y);
    y = fmin(y, DBL_MAX);
    double a = fma(s.z, dx, s.w * dy);
    double b = fma(s.w, dx, -(s.z * dy));
    ar = fma(a, y, ar);
    ai = fma(b, y, ai);
}

__device__ __forceinline__ void pair32(float xh, float yh, float xl, float yl, const float4& s, const float2& l,
                                       float& ar, float& ai)
{
    float dx = (xh - s.x) + (xl - l.x);
    float dy = (yh - s.y) + (yl - l.y);
    float r2 = fmaf(dx, dx, dy * dy);
    float y = fminf(__builtin_amdgcn_rcpf(r2), FLT_MAX);
    float a = fmaf(s.z, dx, s.w * dy);
    float b = fmaf(s.w, dx, -(s.z * dy));
    ar = fmaf(a, y, ar);
    ai = fmaf(b, y, ai);
}

template <int NS, int R>
__global__ void __launch_bounds__(64)
k_p2p64(const P2PItem* __restrict__ items, const int32_t* __restrict__ bstart, const int32_t* __restrict__ bcount,
        const int32_t* __restrict__ s_beg, const int32_t* __restrict__ s_cnt, const int32_t* __restrict__ s_ids,
        const double4* __restrict__ src, double2* __restrict__ out)
{
    constexpr int TW = 64 / NS;
    const P2PItem it = items[blockIdx.x];
    const int lane = threadIdx.x, t = lane % TW, sp = lane / TW;
    const int base = bstart[it.leaf] + it.t0;
    double xi[R], yi[R], ar[R], ai[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int k = t + TW * r;
        double4 v = src[base + (k < it.tn ? k : 0)];
        xi[r] = v.x; yi[r] = v.y; ar[r] = 0.0; ai[r] = 0.0;
    }
    const int e0 = s_beg[it.leaf], ne = s_cnt[it.leaf];
    for (int e = 0; e < ne; ++e) {
        const int S = s_ids[e0 + e];
        const int j0 = bstart[S], nj = bcount[S];
#pragma unroll 4
        for (int j = sp; j < nj; j += NS) {
            const double4 s = src[j0 + j];
#pragma unroll
            for (int r = 0; r < R; ++r) pair64(xi[r], yi[r], s, ar[r], ai[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int o = TW; o < 64; o <<= 1) {
            ar[r] += __shfl_xor(ar[r], o, 64);
            ai[r] += __shfl_xor(ai[r], o, 64);
        }
        int k = t + TW * r;
        if (sp == 0 && k < it.tn) out[base + k] = make_double2(ar[r], ai[r]);
    }
}

template <int NS, int R>
__global__ void __launch_bounds__(64)
k_p2p32(const P2PItem* __restrict__ items, const int32_t* __restrict__ bstart, const int32_t* __restrict__ bcount,
        const int32_t* __restrict__ s_beg, const int32_t* __restrict__ s_cnt, const int32_t* __restrict__ s_ids,
        const float4* __restrict__ src, const float2* __restrict__ lo, double2* __restrict__ out)
{
    constexpr int TW = 64 / NS;
    const P2PItem it = items[blockIdx.x];
    const int lane = threadIdx.x, t = lane % TW, sp = lane / TW;
    const int base = bstart[it.leaf] + it.t0;
    float xh[R], yh[R], xl[R], yl[R], ar[R], ai[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int k = t + TW * r;
        int i = base + (k < it.tn ? k : 0);
        float4 v = src[i];
        float2 w = lo[i];
        xh[r] = v.x; yh[r] = v.y; xl[r] = w.x; yl[r] = w.y; ar[r] = 0.f; ai[r] = 0.f;
    }
    const int e0 = s_beg[it.leaf], ne = s_cnt[it.leaf];
    for (int e = 0; e < ne; ++e) {
        const int S = s_ids[e0 + e];
        const int j0 = bstart[S], nj = bcount[S];
#pragma unroll 4
        for (int j = sp; j < nj; j += NS) {
            const float4 s = src[j0 + j];
            const float2 l = lo[j0 + j];
#pragma unroll
            for (int r = 0; r < R; ++r) pair32(xh[r], yh[r], xl[r], yl[r], s, l, ar[r], ai[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int o = TW; o < 64; o <<= 1) {
            ar[r] += __shfl_xor(ar[r], o, 64);
            ai[r] += __shfl_xor(ai[r], o, 64);
        }
        int k = t + TW * r;
        if (sp == 0 && k < it.tn) out[base + k] = make_double2((double)ar[r], (double)ai[r]);
    }
}

template <int NS, int R>
static void launch_one(bool mixed, const P2PItem* items, int n, const int32_t* bstart, const int32_t* bcount,
                       const int32_t* s_beg, const int32_t* s_cnt, const int32_t* s_ids, const void* src,
                       const void* lo, double* out, hipStream_t s)
{
    if (mixed)
        k_p2p32<NS, R><<<n, 64, 0, s>>>(items, bstart, bcount, s_beg, s_cnt, s_ids, (const float4*)src,
                                       (const float2*)lo, (double2*)out);
    else
        k_p2p64<NS, R><<<n, 64, 0, s>>>(items, bstart, bcount, s_beg, s_cnt, s_ids, (const double4*)src,
                                       (double2*)out);
}

// one launch per (NS, R) class
void launch_p2p(bool mixed, int ns, int r, const void* items, int n, const int32_t* bstart, const int32_t* bcount,
                const int32_t* s_beg, const int32_t* s_cnt, const int32_t* s_ids, const void* src, const void* lo,
                double* out, hipStream_t s)
{
    if (n == 0) return;
    const P2PItem* it = (const P2PItem*)items;
#define CASE(NS_, R_) \
    if (ns == NS_ && r == R_) { launch_one<NS_, R_>(mixed, it, n, bstart, bcount, s_beg, s_cnt, s_ids, src, lo, out, s); check_launch("p2p"); return; }
    CASE(1, 1) CASE(1, 2) CASE(1, 4)
    CASE(2, 1) CASE(2, 2) CASE(2, 4)
    CASE(4, 1) CASE(4, 2) CASE(4, 4)
    CASE(8, 1) CASE(8, 2) CASE(8, 4)
    CASE(16, 1) CASE(16, 2) CASE(16, 4)
#undef CASE
    throw Error(FMM_EINVAL, "unsupported P2P launch shape");
}

}  // namespace fmm
