// p2p.hip -- near-field direct sums over the finest-level strong lists
// (Sec. 2.1: pairs not accounted for by M2L shifts are evaluated directly;
// as in Sec. 3.1, a pair of neighbouring leaves is evaluated once from each
// side, each work item writing only its own targets: no two items write the
// same output and the result is deterministic).
//
//     phi_i += sum_{S in strong(leaf(i))} sum_{j in S, z_j != z_i} m_j / (z_i - z_j)
//
// One wavefront per work item (a leaf, or a group of a large leaf's
// targets).  The sources of all leaves in the strong list are first gathered
// into a contiguous LDS array (one coalesced pass).  The 64 lanes are SUB
// subgroups of NL = 64/SUB lanes: within a subgroup every lane owns one
// source of the current chunk and all TG targets of the subgroup (targets in
// registers), so the inner loop has no memory traffic: per pair only the
// kernel arithmetic.  Padding lanes carry zero strength.  A transposing
// butterfly then sums the 2*TG accumulators over the NL lanes with about
// 2*TG shuffles instead of 2*TG*log2(NL).
// Exclusion by position: r^2 is formed as dx^2 + (dy^2 + tiny) with tiny the
// smallest normal number, which leaves every r^2 of two distinct points
// unchanged and turns r^2 = 0 (z_j = z_i) into a finite reciprocal that
// multiplies an exact zero.
//   FP64:  dz in FP64, 1/r^2 by v_rcp_f64 and one Newton step.
//   mixed: positions in FP64, dz = z_i - z_j in FP64 rounded once to FP32
//          (FP64 adds issue at the FP32 rate on this chip: two instructions
//          per component, against three for a hi + lo FP32 pair), strengths
//          rounded to FP32 as they are staged, everything after dz in FP32
//          with FP32 accumulation.
#include <cfloat>
#include <climits>

#include "fmm_internal.h"
#include "kernels_common.h"
#include "p2p_common.h"

namespace fmm {

struct P2PItem {
    int32_t leaf, t0, tn, pad;
};

// Sources staged in LDS per pass and wavefront.  The buffer and the staging
// registers (a quarter of the buffer per lane) set how many wavefronts a
// SIMD holds, and with them how well the staging loads of one wavefront hide
// behind the arithmetic of the others: 128 for the mixed kernels (16 KiB per
// workgroup, 64 vector registers: 8 wavefronts per SIMD), 192 for FP64
// (29 KiB, 92 registers: 5).  At N = 1e6, N_levels 9 (a list of about 183
// sources) this took the mixed near field from 108 to 99 us and the FP64
// one from 162 to 155 us against a 256-source buffer.
constexpr int kP2PSrcCap32 = 128, kP2PSrcCap64 = 192;


struct Src64 {
    double x, y, mr, mi;
};
struct Src32 {
    double x, y;
    float mr, mi;
};

// 1/r^2 by v_rcp_f64 (relative error below 2^-24, a quarter-rate instruction
// on this chip) and one Newton step: below 2.3e-15 relative over inputs
// spanning 2^-100 .. 2^100 (a second step, two more FMAs per pair, reached
// the correctly rounded quotient)
__device__ __forceinline__ double rcp_pair(double r2)
{
    const double y = __builtin_amdgcn_rcp(r2);
    return fma(y, fma(-r2, y, 1.0), y);
}

__device__ __forceinline__ void pair64(double xi, double yi, const Src64& s, double& ar, double& ai)
{
    double dx = xi - s.x, dy = yi - s.y;
    double r2 = fma(dx, dx, fma(dy, dy, DBL_MIN));
    double y = rcp_pair(r2);
    double a = fma(s.mr, dx, s.mi * dy);
    double b = fma(s.mi, dx, -(s.mr * dy));
    ar = fma(a, y, ar);
    ai = fma(b, y, ai);
}

// the same terms times the Gaussian smoother 1 - exp(-r^2/delta^2) (id2 = 1/delta^2)
__device__ __forceinline__ void pair64s(double xi, double yi, const Src64& s, double id2, double& ar, double& ai)
{
    double dx = xi - s.x, dy = yi - s.y;
    double r2 = fma(dx, dx, fma(dy, dy, DBL_MIN));
    double y = rcp_pair(r2);
    y *= 1.0 - exp(-r2 * id2);
    double a = fma(s.mr, dx, s.mi * dy);
    double b = fma(s.mi, dx, -(s.mr * dy));
    ar = fma(a, y, ar);
    ai = fma(b, y, ai);
}

__device__ __forceinline__ void pair32(double xi, double yi, const Src32& s, float& ar, float& ai)
{
    float dx = (float)(xi - s.x);
    float dy = (float)(yi - s.y);
    float r2 = fmaf(dx, dx, fmaf(dy, dy, FLT_MIN));
    float y = __builtin_amdgcn_rcpf(r2);
    float a = fmaf(s.mr, dx, s.mi * dy);
    float b = fmaf(s.mi, dx, -(s.mr * dy));
    ar = fmaf(a, y, ar);
    ai = fmaf(b, y, ai);
}

__device__ __forceinline__ void pair32s(double xi, double yi, const Src32& s, float id2, float& ar, float& ai)
{
    float dx = (float)(xi - s.x);
    float dy = (float)(yi - s.y);
    float r2 = fmaf(dx, dx, fmaf(dy, dy, FLT_MIN));
    float y = __builtin_amdgcn_rcpf(r2) * (1.0f - __expf(-r2 * id2));
    float a = fmaf(s.mr, dx, s.mi * dy);
    float b = fmaf(s.mi, dx, -(s.mr * dy));
    ar = fmaf(a, y, ar);
    ai = fmaf(b, y, ai);
}

// The logarithmic kernel: log|z_i - z_j| times the real and the imaginary
// part of the strength (real strengths leave the second sum 0).  Coincident
// positions are left out, as in the other kernels; FLT_MIN (DBL_MIN) in r^2
// only keeps the logarithm finite there.
__device__ __forceinline__ void pair32l(double xi, double yi, const Src32& s, float& ar, float& ai)
{
    const float dx = (float)(xi - s.x);
    const float dy = (float)(yi - s.y);
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, FLT_MIN));
    const float lg = (dx != 0.f || dy != 0.f) ? 0.5f * __logf(r2) : 0.f;
    ar = fmaf(s.mr, lg, ar);
    ai = fmaf(s.mi, lg, ai);
}
__device__ __forceinline__ void pair64l(double xi, double yi, const Src64& s, double& ar, double& ai)
{
    const double dx = xi - s.x, dy = yi - s.y;
    const double r2 = fma(dx, dx, fma(dy, dy, DBL_MIN));
    const double lg = (dx != 0.0 || dy != 0.0) ? 0.5 * log(r2) : 0.0;
    ar = fma(s.mr, lg, ar);
    ai = fma(s.mi, lg, ai);
}

// near-field kernels: KERN 0 the plain harmonic kernel, 1 with the Gaussian
// smoother, 2 the logarithmic kernel (each its own instantiation, so the
// plain kernel keeps its registers)
constexpr int kKernPlain = 0, kKernSmooth = 1, kKernLog = 2;

// The value x of a partner lane whose bit M differs from this lane's and
// whose other bits above M agree: lane ^ 1 and lane ^ 2 (quad
// permutations), lane ^ 7 and lane ^ 15 (half-row and row mirrors) by DPP,
// wider distances by a cross-lane permute (lane ^ M).
template <int M>
constexpr int kDppCtrl = M == 1 ? 0xB1 : M == 2 ? 0x4E : M == 4 ? 0x141 : 0x140;
template <int M>
__device__ __forceinline__ float partner(float x)
{
    if constexpr (M <= 8)
        return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), kDppCtrl<M>, 0xF, 0xF, false));
    else
        return __shfl_xor(x, M, 64);
}
template <int M>
__device__ __forceinline__ double partner(double x)
{
    if constexpr (M <= 8) {
        const long long b = __double_as_longlong(x);
        const int lo = __builtin_amdgcn_update_dpp(0, (int)b, kDppCtrl<M>, 0xF, 0xF, false);
        const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kDppCtrl<M>, 0xF, 0xF, false);
        return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    } else {
        return __shfl_xor(x, M, 64);
    }
}

// Sum v[0..NV) over the aligned group of 2M lanes while transposing: at the
// step of distance M the lane keeps the half of its values selected by its
// bit M, summed with the partner's.  Both halves are summed and the sum is
// selected (a select of two array elements would become a run-time index).
// Every step's partner differs from the lane in bit M and in lower bits only,
// so the lanes summed into a value form the whole group, each once.
template <int M, int NV, int V, class T>
__device__ __forceinline__ void butterfly_step(T (&v)[V], int lane)
{
    if constexpr (M >= 1) {
        if constexpr (NV > 1) {
            constexpr int H = NV / 2;
            const bool hi = (lane & M) != 0;
#pragma unroll
            for (int i = 0; i < H; ++i) {
                const T lo_sum = v[i] + partner<M>(v[i]);
                const T hi_sum = v[i + H] + partner<M>(v[i + H]);
                v[i] = hi ? hi_sum : lo_sum;
            }
            butterfly_step<M / 2, H>(v, lane);
        } else {
            v[0] += partner<M>(v[0]);
            butterfly_step<M / 2, 1>(v, lane);
        }
    }
}

// Sum v[0..V) over the NL lanes of the subgroup while transposing:
// afterwards v[0] holds the total of value index butterfly_index<V, NL>.
// Requires V <= NL.
template <int V, int NL, class T>
__device__ __forceinline__ void butterfly(T (&v)[V], int lane)
{
    static_assert(V <= NL, "more values than lanes");
    butterfly_step<NL / 2, V>(v, lane);
}

// value index held by `lane` after butterfly<V, NL>: the bits of the lane
// used by the transposing steps, most significant step first
template <int V, int NL>
__device__ __forceinline__ int butterfly_index(int lane)
{
    int idx = 0, nv = V;
#pragma unroll
    for (int m = NL / 2; m >= 1; m >>= 1) {
        if (nv > 1) {
            nv /= 2;
            if (lane & m) idx += nv;
        }
    }
    return idx;
}

template <int TG, int SUB, int KERN>
__global__ void __launch_bounds__(256)
k_p2p64(const P2PItem* __restrict__ items, int item_base, const int2* __restrict__ xitems, int nx,
        const int32_t* __restrict__ icnt, const int32_t* __restrict__ ioff,
        double* __restrict__ partial, const int32_t* __restrict__ bstart,
        const int32_t* __restrict__ bcount, const int32_t* __restrict__ s_beg, const int32_t* __restrict__ s_cnt,
        const int32_t* __restrict__ s_ids, const double* __restrict__ X, const double* __restrict__ Y,
        const double2* __restrict__ M, double2* __restrict__ out, const long long* __restrict__ guard, double id2,
        const Targets tgt, int src_lim)
{
    if (guard != nullptr && *guard != 0) return;   // lists flagged: this launch is void
    constexpr int NL = 64 / SUB;
    static_assert(kP2PSrcCap64 % NL == 0, "the padded run must fit the staging buffer");
    __shared__ Src64 sbuf[4][kP2PSrcCap64];
    __shared__ int2 smeta[4][64];
    __shared__ int smark[4][kP2PSrcCap64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int xi_ = __builtin_amdgcn_readfirstlane(xcd_block() * 4 + w);   // one work item per wavefront
    if (xi_ >= nx) return;
    // (item, source chunk); without chunk lists every item is one chunk
    const int2 xe = xitems ? xitems[xi_] : make_int2(item_base + xi_, 0);
    const P2PItem it = items[xe.x];
    if (it.tn == 0) return;                        // a spare item of a device-built list
    const int nch = icnt ? icnt[xe.x] : 1;
    Src64* lds = sbuf[w];
    const int g = lane / NL, sl = lane % NL;
    // the targets: the leaf's own points, or evaluation points apart from the sources
    const int base = (tgt.start ? tgt.start : bstart)[it.leaf] + it.t0;
    const double* tx = tgt.start ? tgt.x : X;
    const double* ty = tgt.start ? tgt.y : Y;
    double xi[TG], yi[TG], ar[TG], ai[TG];
#pragma unroll
    for (int t = 0; t < TG; ++t) {
        int k = g * TG + t;
        const int i = base + (k < it.tn ? k : 0);
        xi[t] = tx[i]; yi[t] = ty[i]; ar[t] = 0.0; ai[t] = 0.0;
    }
    // the item's entries, or those of its chunk
    const int e0 = s_beg[it.leaf], ce = chunk_entries(bcount[it.leaf]);
    int e = nch == 1 ? 0 : xe.y * ce, off = 0;
    const int ne = nch == 1 ? s_cnt[it.leaf] : min(s_cnt[it.leaf], e + ce);
    auto load = [&](int j) {
        const double2 m = M[j];
        Src64 s; s.x = X[j]; s.y = Y[j]; s.mr = m.x; s.mi = m.y;
        return s;
    };
    while (e < ne) {
        const int ns = __builtin_amdgcn_readfirstlane(stage_sources<kP2PSrcCap64>(
            lds, smeta[w], smark[w], s_ids, bstart, bcount, e0, ne, e, off, lane, load, src_lim));
        // zero-strength sources (at the origin) pad the staged run to whole passes
        const int npad = (ns + NL - 1) / NL * NL;
        if (lane < npad - ns) lds[ns + lane] = Src64{0.0, 0.0, 0.0, 0.0};
        wave_sync();
        const Src64* sp = lds + sl;
        if constexpr (KERN == kKernSmooth) {     // the smoothed near field
            for (int c = 0; c < npad; c += NL, sp += NL) {
                const Src64 s = *sp;
#pragma unroll
                for (int t = 0; t < TG; ++t) pair64s(xi[t], yi[t], s, id2, ar[t], ai[t]);
            }
        } else if constexpr (KERN == kKernLog) {
            for (int c = 0; c < npad; c += NL, sp += NL) {
                const Src64 s = *sp;
#pragma unroll
                for (int t = 0; t < TG; ++t) pair64l(xi[t], yi[t], s, ar[t], ai[t]);
            }
        } else {
            for (int c = 0; c < npad; c += NL, sp += NL) {
                const Src64 s = *sp;
#pragma unroll
                for (int t = 0; t < TG; ++t) pair64(xi[t], yi[t], s, ar[t], ai[t]);
            }
        }
        wave_sync();
    }
    double v[2 * TG];
#pragma unroll
    for (int t = 0; t < TG; ++t) { v[2 * t] = ar[t]; v[2 * t + 1] = ai[t]; }
    butterfly<2 * TG, NL>(v, lane);
    const int idx = butterfly_index<2 * TG, NL>(sl);
    // lanes holding the same value index: write from the lowest one
    const int t = idx >> 1, comp = idx & 1;
    const bool writer = (sl & ((NL / (2 * TG) > 1) ? (NL / (2 * TG) - 1) : 0)) == 0;
    const int k = g * TG + t;
    if (writer && k < it.tn) {
        if (nch == 1) reinterpret_cast<double*>(out + base + k)[comp] = v[0];
        else partial[((int64_t)(ioff[xe.x] + xe.y) * kItemTargets + k) * 2 + comp] = v[0];
    }
}

template <int TG, int SUB, int KERN>
__global__ void __launch_bounds__(256)
k_p2p32(const P2PItem* __restrict__ items, int item_base, const int2* __restrict__ xitems, int nx,
        const int32_t* __restrict__ icnt, const int32_t* __restrict__ ioff,
        double* __restrict__ partial, const int32_t* __restrict__ bstart,
        const int32_t* __restrict__ bcount, const int32_t* __restrict__ s_beg, const int32_t* __restrict__ s_cnt,
        const int32_t* __restrict__ s_ids, const double* __restrict__ X, const double* __restrict__ Y,
        const double2* __restrict__ M, double2* __restrict__ out, const long long* __restrict__ guard, float id2,
        const Targets tgt, int src_lim)
{
    if (guard != nullptr && *guard != 0) return;   // lists flagged: this launch is void
    constexpr int NL = 64 / SUB;
    static_assert(kP2PSrcCap32 % NL == 0, "the padded run must fit the staging buffer");
    __shared__ Src32 sbuf[4][kP2PSrcCap32];
    __shared__ int2 smeta[4][64];
    __shared__ int smark[4][kP2PSrcCap32];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int xi_ = __builtin_amdgcn_readfirstlane(xcd_block() * 4 + w);   // one work item per wavefront
    if (xi_ >= nx) return;
    // (item, source chunk); without chunk lists every item is one chunk
    const int2 xe = xitems ? xitems[xi_] : make_int2(item_base + xi_, 0);
    const P2PItem it = items[xe.x];
    if (it.tn == 0) return;                        // a spare item of a device-built list
    const int nch = icnt ? icnt[xe.x] : 1;
    Src32* lds = sbuf[w];
    const int g = lane / NL, sl = lane % NL;
    // the targets: the leaf's own points, or evaluation points apart from the sources
    const int base = (tgt.start ? tgt.start : bstart)[it.leaf] + it.t0;
    const double* tx = tgt.start ? tgt.x : X;
    const double* ty = tgt.start ? tgt.y : Y;
    double xi[TG], yi[TG];
    float ar[TG], ai[TG];
#pragma unroll
    for (int t = 0; t < TG; ++t) {
        int k = g * TG + t;
        const int i = base + (k < it.tn ? k : 0);
        xi[t] = tx[i]; yi[t] = ty[i]; ar[t] = 0.f; ai[t] = 0.f;
    }
    // the item's entries, or those of its chunk
    const int e0 = s_beg[it.leaf], ce = chunk_entries(bcount[it.leaf]);
    int e = nch == 1 ? 0 : xe.y * ce, off = 0;
    const int ne = nch == 1 ? s_cnt[it.leaf] : min(s_cnt[it.leaf], e + ce);
    auto load = [&](int j) {
        const double2 m = M[j];
        Src32 s; s.x = X[j]; s.y = Y[j]; s.mr = (float)m.x; s.mi = (float)m.y;
        return s;
    };
    while (e < ne) {
        const int ns = __builtin_amdgcn_readfirstlane(stage_sources<kP2PSrcCap32>(
            lds, smeta[w], smark[w], s_ids, bstart, bcount, e0, ne, e, off, lane, load, src_lim));
        // zero-strength sources (at the origin) pad the staged run to whole passes
        const int npad = (ns + NL - 1) / NL * NL;
        if (lane < npad - ns) lds[ns + lane] = Src32{0.0, 0.0, 0.f, 0.f};
        wave_sync();
        const Src32* sp = lds + sl;
        if constexpr (KERN == kKernSmooth) {     // the smoothed near field
            for (int c = 0; c < npad; c += NL, sp += NL) {
                const Src32 s = *sp;
#pragma unroll
                for (int t = 0; t < TG; ++t) pair32s(xi[t], yi[t], s, id2, ar[t], ai[t]);
            }
        } else if constexpr (KERN == kKernLog) {
            for (int c = 0; c < npad; c += NL, sp += NL) {
                const Src32 s = *sp;
#pragma unroll
                for (int t = 0; t < TG; ++t) pair32l(xi[t], yi[t], s, ar[t], ai[t]);
            }
        } else {
            for (int c = 0; c < npad; c += NL, sp += NL) {
                const Src32 s = *sp;
#pragma unroll
                for (int t = 0; t < TG; ++t) pair32(xi[t], yi[t], s, ar[t], ai[t]);
            }
        }
        wave_sync();
    }
    float v[2 * TG];
#pragma unroll
    for (int t = 0; t < TG; ++t) { v[2 * t] = ar[t]; v[2 * t + 1] = ai[t]; }
    butterfly<2 * TG, NL>(v, lane);
    const int idx = butterfly_index<2 * TG, NL>(sl);
    const int t = idx >> 1, comp = idx & 1;
    const bool writer = (sl & ((NL / (2 * TG) > 1) ? (NL / (2 * TG) - 1) : 0)) == 0;
    const int k = g * TG + t;
    if (writer && k < it.tn) {
        if (nch == 1) reinterpret_cast<double*>(out + base + k)[comp] = (double)v[0];
        else partial[((int64_t)(ioff[xe.x] + xe.y) * kItemTargets + k) * 2 + comp] = (double)v[0];
    }
}

template <int TG, int SUB, int KERN>
static void launch_kern(bool mixed, const P2PItem* items, int item_base, const int2* xitems, int nx,
                        const int32_t* icnt, const int32_t* ioff, double* partial,
                        const int32_t* bstart, const int32_t* bcount, const int32_t* s_beg, const int32_t* s_cnt,
                        const int32_t* s_ids, const double* X, const double* Y, const double2* M, double* out,
                        hipStream_t s, const long long* guard, double id2, const Targets& tgt, int src_lim)
{
    const int grid = (nx + 3) / 4;
    if (mixed)
        k_p2p32<TG, SUB, KERN><<<grid, 256, 0, s>>>(items, item_base, xitems, nx, icnt, ioff, partial, bstart,
                                                   bcount, s_beg, s_cnt, s_ids, X, Y, M, (double2*)out, guard,
                                                   (float)id2, tgt, src_lim);
    else
        k_p2p64<TG, SUB, KERN><<<grid, 256, 0, s>>>(items, item_base, xitems, nx, icnt, ioff, partial, bstart,
                                                   bcount, s_beg, s_cnt, s_ids, X, Y, M, (double2*)out, guard,
                                                   id2, tgt, src_lim);
}

template <int TG, int SUB>
static void launch_one(bool mixed, const P2PItem* items, int item_base, const int2* xitems, int nx, const int32_t* icnt,
                       const int32_t* ioff, double* partial, const int32_t* bstart,
                       const int32_t* bcount, const int32_t* s_beg, const int32_t* s_cnt, const int32_t* s_ids,
                       const double* X, const double* Y, const double2* M, double* out, hipStream_t s,
                       const long long* guard, double id2, bool log_kernel, const Targets& tgt, int src_lim)
{
#define ARGS mixed, items, item_base, xitems, nx, icnt, ioff, partial, bstart, bcount, s_beg, s_cnt, s_ids, X, Y, \
             M, out, s, guard, id2, tgt, src_lim
    if (log_kernel) launch_kern<TG, SUB, kKernLog>(ARGS);
    else if (id2 > 0.0) launch_kern<TG, SUB, kKernSmooth>(ARGS);
    else launch_kern<TG, SUB, kKernPlain>(ARGS);
#undef ARGS
}

// one launch per (targets per subgroup, subgroups) class over its chunks
// xitems[0 .. nx) (entries (item, chunk), item indices into `items`), or,
// without chunk lists (xitems and icnt null), over items item_base + i
void launch_p2p(bool mixed, int tg, int sub, const void* items, int item_base, const int2* xitems, int nx,
                const int32_t* icnt,
                const int32_t* ioff, double* partial, const int32_t* bstart,
                const int32_t* bcount, const int32_t* s_beg, const int32_t* s_cnt, const int32_t* s_ids,
                const double* X, const double* Y, const double2* M, double* out, hipStream_t s,
                const long long* guard, double id2, bool log_kernel, const Targets& tgt, int src_tile)
{
    if (nx == 0) return;
    // sources staged per pass: the LDS buffer, or fewer (a multiple of every
    // subgroup width, so the passes stay whole)
    const int cap = mixed ? kP2PSrcCap32 : kP2PSrcCap64;
    const int src_lim = src_tile > 0 && src_tile < cap ? src_tile : cap;
    const P2PItem* it = (const P2PItem*)items;
#define CASE(TG_, SUB_)                                                                                   \
    if (tg == TG_ && sub == SUB_) {                                                                       \
        launch_one<TG_, SUB_>(mixed, it, item_base, xitems, nx, icnt, ioff, partial, bstart, bcount, s_beg, s_cnt, \
                              s_ids, X, Y, M, out, s, guard, id2, log_kernel, tgt, src_lim);                          \
        check_launch("p2p");                                                                              \
        return;                                                                                           \
    }
    CASE(1, 4) CASE(2, 4) CASE(4, 4)
    CASE(2, 2) CASE(4, 2) CASE(8, 2) CASE(16, 2)
    CASE(4, 1) CASE(8, 1) CASE(16, 1)
#undef CASE
    throw Error(FMM_EINVAL, "unsupported P2P launch shape");
}

}  // namespace fmm
