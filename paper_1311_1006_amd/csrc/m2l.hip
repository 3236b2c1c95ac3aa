// m2l.hip -- multipole-to-local shifts over the weak lists, on MFMA (gfx950).
//
// For a weak pair (target T, source S) at one level, with d = c_T - c_S and
// scaled coefficients (a_k of S, b_l of T, scaling radii rs_S, rs_T), the
// shift of Sec. 2.1 for the harmonic kernel reads
//     b_l += f_l  sum_k C(k+l, k) x_k,   x_k = u^k a_k,  f_l = (1/d) w^l,
//     u = rs_S/d,  w = -rs_T/d.
// The matrix B_lk = C(k+l, k) is the same for every pair, so the work is a
// batched real product Y = B X over complex columns x (real and imaginary
// parts as two MFMA products), followed by the per-pair row scaling by f and
// the sum over the pairs of the target.  Under the theta-criterion
// |u| + |w| <= 2 theta/(1+theta), so every scaled term is at most 1.
//
// One wavefront per target box, blocks of 16 weak pairs (one or two blocks
// per iteration).  Lane (kq, q),
// kq = lane/16, q = lane%16, owns pair q of the block: it computes the powers
// it feeds to the MFMA (x_k for k = kq + 4i, the B operand of k-step i) and
// the row factors of the output rows it holds, and accumulates f_l * Y_lq in
// registers.  FP64 path: powers in FP64.  Mixed path: the centre difference
// in FP64, the powers in FP32 (their rounding stays below that of the FP32
// coefficients they multiply).
// No LDS and no barriers: the geometry and coefficients of the next block
// are loaded while the current one is computed.  At the end the 16 pair
// slots are summed by a butterfly.
// FP32 path: v_mfma_f32_16x16x4f32 (output rows 4 kq + j), FP32 accumulation.
// FP64 path: v_mfma_f64_16x16x4f64 (output rows kq + 4 j).
// p <= 16 uses one 16-row block (PB = 1), p <= 32 two.
#include "fmm_internal.h"
#include "kernels_common.h"

#include <type_traits>

namespace fmm {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <class T> struct Mfma;
template <> struct Mfma<float> {
    using acc = floatx4;
    static __device__ __forceinline__ acc step(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // output element j of lane l sits in row 4*(l/16)+j, column l%16
    static constexpr bool kRowsConsecutive = true;
};
template <> struct Mfma<double> {
    using acc = doublex4;
    static __device__ __forceinline__ acc step(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // output element j of lane l sits in row l/16 + 4*j, column l%16
    static constexpr bool kRowsConsecutive = false;
};

__device__ __forceinline__ double2 csel(bool c, double2 a, double2 b)
{
    return make_double2(c ? a.x : b.x, c ? a.y : b.y);
}

__device__ __forceinline__ float2 csel(bool c, float2 a, float2 b)
{
    return make_float2(c ? a.x : b.x, c ? a.y : b.y);
}

// z^e for e in 0..3 from z and z^2 (e differs between lanes): one product of
// two selected factors, so that no lane-indexed table is needed
template <class C2>
__device__ __forceinline__ C2 cpow_lane(C2 z, C2 z2, int e)
{
    C2 one;
    one.x = 1;
    one.y = 0;
    return cmul(csel(e & 1, z, one), csel(e & 2, z2, one));
}

// The data of one block of pairs held by one lane: source centre and scaling
// radius, and the coefficients a_k, k = kq + 4i, of its pair.
template <class T, int KS>
struct PairData {
    double sx, sy, rs;
    typename Vec2<T>::type a[KS];
};

// Loads that stay where they are written: relaxed atomic loads of wavefront
// scope are plain loads for the hardware, but the compiler neither sinks them
// to their first use nor reissues them, so a prefetch stays a prefetch.
__device__ __forceinline__ double ld_pin(const double* p)
{
    return __longlong_as_double(
        (long long)__hip_atomic_load((const unsigned long long*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT));
}
__device__ __forceinline__ int ld_pin(const int* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ float2 ld_pin(const float2* p)
{
    const unsigned long long u =
        __hip_atomic_load((const unsigned long long*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    return make_float2(__uint_as_float((unsigned)u), __uint_as_float((unsigned)(u >> 32)));
}
__device__ __forceinline__ double2 ld_pin(const double2* p)
{
    const double* d = reinterpret_cast<const double*>(p);
    return make_double2(ld_pin(d), ld_pin(d + 1));
}

template <class T, int KS>
__device__ __forceinline__ void load_pair(PairData<T, KS>& d, int S, int kq, int p, const double* __restrict__ geom,
                                          const T* __restrict__ mp)
{
    const double* gs = geom + 4 * (int64_t)S;
    d.sx = ld_pin(gs);
    d.sy = ld_pin(gs + 1);
    d.rs = ld_pin(gs + 3);
    const typename Vec2<T>::type* a = reinterpret_cast<const typename Vec2<T>::type*>(mp) + (int64_t)S * p;
    // every load in bounds (S is a box, k clamped to p - 1); the values of
    // padding lanes and of k >= p are masked where they are used
#pragma unroll
    for (int i = 0; i < KS; ++i) {
        const int k = kq + 4 * i;
        d.a[i] = ld_pin(a + (k < p ? k : p - 1));
    }
}

// complex product in the storage type: FP32 for the mixed path (the FP64
// power rounded first), FP64 for the FP64 path
__device__ __forceinline__ float2 scale_coef(double2 pw, float2 a)
{
    const float2 w = make_float2((float)pw.x, (float)pw.y);
    return cmul(w, a);
}
__device__ __forceinline__ double2 scale_coef(double2 pw, double2 a) { return cmul(pw, a); }

// 1/(dx^2 + dy^2) by v_rcp_f64 and two Newton steps
__device__ __forceinline__ double rcp_nr(double r2)
{
    double y = __builtin_amdgcn_rcp(r2);
    double e = fma(-r2, y, 1.0);
    y = fma(y, e, y);
    e = fma(-r2, y, 1.0);
    return fma(y, e, y);
}

template <class T, int PB, int G>
__global__ void __launch_bounds__(256)
k_m2l(const int32_t* __restrict__ boxes, const int2* __restrict__ xitems, int nx, const int32_t* __restrict__ icnt,
      const int32_t* __restrict__ ioff, double* __restrict__ partial, const int32_t* __restrict__ w_beg,
      const int32_t* __restrict__ w_cnt, const int32_t* __restrict__ w_ids, const double* __restrict__ geom,
      const double* __restrict__ binom, int p, const T* __restrict__ mp, T* loc,
      const long long* __restrict__ guard)
{
    using M = Mfma<T>;
    using T2 = typename Vec2<T>::type;
    constexpr int KS = 4 * PB;       // k-steps of 4 (K = 16 PB)
    constexpr int S = 16 / G;        // pair slots of one item in a block of 16
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int q = lane & 15, kq = lane >> 4;
    const int grp = q / S, sl = q % S;   // the item of this lane's column, its slot in the item
    const int xi0 = (xcd_block() * 4 + w) * G;
    if (xi0 >= nx) return;               // uniform per wavefront
    if (guard != nullptr && *guard != 0) return;   // lists flagged: this launch is void
    const int xi = xi0 + grp;
    // item (box, chunk of its weak list); without chunk lists every box is one item
    const bool item_ok = xi < nx;
    int2 xe = make_int2(0, 0);
    int g = 0, nch = 1, nw = 0, wb = 0;
    if (item_ok) {
        xe = xitems ? xitems[xi] : make_int2(xi, 0);
        g = boxes ? boxes[xe.x] : xe.x;
        nch = icnt ? icnt[xe.x] : 1;
        const int nw_all = w_cnt[g], p0 = xe.y * kChunkPairs;
        nw = nch == 1 ? nw_all : min(kChunkPairs, nw_all - p0);   // pairs of this item
        wb = w_beg[g] + p0;
    }
    // blocks: as many as the longest item of the wavefront needs
    int nblk = (nw + S - 1) / S;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) nblk = max(nblk, __shfl_xor(nblk, o, 64));
    // padding id: the first weak source of the first item that has pairs
    // (its coefficients are computed; an item without pairs may be a root,
    // whose multipole is not)
    const unsigned long long has = __ballot(nw > 0);
    const int first = nw > 0 ? w_ids[wb] : 0;
    const int pad_id = has ? __shfl(first, __ffsll((long long)has) - 1, 64) : 0;

    // A operands: B_{row,k} = C(k+row, k), row = 16 rb + lane%16, k = 4 ks + lane/16
    T amat[PB][KS];
#pragma unroll
    for (int rb = 0; rb < PB; ++rb)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int row = 16 * rb + q, k = 4 * ks + kq;
            amat[rb][ks] = (row < p && k < p) ? (T)binom[(k + row) * kBinomStride + k] : (T)0;
        }
    T ore[PB][4], oim[PB][4];
#pragma unroll
    for (int rb = 0; rb < PB; ++rb)
#pragma unroll
        for (int j = 0; j < 4; ++j) { ore[rb][j] = (T)0; oim[rb][j] = (T)0; }

    const double ctx = geom[4 * (int64_t)g], cty = geom[4 * (int64_t)g + 1], rsT = geom[4 * (int64_t)g + 3];
    const float rsTf = (float)rsT;
    // first output row of this lane within a 16-row block; the rows it holds
    // are r0 + j (FP32) or r0 + 4 j (FP64)
    const int r0 = M::kRowsConsecutive ? 4 * kq : kq;

    // software pipeline over blocks, unrolled by two with two register
    // buffers: while one buffer's pairs are computed, the other buffer's
    // geometry and coefficients (next block) and the ids of the block after
    // are in flight.  Every load is unconditional (indices clamped into the
    // list, padding replaced by pad_id).
    const int last = nw > 0 ? nw - 1 : 0;
    auto raw_id = [&](int e) { return nw > 0 ? ld_pin(w_ids + wb + (e < last ? e : last)) : pad_id; };
    auto compute = [&](const PairData<T, KS>& c, int bi) {
        const bool valid = bi * S + sl < nw;
        // Padding slots (past the end of an item's list) hold a real weak
        // source, so every coefficient is finite; they get 1/d = 0, hence
        // zero row factors, and add nothing.  Terms k >= p meet zero columns
        // of B and rows l >= p are not stored.
        T2 xv[KS];
        T fre[PB][4], fim[PB][4];
        if constexpr (std::is_same<T, float>::value) {
            // mixed: the centre difference in FP64 (the centres are close in
            // value), everything after it in FP32
            const float dx = (float)(ctx - c.sx), dy = (float)(cty - c.sy);
            const float den = valid ? __builtin_amdgcn_rcpf(dx * dx + dy * dy) : 0.f;
            const float2 id = make_float2(dx * den, -dy * den);        // 1/d (0 for padding)
            const float rs = (float)c.rs;
            const float2 u = make_float2(rs * id.x, rs * id.y);        // rs_S / d
            const float2 wv = make_float2(-rsTf * id.x, -rsTf * id.y); // -rs_T / d
            const float2 u2 = cmul(u, u), u4 = cmul(u2, u2);
            const float2 w2 = cmul(wv, wv), w4 = cmul(w2, w2), w8 = cmul(w4, w4);
            float2 pw = cpow_lane(u, u2, kq);                           // u^kq
#pragma unroll
            for (int i = 0; i < KS; ++i) {
                xv[i] = cmul(pw, c.a[i]);
                if (i + 1 < KS) pw = cmul(pw, u4);
            }
            // output rows 16 rb + 4 kq + j: f = (1/d) w^(4 kq + j) w^(16 rb)
            const float2 f0 = cmul(cpow_lane(w4, w8, kq), id);
#pragma unroll
            for (int rb = 0; rb < PB; ++rb) {
                float2 f = rb > 0 ? cmul(f0, cmul(w8, w8)) : f0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    fre[rb][j] = f.x;
                    fim[rb][j] = f.y;
                    if (j < 3) f = cmul(f, wv);
                }
            }
        } else {
            // ---- FP64 powers of this lane's pair
            const double dx = ctx - c.sx, dy = cty - c.sy;
            const double den = valid ? rcp_nr(dx * dx + dy * dy) : 0.0;
            const double2 id = make_double2(dx * den, -dy * den);          // 1/d (0 for padding)
            const double2 u = make_double2(c.rs * id.x, c.rs * id.y);      // rs_S / d
            const double2 wv = make_double2(-rsT * id.x, -rsT * id.y);     // -rs_T / d
            const double2 u2 = cmul(u, u), u4 = cmul(u2, u2);
            const double2 w2 = cmul(wv, wv), w4 = cmul(w2, w2);
            // B operands x_k, k = kq + 4 i
            double2 pw = cpow_lane(u, u2, kq);
#pragma unroll
            for (int i = 0; i < KS; ++i) {
                xv[i] = scale_coef(pw, c.a[i]);
                if (i + 1 < KS) pw = cmul(pw, u4);
            }
            // row factors f_l = (1/d) w^l of this lane's output rows
            double2 base;                    // w^r0
            if (M::kRowsConsecutive) base = cpow_lane(w4, cmul(w4, w4), kq);
            else base = cpow_lane(wv, w2, kq);
            const double2 step = M::kRowsConsecutive ? wv : w4;
            double2 f0 = cmul(base, id);
#pragma unroll
            for (int rb = 0; rb < PB; ++rb) {
                double2 f = f0;
                if (rb > 0) {                // row r0 + 16: times w^16
                    const double2 w8 = cmul(w4, w4);
                    f = cmul(f0, cmul(w8, w8));
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    fre[rb][j] = (T)f.x;
                    fim[rb][j] = (T)f.y;
                    if (j < 3) f = cmul(f, step);
                }
            }
        }
        // ---- MFMA: Y = B Re(X), B Im(X); scale rows by f and accumulate
#pragma unroll
        for (int rb = 0; rb < PB; ++rb) {
            typename M::acc yr = {0, 0, 0, 0}, yi = {0, 0, 0, 0};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                yr = M::step(amat[rb][ks], xv[ks].x, yr);
                yi = M::step(amat[rb][ks], xv[ks].y, yi);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {   // o += f y, complex, as two fused steps per part
                ore[rb][j] = fma(fre[rb][j], (T)yr[j], fma(-fim[rb][j], (T)yi[j], ore[rb][j]));
                oim[rb][j] = fma(fre[rb][j], (T)yi[j], fma(fim[rb][j], (T)yr[j], oim[rb][j]));
            }
        }
    };
    PairData<T, KS> bufA, bufB;
    int sidA, sidB;
    load_pair<T, KS>(bufA, raw_id(sl), kq, p, geom, mp);
    sidB = raw_id(S + sl);
    for (int bi = 0; bi < nblk; bi += 2) {
        // block bi in bufA; load block bi + 1 into bufB, the id of block bi + 2
        sidA = raw_id((bi + 2) * S + sl);
        load_pair<T, KS>(bufB, sidB, kq, p, geom, mp);
        compute(bufA, bi);
        if (bi + 1 >= nblk) break;
        // block bi + 1 in bufB; load block bi + 2 into bufA, the id of block bi + 3
        sidB = raw_id((bi + 3) * S + sl);
        load_pair<T, KS>(bufA, sidA, kq, p, geom, mp);
        compute(bufB, bi + 1);
    }
    // ---- sum over the S slots of every item (lanes differing in the low bits of q)
#pragma unroll
    for (int rb = 0; rb < PB; ++rb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            T a = ore[rb][j], b = oim[rb][j];
#pragma unroll
            for (int o = 1; o < S; o <<= 1) {
                a += __shfl_xor(a, o, 64);
                b += __shfl_xor(b, o, 64);
            }
            ore[rb][j] = a;
            oim[rb][j] = b;
        }
    // slot j (< 4) of an item writes element j of its rows (zeros for a box
    // without weak pairs, so every box's local expansion is written)
    if (item_ok && sl < 4) {
#pragma unroll
        for (int rb = 0; rb < PB; ++rb) {
            T vr = ore[rb][0], vi = oim[rb][0];
#pragma unroll
            for (int j = 1; j < 4; ++j)
                if (sl == j) { vr = ore[rb][j]; vi = oim[rb][j]; }
            const int row = 16 * rb + r0 + (M::kRowsConsecutive ? sl : 4 * sl);
            if (row < p) {
                if (nch == 1) {
                    T* dst = loc + 2 * ((int64_t)g * p + row);
                    dst[0] = vr;
                    dst[1] = vi;
                } else {                          // partial sum of a split list
                    double* dst = partial + 2 * ((int64_t)(ioff[xe.x] + xe.y) * p + row);
                    dst[0] = (double)vr;
                    dst[1] = (double)vi;
                }
            }
        }
    }
}

template <class T, int PB, int G>
static void m2l_one(const int32_t* boxes, const int2* xitems, int nx, const int32_t* icnt, const int32_t* ioff,
                    double* partial, const int32_t* w_beg, const int32_t* w_cnt, const int32_t* w_ids,
                    const double* geom, const double* binom, int p, const void* mp, void* loc, hipStream_t s,
                    const long long* guard)
{
    const int per_block = 4 * G;   // items per workgroup (4 wavefronts)
    k_m2l<T, PB, G><<<(nx + per_block - 1) / per_block, 256, 0, s>>>(boxes, xitems, nx, icnt, ioff, partial, w_beg,
                                                                     w_cnt, w_ids, geom, binom, p, (const T*)mp,
                                                                     (T*)loc, guard);
}

// the partial local expansions of split lists, added in chunk order
template <class T>
__global__ void k_m2l_combine(const int32_t* __restrict__ boxes, int n, const int32_t* __restrict__ icnt,
                              const int32_t* __restrict__ ioff, const double* __restrict__ partial, int p, T* loc)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * p) return;
    const int i = (int)(t / p), row = (int)(t % p);
    const int c = icnt[i];
    if (c <= 1) return;
    const int64_t o = ioff[i];
    double re = 0.0, im = 0.0;
    for (int k = 0; k < c; ++k) {
        re += partial[2 * ((o + k) * p + row)];
        im += partial[2 * ((o + k) * p + row) + 1];
    }
    T* dst = loc + 2 * ((int64_t)(boxes ? boxes[i] : i) * p + row);
    dst[0] = (T)re;
    dst[1] = (T)im;
}

// Every box of `boxes` (NULL: boxes 0 .. n-1, no lookup) gets its local
// expansion written (zeros for a box without weak pairs).  xitems[0 .. nx): (box index, chunk); icnt/ioff per
// box index; partial holds the chunks of split lists.  batch: pair slots of
// one item in each 16-pair MFMA block: 16 (one item per wavefront), 8 (two)
// or 4 (four items share a wavefront); 0 = automatic (8 for FP32, 4 for
// FP64: the fastest on the uniform million-point case).
template <class T>
void launch_m2l(const int32_t* boxes, int n, const int2* xitems, int nx, const int32_t* icnt, const int32_t* ioff,
                double* partial, bool split, const int32_t* w_beg, const int32_t* w_cnt, const int32_t* w_ids,
                const double* geom, const double* binom, int p, const void* mp, void* loc, hipStream_t s, int batch,
                const long long* guard)
{
    if (nx == 0) return;
    const int slots = batch != 0 ? batch : (std::is_same<T, float>::value ? 8 : 4);
#define ARGS boxes, xitems, nx, icnt, ioff, partial, w_beg, w_cnt, w_ids, geom, binom, p, mp, loc, s, guard
    if (p <= 16) {
        if (slots == 16) m2l_one<T, 1, 1>(ARGS);
        else if (slots == 8) m2l_one<T, 1, 2>(ARGS);
        else if (slots == 4) m2l_one<T, 1, 4>(ARGS);
        else throw Error(FMM_EINVAL, "unsupported M2L batch");
    } else if (p <= 32) {
        if (slots == 16) m2l_one<T, 2, 1>(ARGS);
        else if (slots == 8) m2l_one<T, 2, 2>(ARGS);
        else if (slots == 4) m2l_one<T, 2, 4>(ARGS);
        else throw Error(FMM_EINVAL, "unsupported M2L batch");
    } else {
        throw Error(FMM_EINVAL, "unsupported M2L configuration");
    }
#undef ARGS
    check_launch("m2l");
    if (split) {
        const int64_t nt = (int64_t)n * p;
        k_m2l_combine<T><<<(unsigned)((nt + 255) / 256), 256, 0, s>>>(boxes, n, icnt, ioff, partial, p, (T*)loc);
        check_launch("m2l combine");
    }
}

#define INST_M2L(T)                                                                                        \
    template void launch_m2l<T>(const int32_t*, int, const int2*, int, const int32_t*, const int32_t*, double*, \
                                bool, const int32_t*, const int32_t*, const int32_t*, const double*,            \
                                const double*, int, const void*, void*, hipStream_t, int,     \
                                const long long*);
INST_M2L(double)
INST_M2L(float)
#undef INST_M2L

}  // namespace fmm
