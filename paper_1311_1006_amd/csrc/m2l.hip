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
// One wavefront per target box (or 2 or 4 boxes), blocks of 16 weak pairs.
// Lane (kq, q), kq = lane/16, q = lane%16, feeds column q of the block (a
// pair): it computes the powers
// it feeds to the MFMA (x_k for k = kq + 4i, the B operand of k-step i) and
// the row factors of the output rows it holds, and accumulates f_l * Y_lq in
// registers.  FP64 path: powers in FP64.  Mixed path: the centre difference
// in FP64, the powers in FP32 (their rounding stays below that of the FP32
// coefficients they multiply).
// The blocks go in groups of four: each lane computes the geometry of one
// pair of the group once (centre difference, 1/d, the powers of u and w) and
// shares it through the wavefront's LDS with the other three lanes of that
// pair's column, including the starting power u^kq and the first row factor
// of each of the four lanes, so that a lane reads its own instead of
// selecting them; no workgroup barriers.  Source centres are loaded a
// group ahead, coefficients a block ahead.  At the end the 16 pair slots
// are summed by a butterfly.
// FP32 path: v_mfma_f32_16x16x4f32 (output rows 4 kq + j), FP32 accumulation.
// FP64 path: v_mfma_f64_16x16x4f64 (output rows kq + 4 j).
// p <= 16 uses one 16-row block (PB = 1), p <= 32 two, p <= 48 three and
// p <= 64 four (those with one box per wavefront: the expansion orders of the
// strictest tolerances, where a wavefront's 16 pair slots stay full anyway).
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

// The geometry of one pair, computed once by one lane and shared through
// LDS with the four lanes (kq = 0..3) that feed the pair's MFMA column, with
// u = rs_S/d and w = -rs_T/d: up[kq] = u^kq (the first power lane kq
// scales), u4 = u^4 (its step), f0[kq] = (1/d) w^r0 (the factor of lane
// kq's first output row r0: 4 kq for FP32, kq for FP64) and ws, the factor
// between its consecutive rows (w for FP32, w^4 for FP64).
template <class T>
struct PairGeo {
    using T2 = typename Vec2<T>::type;
    T2 up[4], f0[4], u4, ws;
};
constexpr int kGeoFields = 10;   // up[0..3], f0[0..3], u4, ws

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

// the coefficients a_k, k = kq + 4i, of box S (k clamped to p - 1: every
// load in bounds; the values of k >= p meet zero columns of B)
template <class T, int KS>
__device__ __forceinline__ void load_coef(typename Vec2<T>::type (&a)[KS], int S, int kq, int p,
                                          const T* __restrict__ mp)
{
    const typename Vec2<T>::type* src = reinterpret_cast<const typename Vec2<T>::type*>(mp) + (int64_t)S * p;
#pragma unroll
    for (int i = 0; i < KS; ++i) {
        const int k = kq + 4 * i;
        a[i] = ld_pin(src + (k < p ? k : p - 1));
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
__device__ __forceinline__ float2 scale_coef(float2 pw, float2 a) { return cmul(pw, a); }

// 1/(dx^2 + dy^2) by v_rcp_f64 and two Newton steps
__device__ __forceinline__ double rcp_nr(double r2)
{
    double y = __builtin_amdgcn_rcp(r2);
    double e = fma(-r2, y, 1.0);
    y = fma(y, e, y);
    e = fma(-r2, y, 1.0);
    return fma(y, e, y);
}

// Geometry of the pair (target centre ct, radius rsT; source centre cs,
// radius rs).  A padding pair (valid false) gets 1/d = 0, hence zero
// factors everywhere.  Mixed path: the centre difference in FP64 (the
// centres are close in value), everything after it in FP32.
__device__ __forceinline__ PairGeo<float> make_geo(float, double ctx, double cty, double rsT, double sx, double sy,
                                                   double rs_s, bool valid)
{
    PairGeo<float> g;
    const float dx = (float)(ctx - sx), dy = (float)(cty - sy);
    const float den = valid ? __builtin_amdgcn_rcpf(dx * dx + dy * dy) : 0.f;
    const float2 id = make_float2(dx * den, -dy * den);
    const float rs = (float)rs_s, rt = (float)rsT;
    const float2 u = make_float2(rs * id.x, rs * id.y);
    const float2 w = make_float2(-rt * id.x, -rt * id.y);
    const float2 u2 = cmul(u, u);
    g.up[0] = make_float2(1.f, 0.f);
    g.up[1] = u;
    g.up[2] = u2;
    g.up[3] = cmul(u2, u);
    g.u4 = cmul(u2, u2);
    const float2 w2 = cmul(w, w), w4 = cmul(w2, w2), w8 = cmul(w4, w4);
    g.f0[0] = id;                       // rows 4 kq + j: f0 = (1/d) w^(4 kq)
    g.f0[1] = cmul(id, w4);
    g.f0[2] = cmul(id, w8);
    g.f0[3] = cmul(g.f0[1], w8);
    g.ws = w;
    return g;
}
__device__ __forceinline__ PairGeo<double> make_geo(double, double ctx, double cty, double rsT, double sx, double sy,
                                                    double rs, bool valid)
{
    PairGeo<double> g;
    const double dx = ctx - sx, dy = cty - sy;
    const double den = valid ? rcp_nr(dx * dx + dy * dy) : 0.0;
    const double2 id = make_double2(dx * den, -dy * den);
    const double2 u = make_double2(rs * id.x, rs * id.y);
    const double2 w = make_double2(-rsT * id.x, -rsT * id.y);
    const double2 u2 = cmul(u, u);
    g.up[0] = make_double2(1.0, 0.0);
    g.up[1] = u;
    g.up[2] = u2;
    g.up[3] = cmul(u2, u);
    g.u4 = cmul(u2, u2);
    const double2 w2 = cmul(w, w);
    g.f0[0] = id;                       // rows kq + 4 j: f0 = (1/d) w^kq
    g.f0[1] = cmul(id, w);
    g.f0[2] = cmul(id, w2);
    g.f0[3] = cmul(g.f0[1], w2);
    g.ws = cmul(w2, w2);
    return g;
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

    // first output row of this lane within a 16-row block; the rows it holds
    // are r0 + j (FP32) or r0 + 4 j (FP64)
    const int r0 = M::kRowsConsecutive ? 4 * kq : kq;

    // Blocks go in groups of four.  Lane (kq, q) computes the geometry of the
    // pair in column q of block 4 gi + kq once and puts it (with the source
    // id) into LDS; every block then reads its column's geometry from there.
    // Loads run ahead: the next group's source centres and the ids of the
    // group after it during a group, the coefficients of the next block
    // during a block.  Every load is unconditional (indices clamped into the
    // list, padding replaced by pad_id).
    // one array per field ([field][block][column]): the 16 columns of a
    // block read 16 consecutive entries, free of bank conflicts
    __shared__ T2 sgeo[4][kGeoFields][4][16];
    __shared__ int ssid[4][4][16];
    T2(*geo)[4][16] = sgeo[w];
    int(*gsid)[16] = ssid[w];
    auto put_geo = [&](const PairGeo<T>& c) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            geo[e][kq][q] = c.up[e];
            geo[4 + e][kq][q] = c.f0[e];
        }
        geo[8][kq][q] = c.u4;
        geo[9][kq][q] = c.ws;
    };
    // what lane (kq, q) needs of the pair in column q of block j
    struct LaneGeo {
        T2 up, f0, u4, ws;
    };
    auto get_geo = [&](int j) {
        LaneGeo c;
        c.up = geo[kq][j][q];
        c.f0 = geo[4 + kq][j][q];
        c.u4 = geo[8][j][q];
        c.ws = geo[9][j][q];
        return c;
    };
    const int last = nw > 0 ? nw - 1 : 0;
    auto raw_id = [&](int e) { return nw > 0 ? ld_pin(w_ids + wb + (e < last ? e : last)) : pad_id; };
    auto gpair = [&](int gi) { return (4 * gi + kq) * S + sl; };   // this lane's geometry pair in group gi
    auto compute = [&](const LaneGeo& c, const T2 (&a)[KS]) {
        // Terms k >= p meet zero columns of B and rows l >= p are not stored.
        T2 xv[KS];
        T fre[PB][4], fim[PB][4];
        auto pw = c.up;                                                  // u^kq
#pragma unroll
        for (int i = 0; i < KS; ++i) {
            xv[i] = scale_coef(pw, a[i]);
            if (i + 1 < KS) pw = cmul(pw, c.u4);
        }
        // row factors f_l = (1/d) w^l of this lane's output rows
        const auto step = c.ws;
        T2 w16 = step;                          // w^16: w^(1 * 16) (FP32) or (w^4)^4 (FP64)
        if constexpr (PB > 1) {
#pragma unroll
            for (int e = 0; e < (M::kRowsConsecutive ? 4 : 2); ++e) w16 = cmul(w16, w16);
        }
        auto frb = c.f0;
#pragma unroll
        for (int rb = 0; rb < PB; ++rb) {
            if (rb > 0) frb = cmul(frb, w16);                               // row r0 + 16 rb: times w^(16 rb)
            auto f = frb;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                fre[rb][j] = (T)f.x;
                fim[rb][j] = (T)f.y;
                if (j < 3) f = cmul(f, step);
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
    const int ngrp = (nblk + 3) / 4;
    int gid = raw_id(gpair(0));                 // this lane's geometry pair, group 0
    const double* gs = geom + 4 * (int64_t)gid;
    double gsx = ld_pin(gs), gsy = ld_pin(gs + 1), grs = ld_pin(gs + 3);
    int gid_n = raw_id(gpair(1));               // group 1
    T2 ca[KS], cb[KS];
    load_coef<T, KS>(ca, __shfl(gid, q, 64), kq, p, mp);   // block 0: lane q's geometry pair
    for (int gi = 0; gi < ngrp; ++gi) {
        put_geo(make_geo(T(0), ctx, cty, rsT, gsx, gsy, grs, gpair(gi) < nw));
        gsid[kq][q] = gid;
        // the next group's source centres, the ids of the group after it
        gid = gid_n;
        gs = geom + 4 * (int64_t)gid;
        gsx = ld_pin(gs);
        gsy = ld_pin(gs + 1);
        grs = ld_pin(gs + 3);
        gid_n = raw_id(gpair(gi + 2));
        wave_sync();
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (4 * gi + j >= nblk) break;   // uniform per wavefront
            // the next block's source: the next column of this group, or
            // block 0 of the next group (lane q's geometry pair there)
            const int nsid = j < 3 ? gsid[j + 1][q] : __shfl(gid, q, 64);
            if (j % 2 == 0) {
                load_coef<T, KS>(cb, nsid, kq, p, mp);
                compute(get_geo(j), ca);
            } else {
                load_coef<T, KS>(ca, nsid, kq, p, mp);
                compute(get_geo(j), cb);
            }
        }
        wave_sync();   // the group's LDS is rewritten next
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
    // Every slot of an item holds the item's sums now.  Slot sl writes the
    // elements j of its rows with j = sl (4 or more slots), or j = sl mod S
    // (1 or 2 slots: a lane writes 4 or 2 of its rows).  A box without weak
    // pairs gets zeros, so every box's local expansion is written.
    if (item_ok && sl < 4) {
#pragma unroll
        for (int rb = 0; rb < PB; ++rb)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (S >= 4 ? j != sl : j % S != sl) continue;
                const int row = 16 * rb + r0 + (M::kRowsConsecutive ? j : 4 * j);
                if (row >= p) continue;
                if (nch == 1) {
                    T* dst = loc + 2 * ((int64_t)g * p + row);
                    dst[0] = ore[rb][j];
                    dst[1] = oim[rb][j];
                } else {                          // partial sum of a split list
                    double* dst = partial + 2 * ((int64_t)(ioff[xe.x] + xe.y) * p + row);
                    dst[0] = (double)ore[rb][j];
                    dst[1] = (double)oim[rb][j];
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
    // the values of eight chunks are loaded together, then added in chunk
    // order (a list of thousands of chunks took a memory round trip per chunk)
    const double* pr = partial + 2 * (o * p + row);
    const int64_t step = 2 * (int64_t)p;
    int k = 0;
    for (; k + 8 <= c; k += 8) {
        double vr[8], vi[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            vr[u] = pr[(k + u) * step];
            vi[u] = pr[(k + u) * step + 1];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            re += vr[u];
            im += vi[u];
        }
    }
    for (; k < c; ++k) {
        re += pr[k * step];
        im += pr[k * step + 1];
    }
    T* dst = loc + 2 * ((int64_t)(boxes ? boxes[i] : i) * p + row);
    dst[0] = (T)re;
    dst[1] = (T)im;
}

// Every box of `boxes` (NULL: boxes 0 .. n-1, no lookup) gets its local
// expansion written (zeros for a box without weak pairs).  xitems[0 .. nx): (box index, chunk); icnt/ioff per
// box index; partial holds the chunks of split lists.  batch: pair slots of
// one item in each 16-pair MFMA block: 16 (one item per wavefront), 8 (two)
// or 4 (four items share a wavefront); 0 = automatic (4, the fastest in both
// precisions on the uniform million-point case: mixed 81 us against 93 us
// with 8 slots, FP64 146 us against 161 us).
template <class T>
void launch_m2l(const int32_t* boxes, int n, const int2* xitems, int nx, const int32_t* icnt, const int32_t* ioff,
                double* partial, bool split, const int32_t* w_beg, const int32_t* w_cnt, const int32_t* w_ids,
                const double* geom, const double* binom, int p, const void* mp, void* loc, hipStream_t s, int batch,
                const long long* guard)
{
    if (nx == 0) return;
    const int slots = batch != 0 ? batch : 4;
#define ARGS boxes, xitems, nx, icnt, ioff, partial, w_beg, w_cnt, w_ids, geom, binom, p, mp, loc, s, guard
    if (p <= 16) {
        if (slots == 16) m2l_one<T, 1, 1>(ARGS);
        else if (slots == 8) m2l_one<T, 1, 2>(ARGS);
        else if (slots == 4) m2l_one<T, 1, 4>(ARGS);
        else if (slots == 2) m2l_one<T, 1, 8>(ARGS);
        else if (slots == 1) m2l_one<T, 1, 16>(ARGS);
        else throw Error(FMM_EINVAL, "unsupported M2L batch");
    } else if (p <= 32) {
        if (slots == 16) m2l_one<T, 2, 1>(ARGS);
        else if (slots == 8) m2l_one<T, 2, 2>(ARGS);
        else if (slots == 4) m2l_one<T, 2, 4>(ARGS);
        else if (slots == 2) m2l_one<T, 2, 8>(ARGS);
        else if (slots == 1) m2l_one<T, 2, 16>(ARGS);
        else throw Error(FMM_EINVAL, "unsupported M2L batch");
    } else if (p <= 48) {          // three and four row blocks: one box per wavefront
        m2l_one<T, 3, 1>(ARGS);
    } else if (p <= 64) {
        m2l_one<T, 4, 1>(ARGS);
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
