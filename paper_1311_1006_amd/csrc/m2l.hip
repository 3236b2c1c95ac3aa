// m2l.hip -- multipole-to-local shifts over the weak lists, on MFMA (gfx950).
//
// For a weak pair (target T, source S) at one level, with d = c_T - c_S and
// scaled coefficients (a_k of S, b_l of T, scaling radii rs_S, rs_T), the
// shift of Sec. 2.1 for the harmonic kernel reads
//     b_l += (1/d) (-rs_T/d)^l  sum_k C(k+l, k) (rs_S/d)^k a_k .
// The matrix B_lk = C(k+l, k) is the same for every pair, so the work is the
// batched product Y = B X with X's columns x^(q)_k = u_q^k a^(q)_k
// (u_q = rs_S/d, one complex column per pair, stored as two real columns),
// followed by the per-pair row scaling f^(q)_l = (1/d)(-rs_T/d)^l and the sum
// over the pairs of the target.  Under the theta-criterion |u_S| + |u_T| <=
// 2 theta/(1+theta), so every scaled term is at most 1 in magnitude.
//
// One wavefront per target box.  Per batch of 32 pairs: lanes 0..31 form the
// scaled source columns, lanes 32..63 the target factors (FP64 powers, cast
// to the storage type), both into LDS; then per block of 8 pairs (16 real
// columns) the wavefront issues 16x16x4 MFMAs with the B matrix held in
// registers as the A operand, scales each output row by its pair's factor
// and accumulates; a butterfly over the 8 pair slots finishes the target.
// FP32 path: v_mfma_f32_16x16x4f32, FP32 accumulation.  FP64 path:
// v_mfma_f64_16x16x4f64.  p <= 16 uses one 16-row block, p <= 32 two.
#include "fmm_internal.h"
#include "kernels_common.h"

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
    static __device__ __forceinline__ int row(int lane, int j) { return 4 * (lane >> 4) + j; }
};
template <> struct Mfma<double> {
    using acc = doublex4;
    static __device__ __forceinline__ acc step(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // output element j of lane l sits in row l/16 + 4*j, column l%16
    static __device__ __forceinline__ int row(int lane, int j) { return (lane >> 4) + 4 * j; }
};

__device__ __forceinline__ void wave_sync_m()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double2 cpow_m(double2 b, int e)
{
    double2 r = make_double2(1.0, 0.0);
    while (e) {
        if (e & 1) r = cmul(r, b);
        b = cmul(b, b);
        e >>= 1;
    }
    return r;
}

// B pairs per batch; the 64 lanes are (pair q < B, role, chunk h < H) with
// B * 2 * H = 64: each lane runs PP/H steps of its power recurrence.
// Four independent wavefronts per workgroup, each with its own LDS tile.
template <class T, int PB, int B>
__global__ void __launch_bounds__(256)
k_m2l(const int32_t* __restrict__ boxes, int nbox, const int32_t* __restrict__ w_beg,
      const int32_t* __restrict__ w_cnt, const int32_t* __restrict__ w_ids, const double* __restrict__ geom,
      const double* __restrict__ binom, int p, const T* __restrict__ mp, T* loc)
{
    using T2 = typename Vec2<T>::type;
    using M = Mfma<T>;
    constexpr int PP = 16 * PB;      // padded number of terms
    constexpr int KS = PP / 4;       // k-steps of 4
    constexpr int H = 32 / B;        // k-chunks per (pair, role)
    constexpr int PH = PP / H;       // terms per chunk
    // tile[0] = scaled source columns x, tile[1] = target row factors f
    __shared__ T2 tile_all[4][2][B][PP + 1];
    const int w = threadIdx.x >> 6;
    const int bi = blockIdx.x * 4 + w;
    if (bi >= nbox) return;
    auto& tile = tile_all[w];
    const int g = boxes[bi];
    const int lane = threadIdx.x & 63;
    const int nw = w_cnt[g], wb = w_beg[g];
    const int col = lane & 15, kq = lane >> 4, part = col & 1, slot = col >> 1;

    // A operands: B_{row,k} = C(k+row, k), row = 16 rb + lane%16, k = 4 ks + lane/16
    T amat[PB][KS];
#pragma unroll
    for (int rb = 0; rb < PB; ++rb)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            int row = 16 * rb + (lane & 15), k = 4 * ks + (lane >> 4);
            amat[rb][ks] = (row < p && k < p) ? (T)binom[(k + row) * kBinomStride + k] : (T)0;
        }
    T oacc[PB][4];
#pragma unroll
    for (int rb = 0; rb < PB; ++rb)
#pragma unroll
        for (int j = 0; j < 4; ++j) oacc[rb][j] = (T)0;

    const double ctx = geom[4 * (int64_t)g], cty = geom[4 * (int64_t)g + 1], rsT = geom[4 * (int64_t)g + 3];
    // lane roles of phase 1
    const int q = lane % B, role = (lane / B) & 1, h = lane / (2 * B);
    const int k0 = h * PH;
    for (int b0 = 0; b0 < nw; b0 += B) {
        // ---- phase 1: x_k = (rs_S/d)^k a_k (role 0) or f_l = (1/d)(-rs_T/d)^l (role 1)
        // for k in [k0, k0 + PH), FP64 powers, cast to the storage type
        {
            const bool valid = b0 + q < nw;
            const int S = valid ? w_ids[wb + b0 + q] : g;
            const double* gs = geom + 4 * (int64_t)S;
            const double dx = ctx - gs[0], dy = cty - gs[1];
            const double den = valid ? 1.0 / (dx * dx + dy * dy) : 0.0;
            const double2 id = make_double2(dx * den, -dy * den);     // 1/d (0 for padding)
            const double rb_ = role ? -rsT : gs[3];
            const double2 base = make_double2(rb_ * id.x, rb_ * id.y);
            double2 pw = cpow_m(base, k0);
            if (role) pw = cmul(pw, id);
            const T2* a = reinterpret_cast<const T2*>(mp) + (int64_t)S * p;
#pragma unroll 4
            for (int j = 0; j < PH; ++j) {
                const int k = k0 + j;
                double2 t = pw;
                if (role == 0) {
                    T2 ak;
                    if (k < p && valid) ak = a[k]; else { ak.x = (T)0; ak.y = (T)0; }
                    t = cmul(pw, make_double2((double)ak.x, (double)ak.y));
                }
                T2 v;
                v.x = (T)t.x; v.y = (T)t.y;
                tile[role][q][k] = v;
                pw = cmul(pw, base);
            }
        }
        wave_sync_m();
        // ---- phase 2: MFMA per block of 8 pairs, row scaling, accumulation
        const int nblk = min(B / 8, (nw - b0 + 7) / 8);
        for (int nb = 0; nb < nblk; ++nb) {
            const int qq = 8 * nb + slot;
#pragma unroll
            for (int rb = 0; rb < PB; ++rb) {
                typename M::acc acc = {0, 0, 0, 0};
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    T2 xv = tile[0][qq][4 * ks + kq];
                    acc = M::step(amat[rb][ks], part ? xv.y : xv.x, acc);
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int row = 16 * rb + M::row(lane, j);
                    T mine = acc[j];
                    T other = __shfl_xor(mine, 1, 64);
                    T re = part ? other : mine, im = part ? mine : other;
                    T2 f = tile[1][qq][row];
                    oacc[rb][j] += part ? (f.x * im + f.y * re) : (f.x * re - f.y * im);
                }
            }
        }
        wave_sync_m();
    }
    // ---- sum over the 8 pair slots (lanes differing in bits 1..3)
#pragma unroll
    for (int rb = 0; rb < PB; ++rb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            T v = oacc[rb][j];
            v += __shfl_xor(v, 2, 64);
            v += __shfl_xor(v, 4, 64);
            v += __shfl_xor(v, 8, 64);
            oacc[rb][j] = v;
        }
    if (slot == 0) {
#pragma unroll
        for (int rb = 0; rb < PB; ++rb)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = 16 * rb + M::row(lane, j);
                if (row < p) loc[2 * ((int64_t)g * p + row) + part] = oacc[rb][j];
            }
    }
}

template <class T, int PB, int B>
static void m2l_one(const int32_t* boxes, int n, const int32_t* w_beg, const int32_t* w_cnt, const int32_t* w_ids,
                    const double* geom, const double* binom, int p, const void* mp, void* loc, hipStream_t s)
{
    k_m2l<T, PB, B><<<(n + 3) / 4, 256, 0, s>>>(boxes, n, w_beg, w_cnt, w_ids, geom, binom, p, (const T*)mp,
                                                (T*)loc);
}

// batch: pairs per LDS batch (8, 16, 32; 0 = automatic).  FP64 tiles are
// twice as large, so FP64 defaults to smaller batches.
template <class T>
void launch_m2l(const int32_t* boxes, int n, const int32_t* w_beg, const int32_t* w_cnt, const int32_t* w_ids,
                const double* geom, const double* binom, int p, const void* mp, void* loc, hipStream_t s,
                int batch)
{
    if (n == 0) return;
    const bool dbl = sizeof(T) == 8;
    if (batch <= 0) batch = dbl ? 16 : 32;
    if (batch > 32) batch = 32;
    if (batch != 8 && batch != 16 && batch != 32) batch = 16;
    if (p > 16 && batch == 32 && dbl) batch = 16;   // LDS per workgroup
#define M2L_CASE(PB_, B_) \
    if ((p <= 16 ? 1 : 2) == PB_ && batch == B_) { m2l_one<T, PB_, B_>(boxes, n, w_beg, w_cnt, w_ids, geom, binom, p, mp, loc, s); check_launch("m2l"); return; }
    M2L_CASE(1, 8) M2L_CASE(1, 16) M2L_CASE(1, 32)
    M2L_CASE(2, 8) M2L_CASE(2, 16) M2L_CASE(2, 32)
#undef M2L_CASE
    throw Error(FMM_EINVAL, "unsupported M2L configuration");
}

template void launch_m2l<double>(const int32_t*, int, const int32_t*, const int32_t*, const int32_t*,
                                 const double*, const double*, int, const void*, void*, hipStream_t, int);
template void launch_m2l<float>(const int32_t*, int, const int32_t*, const int32_t*, const int32_t*,
                                const double*, const double*, int, const void*, void*, hipStream_t, int);

}  // namespace fmm
