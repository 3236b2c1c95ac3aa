// expansions.hip -- P2M, M2M, L2L, L2P and the point gathers (Sec. 2.1,
// Fig. 2.2) on gfx950.
//
// Expansions are stored scaled by the box's scaling radius rs (its radius,
// or the nearest ancestor's radius when it is 0):
//     multipole  a_k = sum_j m_j ((z_j - c)/rs)^k        (k < p)
//     local      phi(z) = sum_l b_l ((z - c)/rs)^l
// so that every stored coefficient and every power is bounded by the data
// (|z - c| <= r <= rs inside the box).  In these variables the shifts are
//     M2M  a^P_k = sum_{l<=k} C(k,l) rho^l tau^(k-l) a^C_l
//     L2L  b^C_l = sum_{k>=l} C(k,l) rho^l tau^(k-l) b^P_k
// with rho = rs_C / rs_P and tau = (c_C - c_P) / rs_P (both exact re-centrings
// of the truncated series).  All four operators compute in FP64; T is the
// storage type of the coefficients (double for the FP64 path, float for the
// mixed path).  One 64-lane workgroup (one wavefront) per box.
#include "fmm_internal.h"
#include "kernels_common.h"

namespace fmm {

// strengths into tree order + the P2P source records
template <bool MIXED>
__global__ void k_gather(int64_t n, const int32_t* __restrict__ perm, const double* __restrict__ X,
                         const double* __restrict__ Y, const double2* __restrict__ m, double2* mtree,
                         double4* src64, float4* src32, float2* srclo)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 mm = m[perm[i]];
    double x = X[i], y = Y[i];
    mtree[i] = mm;
    if (MIXED) {
        float xh = (float)x, yh = (float)y;
        src32[i] = make_float4(xh, yh, (float)mm.x, (float)mm.y);
        srclo[i] = make_float2((float)(x - (double)xh), (float)(y - (double)yh));
    } else {
        src64[i] = make_double4(x, y, mm.x, mm.y);
    }
}

// P2M at the leaves.  Lane = point; the p terms m_j w_j^k are reduced over the
// points through LDS, 8 coefficients at a time, in point order.
template <class T>
__global__ void __launch_bounds__(64)
k_p2m(const int32_t* __restrict__ leaves, const int32_t* __restrict__ bstart, const int32_t* __restrict__ bcount,
      const double* __restrict__ geom, const double* __restrict__ X, const double* __restrict__ Y,
      const double2* __restrict__ mt, int p, T* mp)
{
    __shared__ double2 buf[64][9];
    int g = leaves[blockIdx.x];
    int lane = threadIdx.x;
    int st = bstart[g], n = bcount[g];
    double cx = geom[4 * g], cy = geom[4 * g + 1], inv = 1.0 / geom[4 * g + 3];
    double acc[kMaxP / 8];
#pragma unroll
    for (int c = 0; c < kMaxP / 8; ++c) acc[c] = 0.0;
    int kk = lane >> 1, part = lane & 1;   // lanes 0..15: coefficient k0 + kk, component part
    for (int j0 = 0; j0 < n; j0 += 64) {
        int j = j0 + lane;
        double2 w = make_double2(0, 0), pw = make_double2(1, 0), mm = make_double2(0, 0);
        if (j < n) {
            w = make_double2((X[st + j] - cx) * inv, (Y[st + j] - cy) * inv);
            mm = mt[st + j];
        }
        int cnt = min(64, n - j0);
#pragma unroll
        for (int c = 0; c < kMaxP / 8; ++c) {
            if (8 * c >= p) break;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                buf[lane][q] = cmul(mm, pw);
                pw = cmul(pw, w);
            }
            __syncthreads();
            if (lane < 16) {
                double s = 0.0;
                for (int jj = 0; jj < cnt; ++jj) s += part ? buf[jj][kk].y : buf[jj][kk].x;
                acc[c] += s;
            }
            __syncthreads();
        }
    }
    if (lane < 16) {
#pragma unroll
        for (int c = 0; c < kMaxP / 8; ++c) {
            int k = 8 * c + kk;
            if (k < p) mp[2 * ((int64_t)g * p + k) + part] = (T)acc[c];
        }
    }
}

// M2M into one parent from its four children
template <class T>
__global__ void __launch_bounds__(64)
k_m2m(const int32_t* __restrict__ parents, const int32_t* __restrict__ child0, const double* __restrict__ geom,
      const double* __restrict__ binom, int p, T* mp)
{
    __shared__ double2 tau[4][kMaxP];
    __shared__ double rho[4][kMaxP];
    int P = parents[blockIdx.x];
    int lane = threadIdx.x;
    int c0 = child0[P];
    double px = geom[4 * P], py = geom[4 * P + 1], prs = geom[4 * P + 3];
    if (lane < p) {
        for (int c = 0; c < 4; ++c) {
            const double* gc = geom + 4 * (int64_t)(c0 + c);
            double r = gc[3] / prs;
            double2 t = make_double2((gc[0] - px) / prs, (gc[1] - py) / prs);
            double2 tp = make_double2(1, 0);
            double rp = 1.0;
            for (int q = 0; q < lane; ++q) { tp = cmul(tp, t); rp *= r; }
            tau[c][lane] = tp;
            rho[c][lane] = rp;
        }
    }
    __syncthreads();
    if (lane < p) {
        int k = lane;
        double2 acc = make_double2(0, 0);
        for (int c = 0; c < 4; ++c) {
            const T* a = mp + 2 * (int64_t)(c0 + c) * p;
            for (int l = 0; l <= k; ++l) {
                double2 al = make_double2((double)a[2 * l], (double)a[2 * l + 1]);
                double s = binom[k * kBinomStride + l] * rho[c][l];
                double2 t = cmul(al, tau[c][k - l]);
                acc.x += s * t.x;
                acc.y += s * t.y;
            }
        }
        mp[2 * ((int64_t)P * p + k)] = (T)acc.x;
        mp[2 * ((int64_t)P * p + k) + 1] = (T)acc.y;
    }
}

// L2L: add the parent's local expansion to a child's
template <class T>
__global__ void __launch_bounds__(64)
k_l2l(const int32_t* __restrict__ boxes, const int32_t* __restrict__ parent, const double* __restrict__ geom,
      const double* __restrict__ binom, int p, T* loc)
{
    __shared__ double2 tau[kMaxP];
    int C = boxes[blockIdx.x];
    int P = parent[C];
    int lane = threadIdx.x;
    const double* gc = geom + 4 * (int64_t)C;
    const double* gp = geom + 4 * (int64_t)P;
    double prs = gp[3];
    double r = gc[3] / prs;
    if (lane < p) {
        double2 t = make_double2((gc[0] - gp[0]) / prs, (gc[1] - gp[1]) / prs);
        double2 tp = make_double2(1, 0);
        for (int q = 0; q < lane; ++q) tp = cmul(tp, t);
        tau[lane] = tp;
    }
    __syncthreads();
    if (lane < p) {
        int l = lane;
        double rl = 1.0;
        for (int q = 0; q < l; ++q) rl *= r;
        const T* b = loc + 2 * (int64_t)P * p;
        double2 acc = make_double2(0, 0);
        for (int k = l; k < p; ++k) {
            double2 bk = make_double2((double)b[2 * k], (double)b[2 * k + 1]);
            double2 t = cmul(bk, tau[k - l]);
            double s = binom[k * kBinomStride + l];
            acc.x += s * t.x;
            acc.y += s * t.y;
        }
        T* o = loc + 2 * ((int64_t)C * p + l);
        o[0] = (T)((double)o[0] + rl * acc.x);
        o[1] = (T)((double)o[1] + rl * acc.y);
    }
}

// L2P at the leaves, plus the near field, scattered to input order
template <class T>
__global__ void __launch_bounds__(64)
k_l2p(const int32_t* __restrict__ leaves, const int32_t* __restrict__ bstart, const int32_t* __restrict__ bcount,
      const double* __restrict__ geom, const double* __restrict__ X, const double* __restrict__ Y,
      const T* __restrict__ loc, int p, const double2* __restrict__ nearf, const int32_t* __restrict__ perm,
      double2* phi, double2* phi_near, double2* phi_far)
{
    int g = leaves[blockIdx.x];
    int st = bstart[g], n = bcount[g];
    double cx = geom[4 * g], cy = geom[4 * g + 1], inv = 1.0 / geom[4 * g + 3];
    const T* b = loc + 2 * (int64_t)g * p;
    for (int j = threadIdx.x; j < n; j += 64) {
        int i = st + j;
        double2 w = make_double2((X[i] - cx) * inv, (Y[i] - cy) * inv);
        double2 acc = make_double2((double)b[2 * (p - 1)], (double)b[2 * (p - 1) + 1]);
        for (int l = p - 2; l >= 0; --l) {
            acc = cmul(acc, w);
            acc.x += (double)b[2 * l];
            acc.y += (double)b[2 * l + 1];
        }
        double2 nf = nearf[i];
        int o = perm[i];
        if (phi) phi[o] = make_double2(acc.x + nf.x, acc.y + nf.y);
        if (phi_near) phi_near[o] = nf;
        if (phi_far) phi_far[o] = acc;
    }
}

template __global__ void k_gather<false>(int64_t, const int32_t*, const double*, const double*, const double2*,
                                         double2*, double4*, float4*, float2*);
template __global__ void k_gather<true>(int64_t, const int32_t*, const double*, const double*, const double2*,
                                        double2*, double4*, float4*, float2*);

// ------------------------------------------------------------ launchers

void launch_gather(bool mixed, int64_t n, const int32_t* perm, const double* X, const double* Y,
                   const double* m, double* mtree, double* src64, float* src32, float* srclo, hipStream_t s)
{
    int g = (int)((n + 255) / 256);
    if (mixed)
        k_gather<true><<<g, 256, 0, s>>>(n, perm, X, Y, (const double2*)m, (double2*)mtree, nullptr,
                                         (float4*)src32, (float2*)srclo);
    else
        k_gather<false><<<g, 256, 0, s>>>(n, perm, X, Y, (const double2*)m, (double2*)mtree, (double4*)src64,
                                          nullptr, nullptr);
    check_launch("gather");
}

template <class T>
void launch_p2m(const int32_t* leaves, int nleaf, const int32_t* bstart, const int32_t* bcount,
                const double* geom, const double* X, const double* Y, const double* mt, int p, void* mp,
                hipStream_t s)
{
    if (nleaf == 0) return;
    k_p2m<T><<<nleaf, 64, 0, s>>>(leaves, bstart, bcount, geom, X, Y, (const double2*)mt, p, (T*)mp);
    check_launch("p2m");
}

template <class T>
void launch_m2m(const int32_t* parents, int n, const int32_t* child0, const double* geom, const double* binom,
                int p, void* mp, hipStream_t s)
{
    if (n == 0) return;
    k_m2m<T><<<n, 64, 0, s>>>(parents, child0, geom, binom, p, (T*)mp);
    check_launch("m2m");
}

template <class T>
void launch_l2l(const int32_t* boxes, int n, const int32_t* parent, const double* geom, const double* binom,
                int p, void* loc, hipStream_t s)
{
    if (n == 0) return;
    k_l2l<T><<<n, 64, 0, s>>>(boxes, parent, geom, binom, p, (T*)loc);
    check_launch("l2l");
}

template <class T>
void launch_l2p(const int32_t* leaves, int nleaf, const int32_t* bstart, const int32_t* bcount,
                const double* geom, const double* X, const double* Y, const void* loc, int p,
                const double* nearf, const int32_t* perm, double* phi, double* phi_near, double* phi_far,
                hipStream_t s)
{
    if (nleaf == 0) return;
    k_l2p<T><<<nleaf, 64, 0, s>>>(leaves, bstart, bcount, geom, X, Y, (const T*)loc, p, (const double2*)nearf,
                                  perm, (double2*)phi, (double2*)phi_near, (double2*)phi_far);
    check_launch("l2p");
}

#define INST(T)                                                                                          \
    template void launch_p2m<T>(const int32_t*, int, const int32_t*, const int32_t*, const double*,      \
                                const double*, const double*, const double*, int, void*, hipStream_t);   \
    template void launch_m2m<T>(const int32_t*, int, const int32_t*, const double*, const double*, int,  \
                                void*, hipStream_t);                                                     \
    template void launch_l2l<T>(const int32_t*, int, const int32_t*, const double*, const double*, int,  \
                                void*, hipStream_t);                                                     \
    template void launch_l2p<T>(const int32_t*, int, const int32_t*, const int32_t*, const double*,      \
                                const double*, const double*, const void*, int, const double*,           \
                                const int32_t*, double*, double*, double*, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace fmm
