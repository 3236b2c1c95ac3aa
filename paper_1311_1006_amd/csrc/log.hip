// log.hip -- the logarithmic potential (the paper's second kernel, Sec. 3.3;
// its multipole expansion a_0 log(z - z0) + sum_k a_k / (z - z0)^k, Sec. 2.1).
//
// For real strengths q the potential is u(z) = sum_j q_j log|z - z_j| =
// Re F(z), F(z) = sum_j q_j log(z - z_j), and F' is the harmonic field
// f(z) = sum_j q_j / (z - z_j) that the rest of the library expands.  So the
// far field reuses the harmonic expansions and adds one number per box:
//   multipole of S (harmonic coefficients A_k = sum q_j (z_j - c_S)^k):
//       F_S(z) = A_0 log(z - c_S) - sum_{k>=1} A_k / (k (z - c_S)^k);
//   local expansion of T: F(z) = c0_T + sum_{l>=1} (B_{l-1} / l) (z - c_T)^l,
//       B_l the harmonic local coefficients, c0_T the constant term;
//   M2L adds Re F_S(c_T) over the weak list of T to c0_T;
//   L2L adds the parent's whole Re F_P(c_T) (with its own constant);
//   L2P evaluates Re F at the points.
// Stored coefficients are scaled (multipole a_k = A_k / rs^k, local
// b_l = B_l rs^l), so with d = c_T - c_S and x_k = a_k (rs_S / d)^k:
//   Re F_S(c_T) = Re(A_0) log|d| - Re sum_{k>=1} x_k / k,
//   Re F_T(z)   = c0_T + rs_T Re sum_{l>=0} b_l w^(l+1) / (l + 1),  w = (z - c_T) / rs_T.
// The constants are formed in FP64 from the stored coefficients of either
// precision.
#include "fmm_internal.h"
#include "kernels_common.h"

namespace fmm {

__global__ void k_real_to_complex(int64_t n, const double* __restrict__ q, double2* __restrict__ m)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) m[i] = make_double2(q[i], 0.0);
}

// 1/k for the series of the constant terms (a multiplication in place of an
// FP64 division per term)
struct InvK {
    double v[kMaxP];
};
constexpr InvK make_inv_k()
{
    InvK t{};
    for (int k = 1; k < kMaxP; ++k) t.v[k] = 1.0 / k;
    return t;
}
__constant__ InvK kInvK = make_inv_k();

// c0 of every box from its weak list (zero without one): 32 lanes per box,
// lane e takes pairs e, e + 32, ... (on uniform inputs at theta = 0.5 most
// lists are shorter than 64, so one or two passes; clustered inputs reach
// lists of a few hundred entries, which take more passes of the same lanes);
// the lanes' sums are added by a butterfly (a fixed order, so the result is
// reproducible)
template <class T>
__global__ void __launch_bounds__(256)
k_m2l_log0(int nbox, const int32_t* __restrict__ w_beg, const int32_t* __restrict__ w_cnt,
           const int32_t* __restrict__ w_ids, const double* __restrict__ geom, const T* __restrict__ mp, int p,
           double* __restrict__ c0)
{
    const int g = blockIdx.x * 8 + (threadIdx.x >> 5), lane = threadIdx.x & 31;
    const bool live = g < nbox;   // every lane stays for the butterfly
    const int b = live ? w_beg[g] : 0, n = live ? w_cnt[g] : 0;
    const double cx = live ? geom[4 * (int64_t)g] : 0.0, cy = live ? geom[4 * (int64_t)g + 1] : 0.0;
    double acc = 0.0;
    for (int e = lane; e < n; e += 32) {
        const int S = w_ids[b + e];
        const double dx = cx - geom[4 * (int64_t)S], dy = cy - geom[4 * (int64_t)S + 1];
        const double rs = geom[4 * (int64_t)S + 3];
        const double r2 = dx * dx + dy * dy;   // > 0: weak pairs are well separated
        const T* a = mp + 2 * (int64_t)S * p;
        acc += (double)a[0] * 0.5 * log(r2);
        const double2 u = make_double2(rs * dx / r2, -rs * dy / r2);   // rs_S / d
        double2 pw = u;
        for (int k = 1; k < p; ++k) {
            const double2 x = cmul(pw, make_double2((double)a[2 * k], (double)a[2 * k + 1]));
            acc -= x.x * kInvK.v[k];
            pw = cmul(pw, u);
        }
    }
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 32);
    if (live && lane == 0) c0[g] = acc;
}

// c0 of the boxes of one level += Re F_parent(centre): the parent's constant
// plus its local series (complete: M2L and L2L done) at the child's centre
template <class T>
__global__ void k_c0_shift(const int32_t* __restrict__ boxes, int n, const int32_t* __restrict__ parent,
                           const double* __restrict__ geom, const T* __restrict__ loc, int p, double* c0)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int g = boxes[i], P = parent[g];
    if (P < 0) return;
    const double rs = geom[4 * (int64_t)P + 3];
    double v = c0[P];
    if (rs > 0.0) {
        const double2 tau = make_double2((geom[4 * (int64_t)g] - geom[4 * (int64_t)P]) / rs,
                                         (geom[4 * (int64_t)g + 1] - geom[4 * (int64_t)P + 1]) / rs);
        const T* b = loc + 2 * (int64_t)P * p;
        double2 acc = make_double2(0.0, 0.0);
        for (int l = p - 1; l >= 0; --l) {
            acc = cmul(acc, tau);
            acc.x += (double)b[2 * l] / (l + 1);
            acc.y += (double)b[2 * l + 1] / (l + 1);
        }
        v += rs * cmul(acc, tau).x;
    }
    c0[g] += v;
}

// L2P of the logarithmic series at the points of every leaf (a workgroup of
// 64 per leaf), plus the near field, scattered to input order
template <class T>
__global__ void __launch_bounds__(64)
k_l2p_log(const int32_t* __restrict__ leaves, const int32_t* __restrict__ bstart, const int32_t* __restrict__ bcount,
          const double* __restrict__ geom, const double* __restrict__ X, const double* __restrict__ Y,
          const T* __restrict__ loc, int p, const double* __restrict__ c0, const double* __restrict__ near,
          const int32_t* __restrict__ perm, double* __restrict__ u)
{
    __shared__ double2 cf[kMaxP];
    const int g = leaves[blockIdx.x];
    const int st = bstart[g], n = bcount[g];
    const double cx = geom[4 * (int64_t)g], cy = geom[4 * (int64_t)g + 1], rs = geom[4 * (int64_t)g + 3];
    const T* b = loc + 2 * (int64_t)g * p;
    for (int l = threadIdx.x; l < p; l += 64)
        cf[l] = make_double2((double)b[2 * l] / (l + 1), (double)b[2 * l + 1] / (l + 1));
    __syncthreads();
    const double base = c0[g];
    for (int i = threadIdx.x; i < n; i += 64) {
        const int pos = st + i;
        double v = base;
        if (rs > 0.0) {
            const double2 w = make_double2((X[pos] - cx) / rs, (Y[pos] - cy) / rs);
            double2 acc = make_double2(0.0, 0.0);
            for (int l = p - 1; l >= 0; --l) {
                acc = cmul(acc, w);
                acc.x += cf[l].x;
                acc.y += cf[l].y;
            }
            v += rs * cmul(acc, w).x;
        }
        u[perm[pos]] = v + near[2 * (int64_t)pos];
    }
}

void launch_real_to_complex(int64_t n, const double* q, double* m, hipStream_t s)
{
    if (n == 0) return;
    k_real_to_complex<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, q, (double2*)m);
    check_launch("log strengths");
}

// the constant terms of every box: M2L part, then top-down shifts
template <class T>
void launch_log_constants(int nbox, const int32_t* w_beg, const int32_t* w_cnt, const int32_t* w_ids,
                          const double* geom, const void* mp, const void* loc, int p,
                          const int32_t* level_boxes, const std::vector<int64_t>& level_off, int nlevels,
                          const int32_t* parent, double* c0, hipStream_t s)
{
    if (nbox == 0) return;
    k_m2l_log0<T><<<(unsigned)((nbox + 7) / 8), 256, 0, s>>>(nbox, w_beg, w_cnt, w_ids, geom, (const T*)mp, p, c0);
    check_launch("log m2l constants");
    for (int l = 1; l < nlevels; ++l) {
        const int n = (int)(level_off[l + 1] - level_off[l]);
        if (n == 0) continue;
        k_c0_shift<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(level_boxes + level_off[l], n, parent, geom,
                                                                  (const T*)loc, p, c0);
        check_launch("log constant shift");
    }
}

template <class T>
void launch_l2p_log(const int32_t* leaves, int nleaf, const int32_t* bstart, const int32_t* bcount,
                    const double* geom, const double* X, const double* Y, const void* loc, int p, const double* c0,
                    const double* near, const int32_t* perm, double* u, hipStream_t s)
{
    if (nleaf == 0) return;
    k_l2p_log<T><<<(unsigned)nleaf, 64, 0, s>>>(leaves, bstart, bcount, geom, X, Y, (const T*)loc, p, c0, near, perm,
                                                u);
    check_launch("log l2p");
}

template void launch_log_constants<float>(int, const int32_t*, const int32_t*, const int32_t*, const double*,
                                          const void*, const void*, int, const int32_t*, const std::vector<int64_t>&,
                                          int, const int32_t*, double*, hipStream_t);
template void launch_log_constants<double>(int, const int32_t*, const int32_t*, const int32_t*, const double*,
                                           const void*, const void*, int, const int32_t*,
                                           const std::vector<int64_t>&, int, const int32_t*, double*, hipStream_t);
template void launch_l2p_log<float>(const int32_t*, int, const int32_t*, const int32_t*, const double*, const double*,
                                    const double*, const void*, int, const double*, const double*, const int32_t*,
                                    double*, hipStream_t);
template void launch_l2p_log<double>(const int32_t*, int, const int32_t*, const int32_t*, const double*,
                                     const double*, const double*, const void*, int, const double*, const double*,
                                     const int32_t*, double*, hipStream_t);

}  // namespace fmm
