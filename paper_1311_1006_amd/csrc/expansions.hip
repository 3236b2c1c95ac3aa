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
// mixed path).
#include "fmm_internal.h"
#include "kernels_common.h"

namespace fmm {

// strengths into tree order (with the tree's positions, the near field's
// sources)
__global__ void k_gather(int64_t n, const int32_t* __restrict__ perm, const double2* __restrict__ m, double2* mtree)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    mtree[i] = m[perm[i]];
}

__device__ __forceinline__ void wave_sync_e()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// P2M at the leaves.  G lanes per leaf (64/G leaves per wavefront, four
// wavefronts per workgroup): each lane takes the points j = lane, lane + G,
// ... of its leaf and accumulates the P terms m_j w_j^k, k = k0 .. k0+P-1
// (w_j = (z_j - c)/rs) in FP64 registers; a transposing butterfly then sums
// them over the G lanes.  P = 16 or 32; p > 32 takes two launches (k0 = 0
// and 32).
__device__ __forceinline__ double2 cpow(double2 b, int e)
{
    double2 r = make_double2(1.0, 0.0);
    while (e) {
        if (e & 1) r = cmul(r, b);
        b = cmul(b, b);
        e >>= 1;
    }
    return r;
}
__device__ __forceinline__ double rpow(double b, int e)
{
    double r = 1.0;
    while (e) {
        if (e & 1) r *= b;
        b *= b;
        e >>= 1;
    }
    return r;
}

// P2M (and with LEAF_M2M, G = 16, the M2M of the leaves' parents: a
// wavefront holds four leaves, which are one sibling group when every
// problem has the same depth; it then forms their parent's expansion with
// the lane layout and the operations of k_m2m, from the children's
// coefficients rounded to the storage type as k_m2m reads them, so that the
// result does not depend on which kernel forms it).
template <class T, int G, int P, bool LEAF_M2M, bool GATHER>
__global__ void __launch_bounds__(256)
k_p2m(const int32_t* __restrict__ leaves, int nleaf, const int32_t* __restrict__ bstart,
      const int32_t* __restrict__ bcount, const double* __restrict__ geom, const double* __restrict__ X,
      const double* __restrict__ Y, const double2* __restrict__ mt, int p, int k0, T* mp,
      const int32_t* __restrict__ parent, const double* __restrict__ binom, GatherOut go)
{
    static_assert(!LEAF_M2M || G == 16, "a sibling group per wavefront needs 16 lanes per leaf");
    constexpr int V = 2 * P;
    const int lane = threadIdx.x & 63;
    const int li = (blockIdx.x * 4 + (threadIdx.x >> 6)) * (64 / G) + lane / G;
    const int sl = lane % G;
    const bool valid = li < nleaf;
    int g = 0, st = 0, n = 0;
    double cx = 0.0, cy = 0.0, inv = 0.0;
    if (valid) {
        g = leaves[li];
        st = bstart[g];
        n = bcount[g];
        cx = geom[4 * (int64_t)g];
        cy = geom[4 * (int64_t)g + 1];
        inv = 1.0 / geom[4 * (int64_t)g + 3];
    }
    double v[V];
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] = 0.0;
    for (int j = sl; j < n; j += G) {
        const int i = st + j;
        double2 w, t;
        if constexpr (GATHER) {
            // the gather's outputs for this point, as k_gather writes them
            const double2 mm = go.m[go.perm[i]];
            const double x = X[i], y = Y[i];
            go.mtree[i] = mm;
            w = make_double2((x - cx) * inv, (y - cy) * inv);
            t = mm;
        } else {
            w = make_double2((X[i] - cx) * inv, (Y[i] - cy) * inv);
            t = mt[i];
        }
        if (k0 != 0) t = cmul(t, cpow(w, k0));   // the block of terms from k0 on
#pragma unroll
        for (int k = 0; k < P; ++k) {
            v[2 * k] += t.x;
            v[2 * k + 1] += t.y;
            if (k + 1 < P) t = cmul(t, w);
        }
    }
    treduce<V, G>(v, lane);
    const int base = treduce_base<V, G>(sl);
    constexpr int NV = V >= G ? V / G : 1;
    const bool writer = V >= G || (sl & (G / V - 1)) == 0;
    if (valid && writer) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int idx = base + i, k = k0 + (idx >> 1);
            if (k < p) mp[2 * ((int64_t)g * p + k) + (idx & 1)] = (T)v[i];
        }
    }
    if constexpr (LEAF_M2M) {
        __shared__ double2 coef[4][4][P], tau[4][4][P], part[4][4][P];
        __shared__ double rho[4][4][P];
        const int w = threadIdx.x >> 6, c = lane >> 4, j0 = lane & 15;
        if (valid && writer) {
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const int idx = base + i, k = idx >> 1;
                if (k < p) {
                    const double val = (double)(T)v[i];
                    if (idx & 1) coef[w][c][k].y = val;
                    else coef[w][c][k].x = val;
                }
            }
        }
        int pg = 0;
        if (valid) {            // the four leaves of the wavefront are valid together
            pg = parent[g];
            const double* gp = geom + 4 * (int64_t)pg;
            const double prs = gp[3];
            const double r = geom[4 * (int64_t)g + 3] / prs;
            const double2 t = make_double2((cx - gp[0]) / prs, (cy - gp[1]) / prs);
            for (int j = j0; j < p; j += 16) {
                tau[w][c][j] = cpow(t, j);
                rho[w][c][j] = rpow(r, j);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (valid) {
            for (int k = j0; k < p; k += 16) {
                double2 acc = make_double2(0, 0);
                for (int l = 0; l <= k; ++l) {
                    double s = binom[k * kBinomStride + l] * rho[w][c][l];
                    double2 vv = cmul(coef[w][c][l], tau[w][c][k - l]);
                    acc.x += s * vv.x;
                    acc.y += s * vv.y;
                }
                part[w][c][k] = acc;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (valid) {
            for (int k = lane; k < p; k += 64) {
                double2 v0 = part[w][0][k], v1 = part[w][1][k], v2 = part[w][2][k], v3 = part[w][3][k];
                mp[2 * ((int64_t)pg * p + k)] = (T)(((v0.x + v1.x) + v2.x) + v3.x);
                mp[2 * ((int64_t)pg * p + k) + 1] = (T)(((v0.y + v1.y) + v2.y) + v3.y);
            }
        }
    }
}


// M2M into one parent from its four children.  Lane (c, j): c = lane/16
// child, j = lane%16 (+16 for p > 16).  The children's coefficients and the
// powers rho_c^j, tau_c^j are staged in LDS; each lane forms one child's
// contribution to one coefficient; the four contributions are added in child
// order.
template <class T>
__global__ void __launch_bounds__(64)
k_m2m(const int32_t* __restrict__ parents, const int32_t* __restrict__ child0, const double* __restrict__ geom,
      const double* __restrict__ binom, int p, T* mp)
{
    __shared__ double2 coef[4][kMaxP], tau[4][kMaxP], part[4][kMaxP];
    __shared__ double rho[4][kMaxP];
    const int P = parents[blockIdx.x];
    const int lane = threadIdx.x, c = lane >> 4, j0 = lane & 15;
    const int ch = child0[P] + c;
    const double* gp = geom + 4 * (int64_t)P;
    const double* gc = geom + 4 * (int64_t)ch;
    const double prs = gp[3];
    const double r = gc[3] / prs;
    const double2 t = make_double2((gc[0] - gp[0]) / prs, (gc[1] - gp[1]) / prs);
    const T* a = mp + 2 * (int64_t)ch * p;
    for (int j = j0; j < p; j += 16) {
        coef[c][j] = make_double2((double)a[2 * j], (double)a[2 * j + 1]);
        tau[c][j] = cpow(t, j);
        rho[c][j] = rpow(r, j);
    }
    __syncthreads();
    for (int k = j0; k < p; k += 16) {
        double2 acc = make_double2(0, 0);
        for (int l = 0; l <= k; ++l) {
            double s = binom[k * kBinomStride + l] * rho[c][l];
            double2 v = cmul(coef[c][l], tau[c][k - l]);
            acc.x += s * v.x;
            acc.y += s * v.y;
        }
        part[c][k] = acc;
    }
    __syncthreads();
    for (int k = lane; k < p; k += 64) {
        double2 v0 = part[0][k], v1 = part[1][k], v2 = part[2][k], v3 = part[3][k];
        mp[2 * ((int64_t)P * p + k)] = (T)(((v0.x + v1.x) + v2.x) + v3.x);
        mp[2 * ((int64_t)P * p + k) + 1] = (T)(((v0.y + v1.y) + v2.y) + v3.y);
    }
}

// L2L from one parent into its four children (lane (c, l) as in k_m2m)
template <class T>
__global__ void __launch_bounds__(64)
k_l2l(const int32_t* __restrict__ parents, const int32_t* __restrict__ child0, const double* __restrict__ geom,
      const double* __restrict__ binom, int p, T* loc)
{
    __shared__ double2 bp[kMaxP], tau[4][kMaxP];
    const int P = parents[blockIdx.x];
    const int lane = threadIdx.x, c = lane >> 4, j0 = lane & 15;
    const int ch = child0[P] + c;
    const double* gp = geom + 4 * (int64_t)P;
    const double* gc = geom + 4 * (int64_t)ch;
    const double prs = gp[3];
    const double r = gc[3] / prs;
    const double2 t = make_double2((gc[0] - gp[0]) / prs, (gc[1] - gp[1]) / prs);
    const T* b = loc + 2 * (int64_t)P * p;
    for (int j = lane; j < p; j += 64) bp[j] = make_double2((double)b[2 * j], (double)b[2 * j + 1]);
    for (int j = j0; j < p; j += 16) tau[c][j] = cpow(t, j);
    __syncthreads();
    for (int l = j0; l < p; l += 16) {
        double2 acc = make_double2(0, 0);
        for (int k = l; k < p; ++k) {
            double s = binom[k * kBinomStride + l];
            double2 v = cmul(bp[k], tau[c][k - l]);
            acc.x += s * v.x;
            acc.y += s * v.y;
        }
        double rl = rpow(r, l);
        T* o = loc + 2 * ((int64_t)ch * p + l);
        o[0] = (T)((double)o[0] + rl * acc.x);
        o[1] = (T)((double)o[1] + rl * acc.y);
    }
}

// L2P at the leaves, plus the near field, scattered to input order.  G
// lanes per leaf as in P2M; every lane holds the leaf's P coefficients (FP64)
// and evaluates the series by Horner's rule at its points.
// L2P (and with LEAF_L2L the L2L from the leaf's parent first: lane l of
// the leaf's group forms rho^l sum_{k>=l} C(k, l) b_k(parent) tau^(k-l) with
// the operations of k_l2l, adds it to coefficient l and stores the
// completed coefficient, so that the leaf's local expansion in `loc` is
// whole afterwards; the group shares the coefficients through LDS).
template <class T, int G, int P, bool LEAF_L2L>
__global__ void __launch_bounds__(256)
k_l2p(const int32_t* __restrict__ leaves, int nleaf, const int32_t* __restrict__ bstart,
      const int32_t* __restrict__ bcount, const double* __restrict__ geom, const double* __restrict__ X,
      const double* __restrict__ Y, T* loc, int p, const double2* __restrict__ nearf,
      const int32_t* __restrict__ perm, double2* phi, double2* phi_near, double2* phi_far,
      const long long* __restrict__ guard, const int32_t* __restrict__ parent, const double* __restrict__ binom)
{
    if (guard != nullptr && *guard != 0) return;   // lists flagged: this launch is void
    using T2 = typename Vec2<T>::type;
    // P = 64: the coefficients stay in LDS (64 complex FP64 values would
    // take every register of a lane); below that they go to registers
    constexpr bool kLdsCoef = P > 32;
    __shared__ double2 sco[LEAF_L2L || kLdsCoef ? 256 / G : 1][LEAF_L2L || kLdsCoef ? P : 1];
    __shared__ double2 stau[LEAF_L2L ? 256 / G : 1][LEAF_L2L ? P : 1];
    const int lane = threadIdx.x & 63;
    const int li = (blockIdx.x * 4 + (threadIdx.x >> 6)) * (64 / G) + lane / G;
    const int sl = lane % G;
    if (li >= nleaf) return;
    const int g = leaves[li];
    const int st = bstart[g], n = bcount[g];
    const double cx = geom[4 * (int64_t)g], cy = geom[4 * (int64_t)g + 1], inv = 1.0 / geom[4 * (int64_t)g + 3];
    T2* b = reinterpret_cast<T2*>(loc) + (int64_t)g * p;
    double2 bl[kLdsCoef ? 1 : P];
    double2* co = sco[(LEAF_L2L || kLdsCoef) ? threadIdx.x / G : 0];
    if constexpr (LEAF_L2L) {
        const int pg = parent[g];
        const double prs = geom[4 * (int64_t)pg + 3];
        const double rho = geom[4 * (int64_t)g + 3] / prs;
        const double2 tau = make_double2((cx - geom[4 * (int64_t)pg]) / prs, (cy - geom[4 * (int64_t)pg + 1]) / prs);
        const T2* bp = reinterpret_cast<const T2*>(loc) + (int64_t)pg * p;
        double2* tp = stau[threadIdx.x / G];
        for (int j = sl; j < p; j += G) tp[j] = cpow(tau, j);   // the table of k_l2l
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int l = sl; l < p; l += G) {
            // the operations of k_l2l, in its order, so that the result does not
            // depend on which of the two kernels hands the expansion over
            double2 acc = make_double2(0, 0);
            for (int k = l; k < p; ++k) {
                const T2 bk = bp[k];
                double s = binom[k * kBinomStride + l];
                double2 v = cmul(make_double2((double)bk.x, (double)bk.y), tp[k - l]);
                acc.x += s * v.x;
                acc.y += s * v.y;
            }
            const double rl = rpow(rho, l);
            const T2 own = b[l];
            const T tx = (T)((double)own.x + rl * acc.x), ty = (T)((double)own.y + rl * acc.y);
            b[l] = T2{tx, ty};
            co[l] = make_double2((double)tx, (double)ty);
        }
        if constexpr (kLdsCoef)
            for (int l = p + sl; l < P; l += G) co[l] = make_double2(0.0, 0.0);
        // the group lies in one wavefront
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if constexpr (!kLdsCoef) {
#pragma unroll
            for (int k = 0; k < P; ++k) bl[k] = k < p ? co[k] : make_double2(0.0, 0.0);
        }
    } else if constexpr (kLdsCoef) {
        for (int k = sl; k < P; k += G) {
            if (k < p) { const T2 v = b[k]; co[k] = make_double2((double)v.x, (double)v.y); }
            else co[k] = make_double2(0.0, 0.0);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
#pragma unroll
        for (int k = 0; k < P; ++k) {
            if (k < p) { const T2 v = b[k]; bl[k] = make_double2((double)v.x, (double)v.y); }
            else bl[k] = make_double2(0.0, 0.0);
        }
    }
    for (int j = sl; j < n; j += G) {
        const int i = st + j;
        const double2 w = make_double2((X[i] - cx) * inv, (Y[i] - cy) * inv);
        double2 acc;
        if constexpr (kLdsCoef) {
            acc = co[P - 1];
            for (int l = P - 2; l >= 0; --l) {
                acc = cmul(acc, w);
                acc.x += co[l].x;
                acc.y += co[l].y;
            }
        } else {
            acc = bl[P - 1];
#pragma unroll
            for (int l = P - 2; l >= 0; --l) {
                acc = cmul(acc, w);
                acc.x += bl[l].x;
                acc.y += bl[l].y;
            }
        }
        const double2 nf = nearf[i];
        const int o = perm[i];
        if (phi) phi[o] = make_double2(acc.x + nf.x, acc.y + nf.y);
        if (phi_near) phi_near[o] = nf;
        if (phi_far) phi_far[o] = acc;
    }
}

// ------------------------------------------------------------ launchers

void launch_gather(int64_t n, const int32_t* perm, const double* m, double* mtree, hipStream_t s)
{
    k_gather<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, perm, (const double2*)m, (double2*)mtree);
    check_launch("gather");
}

// lanes per leaf: the smallest of 16, 32, 64 not below the largest leaf
static int leaf_lanes(int leaf_max) { return leaf_max <= 16 ? 16 : (leaf_max <= 32 ? 32 : 64); }

template <class T>
void launch_p2m(const int32_t* leaves, int nleaf, const int32_t* bstart, const int32_t* bcount, int leaf_max,
                const double* geom, const double* X, const double* Y, const double* mt, int p, void* mp,
                hipStream_t s, const int32_t* parent, const double* binom, const GatherOut* go)
{
    const GatherOut none{};
    const GatherOut& gg = go ? *go : none;
    if (nleaf == 0) return;
    if (p > 32 && parent) throw Error(FMM_EINVAL, "P2M with the leaves' M2M needs p <= 32");
    const int G = leaf_lanes(leaf_max);
    const int PB = p <= 16 ? 16 : 32;
    const unsigned grid = (unsigned)((nleaf + 4 * (64 / G) - 1) / (4 * (64 / G)));
    // blocks of PB terms: the first one does the gather, the second (p > 32)
    // reads the strengths it put into tree order
    for (int k0 = 0; k0 < p; k0 += PB) {
        const bool gat = go && k0 == 0;
        const double2* mtk = (const double2*)(k0 == 0 ? mt : (go ? (const double*)go->mtree : mt));
#define P2M_CASE(G_, P_)                                                                                   \
    if (G == G_ && PB == P_) {                                                                            \
        if constexpr (G_ == 16)                                                                           \
            if (parent) {                                                                                 \
                if (gat)                                                                                  \
                    k_p2m<T, G_, P_, true, true><<<grid, 256, 0, s>>>(leaves, nleaf, bstart, bcount, geom, X, \
                        Y, mtk, p, k0, (T*)mp, parent, binom, gg);                                        \
                else                                                                                      \
                    k_p2m<T, G_, P_, true, false><<<grid, 256, 0, s>>>(leaves, nleaf, bstart, bcount, geom, X, \
                        Y, mtk, p, k0, (T*)mp, parent, binom, gg);                                        \
                check_launch("p2m");                                                                      \
                continue;                                                                                 \
            }                                                                                             \
        if (gat)                                                                                          \
            k_p2m<T, G_, P_, false, true><<<grid, 256, 0, s>>>(leaves, nleaf, bstart, bcount, geom, X, Y, \
                mtk, p, k0, (T*)mp, nullptr, nullptr, gg);                                                \
        else                                                                                              \
            k_p2m<T, G_, P_, false, false><<<grid, 256, 0, s>>>(leaves, nleaf, bstart, bcount, geom, X, Y, \
                mtk, p, k0, (T*)mp, nullptr, nullptr, gg);                                                \
        check_launch("p2m");                                                                              \
        continue;                                                                                         \
    }
        P2M_CASE(16, 16) P2M_CASE(32, 16) P2M_CASE(64, 16) P2M_CASE(16, 32) P2M_CASE(32, 32) P2M_CASE(64, 32)
#undef P2M_CASE
        throw Error(FMM_EINVAL, "unsupported P2M configuration");
    }
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
void launch_l2l(const int32_t* parents, int n, const int32_t* child0, const double* geom, const double* binom,
                int p, void* loc, hipStream_t s)
{
    if (n == 0) return;
    k_l2l<T><<<n, 64, 0, s>>>(parents, child0, geom, binom, p, (T*)loc);
    check_launch("l2l");
}

template <class T>
void launch_l2p(const int32_t* leaves, int nleaf, const int32_t* bstart, const int32_t* bcount, int leaf_max,
                const double* geom, const double* X, const double* Y, void* loc, int p,
                const double* nearf, const int32_t* perm, double* phi, double* phi_near, double* phi_far,
                hipStream_t s, const long long* guard, const int32_t* parent, const double* binom)
{
    if (nleaf == 0) return;
    const int G = leaf_lanes(leaf_max);
    const unsigned grid = (unsigned)((nleaf + 4 * (64 / G) - 1) / (4 * (64 / G)));
#define L2P_CASE(G_, P_)                                                                                   \
    if (G == G_ && (p <= 16 ? 16 : (p <= 32 ? 32 : 64)) == P_) {                                          \
        if (parent)                                                                                       \
            k_l2p<T, G_, P_, true><<<grid, 256, 0, s>>>(leaves, nleaf, bstart, bcount, geom, X, Y, (T*)loc, p, \
                                                        (const double2*)nearf, perm, (double2*)phi,       \
                                                        (double2*)phi_near, (double2*)phi_far, guard,     \
                                                        parent, binom);                                   \
        else                                                                                              \
            k_l2p<T, G_, P_, false><<<grid, 256, 0, s>>>(leaves, nleaf, bstart, bcount, geom, X, Y, (T*)loc, p, \
                                                         (const double2*)nearf, perm, (double2*)phi,      \
                                                         (double2*)phi_near, (double2*)phi_far, guard,    \
                                                         nullptr, nullptr);                               \
        check_launch("l2p");                                                                              \
        return;                                                                                           \
    }
    L2P_CASE(16, 16) L2P_CASE(32, 16) L2P_CASE(64, 16) L2P_CASE(16, 32) L2P_CASE(32, 32) L2P_CASE(64, 32)
    L2P_CASE(16, 64) L2P_CASE(32, 64) L2P_CASE(64, 64)
#undef L2P_CASE
    throw Error(FMM_EINVAL, "unsupported L2P configuration");
}

#define INST(T)                                                                                          \
    template void launch_p2m<T>(const int32_t*, int, const int32_t*, const int32_t*, int, const double*, \
                                const double*, const double*, const double*, int, void*, hipStream_t,    \
                                const int32_t*, const double*, const GatherOut*);                        \
    template void launch_m2m<T>(const int32_t*, int, const int32_t*, const double*, const double*, int,  \
                                void*, hipStream_t);                                                     \
    template void launch_l2l<T>(const int32_t*, int, const int32_t*, const double*, const double*, int,  \
                                void*, hipStream_t);                                                     \
    template void launch_l2p<T>(const int32_t*, int, const int32_t*, const int32_t*, int, const double*, \
                                const double*, const double*, void*, int, const double*,                 \
                                const int32_t*, double*, double*, double*, hipStream_t,                  \
                                const long long*, const int32_t*, const double*);
INST(double)
INST(float)
#undef INST

}  // namespace fmm
