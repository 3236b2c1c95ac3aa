// points.hip -- the field of the sources at evaluation points apart from them
// (eq. 2.2), from a plan over the sources' tree (Sec. 2.1, 2.2).
//
// A point y goes down the tree from the root, at every level into the child
// whose disc (centre c, radius r: the disc around the tight bounding box that
// the theta-criterion (2.3) is stated for) holds it with the smallest
// |y - c| / r, as deep as it can: box B.  The complete local expansion of B
// (after the M2L and L2L sweep over every level) holds the field of every
// source outside the boxes of B's strong list -- at every level the strong
// and weak lists of a box and of its ancestors partition the sources -- and
// it converges at y with the bound of the sources' own evaluation, because y
// lies in the disc of B and of each of its ancestors, the discs whose radii
// entered the theta-criterion of those M2L shifts.  The discs overlap and
// cover the gaps between the tight boxes, so nearly every point among the
// sources reaches a leaf.
//
// When B is a leaf, the sources of its strong list (leaves) are summed
// directly, as for the sources of B, so the point's value has the accuracy
// of theirs.  Otherwise (a point outside the discs of B's children) every box
// of B's strong list is descended: a box well separated from the point
// contributes its multipole expansion at y, a leaf that is not contributes
// its points directly, any other box is opened.
// "Well separated" is the criterion (2.3) between the box and a box of the
// same radius r around the point, r (1 + theta) <= theta d (squared, every
// operation rounded alone as in the list build), so that these expansions
// are used at the distances the M2L shifts of the plan use them.  The root
// is always opened (no list needs its multipole expansion, so the upward
// pass stops at level 1): a point outside every disc of level 1 gets its
// whole field from the descent of the root.  A source at y's position is
// left out, as (2.2) says.  The points join neither the tree nor the lists,
// so they change nothing of the sources' own evaluation.
//
// Expansions are the scaled ones of expansions.hip (a_k = sum m_j w_j^k,
// w_j = (z_j - c)/rs; phi(z) = sum b_l ((z - c)/rs)^l), so with u = rs/(y - c)
//     multipole at y:  (u/rs) sum_k a_k u^k,
//     its derivative:  -(u/rs)^2 sum_k (k+1) a_k u^k.
// Coefficients are read in their storage type and used in FP64; the direct
// sums of the mixed path are FP32 with the double-float difference of the
// near-field kernel.
//
// The points are sorted by B (a counting sort: count, scan, scatter).  The
// near field of the points in leaves is the near-field kernel of the sources
// (p2p.hip) with the points as its targets: sources of the leaf's strong list
// staged in LDS, a lane subgroup per few points.  The descents run a
// wavefront per point, lanes over the boxes of a frontier.  The far field is
// one lane per point.  With the derivative, every point's near field is a
// descent (whose first frontier, for a point in a leaf, is summed directly).
#include <algorithm>
#include <cfloat>
#include <type_traits>

#include "fmm_internal.h"
#include "kernels_common.h"

namespace fmm {

void far_field_all(Plan& pl, const double* m, hipStream_t s);
void launch_exclusive_scan(const int32_t* v, int n, int32_t* bsum, int32_t* out, hipStream_t s);

// near-field work items over the points: at most kPtsItem points of one box
// each, for the (4 targets per lane, 4 subgroups) shape
constexpr int kPtsItem = 16;
struct PtsItem {
    int32_t leaf, t0, tn, pad;
};

__global__ void k_pts_clear(int32_t* a, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0;
}

// the deepest box whose disc (centre c, radius r: the disc of the
// theta-criterion, around the tight bounding box) holds each point, going
// down from the root into the child that holds it with the smallest
// |y - c| / r, the points per box and each point's rank among its box's
// points (the order the counter gave them).  The geometry of levels 1 ..
// kLocTop is read from a copy in LDS (the first kLocTop of a point's
// dependent loads), deeper levels from the tree.
constexpr int kLocTop = 4;
constexpr int kLocTopBoxes = 340;   // boxes of levels 1 .. kLocTop
__device__ __forceinline__ void locate_child(const double2 q, const double* g, int k, int& best, double& bq)
{
    const double dx = q.x - g[0], dy = q.y - g[1];
    const double d2 = dx * dx + dy * dy, r2 = g[2] * g[2];
    if (!(d2 <= r2)) return;                                // outside (a zero-radius disc holds its centre)
    const double qk = r2 > 0.0 ? d2 / r2 : 0.0;
    if (qk < bq) {
        bq = qk;
        best = k;
    }
}
__global__ void __launch_bounds__(256)
k_pts_locate(const double2* __restrict__ y, int64_t M, int L, const double* __restrict__ geom, int32_t* box,
             int32_t* cnt, int32_t* rank)
{
    static_assert(kLocTopBoxes == ((4 << (2 * kLocTop)) - 1) / 3 - 1, "levels 1 .. kLocTop");
    __shared__ double sg[kLocTopBoxes][3];
    const int top = L - 1 < kLocTop ? L - 1 : kLocTop;     // levels cached
    const int ntop = (int)(level_base(top + 1) - 1);
    for (int t = threadIdx.x; t < ntop; t += blockDim.x) {
        const double* g = geom + 4 * (int64_t)(t + 1);
        sg[t][0] = g[0];
        sg[t][1] = g[1];
        sg[t][2] = g[2];
    }
    __syncthreads();
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= M) return;
    const double2 q = y[i];
    int64_t b = 0, j = 0;
    for (int l = 0; l + 1 < L; ++l) {
        const int64_t c0 = level_base(l + 1) + 4 * j;
        int best = -1;
        double bq = 2.0;     // the smallest (|y - c| / r)^2 so far; at most 1 inside a disc
        if (l + 1 <= top) {
            for (int k = 0; k < 4; ++k) locate_child(q, sg[c0 + k - 1], k, best, bq);
        } else {
            for (int k = 0; k < 4; ++k) locate_child(q, geom + 4 * (c0 + k), k, best, bq);
        }
        if (best < 0) break;
        b = c0 + best;
        j = 4 * j + best;
    }
    box[i] = (int32_t)b;
    rank[i] = atomicAdd(&cnt[b], 1);
}

// sorted position of every point: its box's offset plus its rank in the box
// (the order inside a box is immaterial: each point's value depends on its
// own position only)
__global__ void k_pts_scatter(const int32_t* __restrict__ box, int64_t M, const int32_t* __restrict__ off,
                              const int32_t* __restrict__ rank, int32_t* order)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= M) return;
    order[off[box[i]] + rank[i]] = (int32_t)i;
}

// the points' positions in box order, as the near-field kernel reads its
// targets (x[], y[])
__global__ void k_pts_records(const double2* __restrict__ y, int64_t M, const int32_t* __restrict__ order,
                              double* rx, double* ry)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= M) return;
    const double2 v = y[order[q]];
    rx[q] = v.x;
    ry[q] = v.y;
}

// items per leaf: the leaf's points in groups of kPtsItem
__global__ void k_pts_item_counts(int64_t lb, int nleaf, const int32_t* __restrict__ cnt, int32_t* icnt)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < nleaf) icnt[j] = (cnt[lb + j] + kPtsItem - 1) / kPtsItem;
}

__global__ void k_pts_items(int64_t lb, int nleaf, const int32_t* __restrict__ cnt, const int32_t* __restrict__ ioff,
                            PtsItem* items)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nleaf) return;
    const int c = cnt[lb + j];
    for (int t0 = 0, k = ioff[j]; t0 < c; t0 += kPtsItem, ++k)
        items[k] = PtsItem{(int32_t)(lb + j), t0, min(kPtsItem, c - t0), 0};
}

// point criterion: a box of radius r at squared distance d2 is well separated
// from a point when r^2 <= t^2 d2 (d2 > 0), t = theta / (1 + theta)
__device__ __forceinline__ bool point_separated(double r, double dx, double dy, double theta)
{
#pragma clang fp contract(off)     // every product and sum rounded alone, as in the list build
    const double d2 = ((dx * dx) + (dy * dy));
    const double rr = (r * r);
    return (d2 > 0.0) && (rr <= ((theta * theta) * d2));
}

template <class T>
__device__ __forceinline__ double2 coef(const T* c, int k)
{
    return make_double2((double)c[2 * k], (double)c[2 * k + 1]);
}

// multipole expansion of a box at the point: phi += (u/rs) sum a_k u^k and
// dphi -= (u/rs)^2 sum (k+1) a_k u^k, u = rs/(y - c)
template <class T, bool DER>
__device__ __forceinline__ void m2p(const T* a, int p, double rs, double dx, double dy, double2& phi, double2& dphi)
{
    const double id = 1.0 / (dx * dx + dy * dy);
    const double2 inv = make_double2(dx * id, -dy * id);       // 1 / (y - c)
    const double2 u = make_double2(rs * inv.x, rs * inv.y);
    double2 s = coef(a, p - 1), t = make_double2((double)p * s.x, (double)p * s.y);
    for (int k = p - 2; k >= 0; --k) {
        const double2 ak = coef(a, k);
        s = cmul(s, u);
        s.x += ak.x;
        s.y += ak.y;
        if (DER) {
            t = cmul(t, u);
            t.x += (double)(k + 1) * ak.x;
            t.y += (double)(k + 1) * ak.y;
        }
    }
    const double2 f = cmul(s, inv);
    phi.x += f.x;
    phi.y += f.y;
    if (DER) {
        const double2 g = cmul(t, cmul(inv, inv));
        dphi.x -= g.x;
        dphi.y -= g.y;
    }
}

// the points of one leaf, directly: phi += m/(y - x), dphi -= m/(y - x)^2
template <bool DER>
__device__ __forceinline__ void direct64(const double* __restrict__ X, const double* __restrict__ Y,
                                         const double2* __restrict__ mt, int st, int n, double yx, double yy,
                                         double2& phi, double2& dphi)
{
#pragma unroll 8
    for (int q = 0; q < n; ++q) {         // unrolled: eight loads in flight
        const double2 m = mt[st + q];
        const double4 sv = make_double4(X[st + q], Y[st + q], m.x, m.y);   // x, y, Re m, Im m
        const double dx = yx - sv.x, dy = yy - sv.y;
        const double r2 = dx * dx + (dy * dy + DBL_MIN);     // 0/DBL_MIN: a coincident source adds 0
        const double id = 1.0 / r2;
        const double a = sv.z * dx + sv.w * dy, b = sv.w * dx - sv.z * dy;   // m conj(y - x)
        phi.x += a * id;
        phi.y += b * id;
        if (DER) {
            // m conj(y - x)^2 / |y - x|^4, as (c id) id: a coincident source
            // (c = d = 0) adds 0, not 0 * inf
            const double c = a * dx + b * dy, d = b * dx - a * dy;
            dphi.x -= (c * id) * id;
            dphi.y -= (d * id) * id;
        }
    }
}

// (the difference in FP64 rounded once to FP32, the strengths rounded to
// FP32, as in the near-field kernel)
template <bool DER>
__device__ __forceinline__ void direct32(const double* __restrict__ X, const double* __restrict__ Y,
                                         const double2* __restrict__ mt, int st, int n, double yx, double yy,
                                         float2& phi, float2& dphi)
{
    // unrolled by four: with eight sources' loads in flight the descent kernel
    // held 129 vector registers (3 wavefronts per SIMD) and ran 1.6x longer
#pragma unroll 4
    for (int q = 0; q < n; ++q) {
        const double2 m = mt[st + q];
        const float mr = (float)m.x, mi = (float)m.y;
        const float dx = (float)(yx - X[st + q]);
        const float dy = (float)(yy - Y[st + q]);
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, FLT_MIN));
        const float id = __builtin_amdgcn_rcpf(r2);
        const float a = fmaf(mr, dx, mi * dy), b = fmaf(mi, dx, -(mr * dy));
        phi.x = fmaf(a, id, phi.x);
        phi.y = fmaf(b, id, phi.y);
        if (DER) {
            // (c id) id: a coincident source (c = d = 0) adds 0, not 0 * inf
            const float c = fmaf(a, dx, b * dy), d = fmaf(b, dx, -(a * dy));
            dphi.x = fmaf(-(c * id), id, dphi.x);
            dphi.y = fmaf(-(d * id), id, dphi.y);
        }
    }
}

// What a box adds to a point's near field: its multipole expansion when it
// is well separated from the point (never the root, which has none), its
// points when it is a leaf; returns false (nothing added) when the box must
// be opened.  The mixed direct sums go to FP32 accumulators (nf, nd).
template <class T, bool DER>
struct Visit {
    double2 y;
    int L, p;
    double theta;
    const int8_t* level;
    const double* geom;
    const int32_t *bstart, *bcount;
    const T* mpole;
    const double *X, *Y;            // the sources: positions and strengths in tree order
    const double2* mt;

    __device__ __forceinline__ bool operator()(int32_t bx, int lv, double2& phi, double2& dphi, float2& nf,
                                               float2& nd, bool direct = false) const
    {
        const double* g = geom + 4 * (int64_t)bx;
        const double dx = y.x - g[0], dy = y.y - g[1];
        if (!direct && lv > 0 && point_separated(g[2], dx, dy, theta)) {
            m2p<T, DER>(mpole + 2 * (int64_t)bx * p, p, g[3], dx, dy, phi, dphi);
            return true;
        }
        if (lv != L - 1) return false;
        if constexpr (std::is_same<T, float>::value) direct32<DER>(X, Y, mt, bstart[bx], bcount[bx], y.x, y.y, nf, nd);
        else direct64<DER>(X, Y, mt, bstart[bx], bcount[bx], y.x, y.y, phi, dphi);
        return true;
    }

    // the whole subtree of box S, one box after the other (no stack: the
    // next box is the next sibling, or that of the nearest ancestor that has
    // one; done when back at S)
    __device__ void subtree(int32_t S, double2& phi, double2& dphi, float2& nf, float2& nd) const
    {
        int32_t cur = S;
        int lv = level[S];
        while (true) {
            if (!(*this)(cur, lv, phi, dphi, nf, nd)) {
                cur = (int32_t)(level_base(lv + 1) + 4 * ((int64_t)cur - level_base(lv)));   // first child
                ++lv;
                continue;
            }
            bool done = false;
            while (true) {
                if (cur == S) { done = true; break; }
                const int64_t j = (int64_t)cur - level_base(lv);
                if ((j & 3) != 3) { ++cur; break; }
                cur = (int32_t)(level_base(lv - 1) + (j >> 2));
                --lv;
            }
            if (done) return;
        }
    }
};

constexpr int kFront = 512;   // frontier boxes per wavefront (LDS)

// The near field of the points at box-order positions q < nq by descents of
// their box's strong list: one wavefront per point, breadth first, lanes over
// the frontier (the first frontier is the strong list itself, read from the
// pool; later ones are in LDS).  A lane's box adds its expansion or its
// points, or puts its four children in the next frontier; a box whose
// children no longer fit is descended by its lane alone.  The lanes' sums
// are added by a fixed butterfly, so the result does not depend on timing.
// Results go to tnear (and tdnear) in box order.  A descent is a chain of
// dependent loads, so wavefronts in flight set its rate: the mixed kernel
// without the derivative is held to 80 registers (six wavefronts per SIMD,
// no spills); the others need 97-120 and would spill below that.
template <class T, bool DER>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && !DER ? 6 : 1)))
k_pts_descend(const double2* __restrict__ y, const int32_t* __restrict__ order, const int32_t* __restrict__ box,
              const int32_t* __restrict__ nq_dev, int nq_host, int L, const int8_t* __restrict__ level,
              const double* __restrict__ geom, const int32_t* __restrict__ bstart, const int32_t* __restrict__ bcount,
              const int32_t* __restrict__ s_beg, const int32_t* __restrict__ s_cnt, const int32_t* __restrict__ s_ids,
              const T* __restrict__ mpole, int p, double theta, const double* __restrict__ X,
              const double* __restrict__ Y, const double2* __restrict__ mt, double2* tnear, double2* tdnear)
{
    __shared__ int32_t front[4][2][kFront];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int nq = nq_dev ? *nq_dev : nq_host;
    const int nw = (int)gridDim.x * 4;
    for (int q = (int)blockIdx.x * 4 + w; q < nq; q += nw) {      // uniform in the wavefront
        const int32_t i = order[q];
        Visit<T, DER> vis;
        vis.y = y[i];
        vis.L = L; vis.p = p; vis.theta = theta; vis.level = level; vis.geom = geom;
        vis.bstart = bstart; vis.bcount = bcount; vis.mpole = mpole;
        vis.X = X; vis.Y = Y; vis.mt = mt;
        const int32_t B = box[i];
        double2 phi = make_double2(0.0, 0.0), dphi = make_double2(0.0, 0.0);
        float2 nf = make_float2(0.f, 0.f), nd = make_float2(0.f, 0.f);
        int32_t* cur = front[w][0];
        int32_t* nxt = front[w][1];
        const int e0 = s_beg[B];
        int n = s_cnt[B];
        bool first = true;
        // a point in a leaf sums the leaves of its strong list directly, as
        // the sources of that leaf do
        const bool in_leaf = level[B] == L - 1;
        while (n > 0) {
            int nn = 0;
            for (int c0 = 0; c0 < n; c0 += 64) {
                const int k = c0 + lane;
                int32_t bx = -1;
                if (k < n) bx = first ? s_ids[e0 + k] : cur[k];
                bool open = false;
                int lv = 0;
                if (bx >= 0) {
                    lv = level[bx];
                    open = !vis(bx, lv, phi, dphi, nf, nd, first && in_leaf);
                }
                const unsigned long long om = __ballot(open);
                if (open) {
                    const int pos = nn + 4 * __popcll(om & below);
                    if (pos + 4 <= kFront) {
                        const int32_t c = (int32_t)(level_base(lv + 1) + 4 * ((int64_t)bx - level_base(lv)));
                        for (int t = 0; t < 4; ++t) nxt[pos + t] = c + t;
                    } else {
                        vis.subtree(bx, phi, dphi, nf, nd);
                    }
                }
                nn = min(nn + 4 * __popcll(om), kFront);
            }
            wave_sync();
            int32_t* t = cur;
            cur = nxt;
            nxt = t;
            n = nn;
            first = false;
        }
        phi.x += (double)nf.x;
        phi.y += (double)nf.y;
        dphi.x += (double)nd.x;
        dphi.y += (double)nd.y;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            phi.x += __shfl_xor(phi.x, o, 64);
            phi.y += __shfl_xor(phi.y, o, 64);
            if (DER) {
                dphi.x += __shfl_xor(dphi.x, o, 64);
                dphi.y += __shfl_xor(dphi.y, o, 64);
            }
        }
        if (lane == 0) {
            tnear[q] = phi;
            if (DER) tdnear[q] = dphi;
        }
        wave_sync();
    }
}

// the far field of every point (B's local expansion; the root has none) plus
// its near field (tnear, box order), into the outputs in input order
template <class T, bool DER>
__global__ void __launch_bounds__(256)
k_pts_far(const double2* __restrict__ y, int64_t M, const int32_t* __restrict__ order, const int32_t* __restrict__ box,
          const int8_t* __restrict__ level, const double* __restrict__ geom, const T* __restrict__ local, int p,
          const double2* __restrict__ tnear, const double2* __restrict__ tdnear, double2* __restrict__ phi_out,
          double2* __restrict__ dphi_out)
{
    const int64_t qi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (qi >= M) return;
    const int32_t i = order[qi];
    const double2 yv = y[i];
    const int32_t B = box[i];
    double2 phi = tnear[qi], dphi = DER ? tdnear[qi] : make_double2(0.0, 0.0);
    if (level[B] > 0) {
        const double* g = geom + 4 * (int64_t)B;
        const double irs = 1.0 / g[3];
        const double2 w = make_double2((yv.x - g[0]) * irs, (yv.y - g[1]) * irs);
        const T* b = local + 2 * (int64_t)B * p;
        double2 s = coef(b, p - 1), t = make_double2((double)(p - 1) * s.x, (double)(p - 1) * s.y);
        for (int l = p - 2; l >= 0; --l) {
            const double2 bl = coef(b, l);
            s = cmul(s, w);
            s.x += bl.x;
            s.y += bl.y;
            if (DER && l >= 1) {
                t = cmul(t, w);
                t.x += (double)l * bl.x;
                t.y += (double)l * bl.y;
            }
        }
        phi.x += s.x;
        phi.y += s.y;
        if (DER && p > 1) {
            dphi.x += t.x * irs;
            dphi.y += t.y * irs;
        }
    }
    phi_out[i] = phi;
    if (DER) dphi_out[i] = dphi;
}

void evaluate_points_device(Plan& pl, const double* m, const double* y, int64_t M, double* phi, double* dphi,
                            hipStream_t s)
{
    Tree& t = *pl.tree;
    TreeSchedule& sc = *t.sched;
    if (sc.nprob != 1) throw Error(FMM_EINVAL, "evaluation points need a plan over a single problem");
    if (M < 0 || M >= INT32_MAX) throw Error(FMM_EINVAL, "the number of evaluation points must be in [0, 2^31 - 1)");
    if (M == 0) return;
    const bool mixed = pl.precision == FMM_MIXED, der = dphi != nullptr;
    const int L = sc.L[0];
    // the near field of a point in a leaf is the direct sum over the sources
    // of the leaf's strong list (the near-field kernel); a point stopped
    // higher up (outside the discs of the leaves, a few per cent of points
    // among the sources) descends its box's strong list instead, a wavefront
    // per point
    const int ld = L - 1;
    const int64_t nb = sc.nbox, lb = level_base(ld);
    const int nleaf = (int)(nb - lb);
    // a point takes a box's multipole expansion when the box would be well
    // separated from a box of its own radius around the point: r (1 + theta)
    // <= theta d, i.e. r <= theta' d with theta' = theta / (1 + theta); the
    // ratio r/d of every such expansion is then that of the M2L shifts of the
    // plan, and so is its truncation
    const double theta_pt = pl.theta / (1.0 + pl.theta);
    // item list: at most M / kPtsItem + nleaf items (spares have no target)
    const int64_t nx = M / kPtsItem + nleaf + 1;
    if (nx >= INT32_MAX / 4) throw Error(FMM_EINVAL, "too many evaluation points");
    DBuf<int32_t> box, rank, order, cnt, off, bsum, icnt, ioff;
    DBuf<double> rx, ry, tnear, tdnear;
    DBuf<PtsItem> items;
    box.alloc(M, s);
    rank.alloc(M, s);
    order.alloc(M, s);
    cnt.alloc(nb, s);
    off.alloc(nb + 1, s);
    bsum.alloc((std::max<int64_t>(nb, nleaf) + 1023) / 1024, s);
    if (!der) {
        icnt.alloc(nleaf, s);
        ioff.alloc(nleaf + 1, s);
        items.alloc(nx, s);
        rx.alloc(M, s);
        ry.alloc(M, s);
    }
    tnear.alloc(2 * M, s);
    if (der) tdnear.alloc(2 * M, s);
    far_field_all(pl, m, s);
    const unsigned gb = (unsigned)((nb + 255) / 256), gm = (unsigned)((M + 255) / 256);
    k_pts_clear<<<gb, 256, 0, s>>>(cnt.p, nb);
    k_pts_locate<<<gm, 256, 0, s>>>((const double2*)y, M, L, t.geom.p, box.p, cnt.p, rank.p);
    launch_exclusive_scan(cnt.p, (int)nb, bsum.p, off.p, s);
    k_pts_scatter<<<gm, 256, 0, s>>>(box.p, M, off.p, rank.p, order.p);
    check_launch("point order");
    if (!der) {
        // the near field of the points in leaves: the near-field kernel, with
        // the points as its targets and the sources of the leaf's strong list
        k_pts_records<<<gm, 256, 0, s>>>((const double2*)y, M, order.p, rx.p, ry.p);
        const unsigned gl = (unsigned)((nleaf + 255) / 256);
        k_pts_clear<<<(unsigned)((4 * nx + 255) / 256), 256, 0, s>>>((int32_t*)items.p, 4 * nx);
        k_pts_item_counts<<<gl, 256, 0, s>>>(lb, nleaf, cnt.p, icnt.p);
        launch_exclusive_scan(icnt.p, nleaf, bsum.p, ioff.p, s);
        k_pts_items<<<gl, 256, 0, s>>>(lb, nleaf, cnt.p, ioff.p, items.p);
        check_launch("point items");
        Targets tgt;
        tgt.x = rx.p;
        tgt.y = ry.p;
        tgt.start = off.p;
        launch_p2p(mixed, 4, 4, items.p, 0, nullptr, (int)nx, nullptr, nullptr, nullptr, sc.d_box_start.p,
                   sc.d_box_count.p, pl.s_beg.p, pl.s_cnt.p, pl.s_ids.p,
                   t.x.p, t.y.p, (const double2*)pl.mtree.p, tnear.p, s, nullptr, 0.0, false, tgt,
                   pl.tune.p2p_src_tile);
    }
    // descents: the points that stopped above the leaves (box-order positions
    // before the first leaf), or with the derivative every point
    // workgroups of the descents: those the occupancy holds at once (six
    // wavefronts per SIMD for the mixed kernel without the derivative, four
    // for the others)
    const unsigned gd = (unsigned)std::min<int64_t>((M + 3) / 4, mixed && !der ? 1536 : 1024);
    const int32_t* nq_dev = der ? nullptr : off.p + lb;
#define DESC_ARGS                                                                                             \
    (const double2*)y, order.p, box.p, nq_dev, (int)M, L, sc.d_box_level.p, t.geom.p, sc.d_box_start.p,       \
        sc.d_box_count.p, pl.s_beg.p, pl.s_cnt.p, pl.s_ids.p
#define FAR_ARGS (const double2*)y, M, order.p, box.p, sc.d_box_level.p, t.geom.p
#define SRC_ARGS t.x.p, t.y.p, (const double2*)pl.mtree.p
    double2* tn = (double2*)tnear.p;
    double2* td = der ? (double2*)tdnear.p : nullptr;
    if (mixed) {
        const float* mp = (const float*)pl.mpole.p;
        const float* lc = (const float*)pl.local.p;
        if (der) {
            k_pts_descend<float, true><<<gd, 256, 0, s>>>(DESC_ARGS, mp, pl.p, theta_pt, SRC_ARGS, tn, td);
            k_pts_far<float, true><<<gm, 256, 0, s>>>(FAR_ARGS, lc, pl.p, tn, td, (double2*)phi, (double2*)dphi);
        } else {
            k_pts_descend<float, false><<<gd, 256, 0, s>>>(DESC_ARGS, mp, pl.p, theta_pt, SRC_ARGS, tn, nullptr);
            k_pts_far<float, false><<<gm, 256, 0, s>>>(FAR_ARGS, lc, pl.p, tn, nullptr, (double2*)phi, nullptr);
        }
    } else {
        const double* mp = (const double*)pl.mpole.p;
        const double* lc = (const double*)pl.local.p;
        if (der) {
            k_pts_descend<double, true><<<gd, 256, 0, s>>>(DESC_ARGS, mp, pl.p, theta_pt, SRC_ARGS, tn, td);
            k_pts_far<double, true><<<gm, 256, 0, s>>>(FAR_ARGS, lc, pl.p, tn, td, (double2*)phi, (double2*)dphi);
        } else {
            k_pts_descend<double, false><<<gd, 256, 0, s>>>(DESC_ARGS, mp, pl.p, theta_pt, SRC_ARGS, tn, nullptr);
            k_pts_far<double, false><<<gm, 256, 0, s>>>(FAR_ARGS, lc, pl.p, tn, nullptr, (double2*)phi, nullptr);
        }
    }
#undef DESC_ARGS
#undef FAR_ARGS
#undef SRC_ARGS
    check_launch("points");
}

}  // namespace fmm
