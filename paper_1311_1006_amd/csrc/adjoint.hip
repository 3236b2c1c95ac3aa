// adjoint.hip -- gradients of a real loss through the FMM with the tree
// geometry (centres, radii, lists) frozen: the transposed chain.
//
// Convention: for complex w, G_w = dL/dRe(w) + i dL/dIm(w); input g = G_phi.
// The frozen-geometry FMM is phi = A(z) m, complex-linear in m and
// holomorphic in every z, hence with gb = conj(g)
//     G_m = conj(A^T gb)
//     G_z_k = conj( gb_k dphi_k/dz_k  +  sum_i gb_i dphi_i/dz_k ).
// Transposes of the operators (scaled expansions, see expansions.hip):
//   L2P^T: point values -> leaf "local" sensitivities, mu_l(T) = sum gb_i v_i^l:
//          the P2M operator applied to the strengths gb;
//   L2L^T: child -> parent; L2L(C<-P) = M2M(P<-C)^T (same rho, tau), so this is M2M;
//   M2L^T: K(T,S)^T = -K(S,T) (swap d -> -d), so lambda = -M2L(mu) over the
//          symmetric weak lists;
//   M2M^T: parent -> child, i.e. the L2L operator;
//   P2M^T: leaf multipole sensitivities -> points, i.e. the L2P evaluation;
//   P2P^T: sum_i gb_i/(z_i - z_k) = -(P2P of gb)(z_k).
// So A^T gb = -FMM(gb), which the chain below computes operator by operator
// (the sign is folded into the strengths of the far-field chain).
// Position derivatives (geometry frozen, so z enters P2P, P2M and L2P):
//   target part  dphi_k/dz_k = -sum_j m_j/(z_k - z_j)^2 + L2P'(b)(z_k)
//                (b: the forward local expansions);
//   source part  sum_i gb_i dphi_i/dz_k = m_k ( sum_i gb_i/(z_k - z_i)^2 + L2P'(lambda)(z_k) )
//                (dP2M/dz_k: a_q += m_k q w^(q-1)/rs, contracted with lambda).
#include <cfloat>
#include <climits>
#include <type_traits>

#include "fmm_internal.h"
#include "kernels_common.h"
#include "p2p_common.h"
#include "plan_extra.h"

namespace fmm {

template <class T>
void launch_p2m(const int32_t*, int, const int32_t*, const int32_t*, int, const double*, const double*,
                const double*, const double*, int, void*, hipStream_t, const int32_t* = nullptr,
                const double* = nullptr, const GatherOut* = nullptr);
template <class T>
void launch_m2m(const int32_t*, int, const int32_t*, const double*, const double*, int, void*, hipStream_t);
template <class T>
void launch_l2l(const int32_t*, int, const int32_t*, const double*, const double*, int, void*, hipStream_t);
template <class T>
void launch_m2l(const int32_t*, int, const int2*, int, const int32_t*, const int32_t*, double*, bool,
                const int32_t*, const int32_t*, const int32_t*, const double*, const double*, int, const void*, void*,
                hipStream_t, int, const long long*);
void launch_gather(int64_t n, const int32_t* perm, const double* m, double* mtree, hipStream_t s);

struct P2PItemA {
    int32_t leaf, t0, tn, pad;
};

// conj(g) in tree order (for P2P^T) and -conj(g) (strengths of the far chain)
__global__ void k_gather_adj(int64_t n, const int32_t* __restrict__ perm, const double2* __restrict__ g,
                             double2* gb, double2* ngb, float2* gb32)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 v = g[perm[i]];
    gb[i] = make_double2(v.x, -v.y);
    ngb[i] = make_double2(-v.x, v.y);
    if (gb32) gb32[i] = make_float2((float)v.x, (float)-v.y);
}


// Near field of the adjoint, per target k over its strong list:
//   A_k = sum gb_j/(z_k - z_j),  B_k = sum gb_j/(z_k - z_j)^2,  C_k = sum m_j/(z_k - z_j)^2
// (coincident positions excluded).  Same lane layout as the forward P2P:
// SUB subgroups, TG targets per lane, one source per lane, sources staged in
// LDS; the 6 accumulators of a target (padded to 8) are summed by a
// transposing butterfly.  With DER only C_k is formed (the field derivative
// needs nothing else): 2 accumulators per target, written to entries 4 and 5
// of the target's six; entries 0-3 are then left undefined.
template <class R>
struct AdjSrc {
    double x, y;           // positions in FP64: dz is formed in FP64, then rounded to R
    R mr, mi, gr, gi;
};

template <class R, int TG, int SUB, bool DER>
__global__ void __launch_bounds__(256)
k_p2p_adj(const P2PItemA* __restrict__ items, int item_base, const int2* __restrict__ xitems, int nx,
          const int32_t* __restrict__ icnt, const int32_t* __restrict__ ioff,
          double* __restrict__ partial, const int32_t* __restrict__ bstart,
          const int32_t* __restrict__ bcount, const int32_t* __restrict__ s_beg, const int32_t* __restrict__ s_cnt,
          const int32_t* __restrict__ s_ids, const double* __restrict__ X, const double* __restrict__ Y,
          const double2* __restrict__ mt, const double2* __restrict__ gb, double* __restrict__ out)
{
    constexpr int NL = 64 / SUB;
    constexpr int CAP = sizeof(R) == 4 ? 256 : 128;
    constexpr int NA = DER ? 2 : 6;                // accumulators per target
    constexpr int VS = DER ? 2 : 8;                // their stride (a power of two)
    constexpr int V = VS * TG;
    __shared__ AdjSrc<R> sbuf[4][CAP];
    __shared__ int2 smeta[4][64];
    __shared__ int smark[4][CAP];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int xi = xcd_block() * 4 + w;
    if (xi >= nx) return;
    // (item, source chunk); without chunk lists every item is one chunk
    const int2 xe = xitems ? xitems[xi] : make_int2(item_base + xi, 0);
    const P2PItemA it = items[xe.x];
    const int nch = icnt ? icnt[xe.x] : 1;
    AdjSrc<R>* lds = sbuf[w];
    const int g = lane / NL, sl = lane % NL;
    const int base = bstart[it.leaf] + it.t0;
    double tx[TG], ty[TG];   // the targets' positions
    R acc[TG][NA];
#pragma unroll
    for (int t = 0; t < TG; ++t) {
        int k = g * TG + t;
        int i = base + (k < it.tn ? k : 0);
        tx[t] = X[i];
        ty[t] = Y[i];
#pragma unroll
        for (int q = 0; q < NA; ++q) acc[t][q] = (R)0;
    }
    // the item's entries, or those of its chunk
    const int e0 = s_beg[it.leaf], ce = chunk_entries(bcount[it.leaf]);
    int e = nch == 1 ? 0 : xe.y * ce, off = 0;
    const int ne = nch == 1 ? s_cnt[it.leaf] : min(s_cnt[it.leaf], e + ce);
    auto load = [&](int j) {
        AdjSrc<R> s;
        s.x = X[j];
        s.y = Y[j];
        const double2 mm = mt[j], gg = DER ? make_double2(0.0, 0.0) : gb[j];
        s.mr = (R)mm.x; s.mi = (R)mm.y; s.gr = (R)gg.x; s.gi = (R)gg.y;
        return s;
    };
    while (e < ne) {
        const int ns = stage_sources<CAP>(lds, smeta[w], smark[w], s_ids, bstart, bcount, e0, ne, e, off, lane, load);
        for (int c = 0; c < ns; c += NL) {
            int f = c + sl;
            AdjSrc<R> s = lds[f < ns ? f : 0];
            if (f >= ns) { s.mr = (R)0; s.mi = (R)0; s.gr = (R)0; s.gi = (R)0; }
#pragma unroll
            for (int t = 0; t < TG; ++t) {
                R dx = (R)(tx[t] - s.x);
                R dy = (R)(ty[t] - s.y);
                R r2 = dx * dx + dy * dy;
                R q;
                if (sizeof(R) == 8) {
                    // v_rcp_f64 and one Newton step (below 2.3e-15 relative)
                    double yv = __builtin_amdgcn_rcp((double)r2);
                    yv = fma(yv, fma(-(double)r2, yv, 1.0), yv);
                    q = (R)fmin(yv, DBL_MAX);
                } else {
                    q = (R)fminf(__builtin_amdgcn_rcpf((float)r2), FLT_MAX);
                }
                // w = 1/dz = conj(dz)/|dz|^2, w2 = w*w
                R wr = dx * q, wi = -dy * q;
                R w2r = wr * wr - wi * wi, w2i = (R)2 * wr * wi;
                if constexpr (DER) {
                    acc[t][0] += s.mr * w2r - s.mi * w2i;
                    acc[t][1] += s.mr * w2i + s.mi * w2r;
                } else {
                    acc[t][0] += s.gr * wr - s.gi * wi;
                    acc[t][1] += s.gr * wi + s.gi * wr;
                    acc[t][2] += s.gr * w2r - s.gi * w2i;
                    acc[t][3] += s.gr * w2i + s.gi * w2r;
                    acc[t][4] += s.mr * w2r - s.mi * w2i;
                    acc[t][5] += s.mr * w2i + s.mi * w2r;
                }
            }
        }
        wave_sync();
    }
    R v[V];
#pragma unroll
    for (int t = 0; t < TG; ++t) {
#pragma unroll
        for (int q = 0; q < NA; ++q) v[VS * t + q] = acc[t][q];
#pragma unroll
        for (int q = NA; q < VS; ++q) v[VS * t + q] = (R)0;
    }
    // transposing butterfly over the NL lanes of the subgroup: afterwards this
    // lane holds the totals of value indices base + i, i < NV
    treduce<V, NL>(v, lane);
    constexpr int NV = V >= NL ? V / NL : 1;
    const int base0 = treduce_base<V, NL>(sl);
    const bool writer = V >= NL || (sl & (NL / V - 1)) == 0;
    if (writer) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int idx = base0 + i, t = idx / VS, q = idx % VS + (DER ? 4 : 0);
            const int k = g * TG + t;
            if (q < 6 && k < it.tn) {
                if (nch == 1) out[6 * (int64_t)(base + k) + q] = (double)v[i];
                else partial[((int64_t)(ioff[xe.x] + xe.y) * kItemTargets + k) * 6 + q] = (double)v[i];
            }
        }
    }
}

// Final per-leaf combination: value and derivative of the local expansions
// (forward b, adjoint lambda) at the points, plus the near-field sums.  G
// lanes per leaf (256/G leaves per workgroup), both expansions of every leaf
// in LDS (FP64).
template <class T, int G, int P>
__global__ void __launch_bounds__(256)
k_adj_final(const int32_t* __restrict__ leaves, int nleaf, const int32_t* __restrict__ bstart,
            const int32_t* __restrict__ bcount, const double* __restrict__ geom, const double* __restrict__ X,
            const double* __restrict__ Y, const T* __restrict__ loc, const T* __restrict__ lam, int p,
            const double* __restrict__ nadj, const double2* __restrict__ mt, const double2* __restrict__ gb,
            const int32_t* __restrict__ perm, double2* gm, double2* gz)
{
    using T2 = typename Vec2<T>::type;
    constexpr int NLEAF = 256 / G;                 // leaves per workgroup
    __shared__ double2 sbl[NLEAF][P], sll[NLEAF][P];
    const int lane = threadIdx.x & 63;
    const int slot = threadIdx.x / G;             // leaf slot in the workgroup
    const int li = blockIdx.x * NLEAF + slot;
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
        const T2* bsrc = reinterpret_cast<const T2*>(loc) + (int64_t)g * p;
        const T2* lsrc = reinterpret_cast<const T2*>(lam) + (int64_t)g * p;
        for (int k = sl; k < P; k += G) {
            const T2 zero = {(T)0, (T)0};
            const T2 b = k < p ? bsrc[k] : zero, a = k < p ? lsrc[k] : zero;
            sbl[slot][k] = make_double2((double)b.x, (double)b.y);
            sll[slot][k] = make_double2((double)a.x, (double)a.y);
        }
    }
    __syncthreads();
    const double2* bl = sbl[slot];
    const double2* ll = sll[slot];
    for (int j = sl; j < n; j += G) {
        const int i = st + j;
        const double2 v = make_double2((X[i] - cx) * inv, (Y[i] - cy) * inv);
        // Horner for value and derivative (in v) of both expansions
        double2 bv = bl[P - 1], bd = make_double2(0, 0), lv = ll[P - 1], ld = make_double2(0, 0);
        // partly unrolled so that the coefficients are read from LDS at use
        // (fully unrolled, they would all be hoisted into registers)
#pragma unroll 2
        for (int l = P - 2; l >= 0; --l) {
            bd = cmul(bd, v); bd.x += bv.x; bd.y += bv.y;
            bv = cmul(bv, v); bv.x += bl[l].x; bv.y += bl[l].y;
            ld = cmul(ld, v); ld.x += lv.x; ld.y += lv.y;
            lv = cmul(lv, v); lv.x += ll[l].x; lv.y += ll[l].y;
        }
        // d/dz = (1/rs) d/dv
        const double2 D = make_double2(bd.x * inv, bd.y * inv);
        const double2 E = make_double2(ld.x * inv, ld.y * inv);
        const double2 F = lv;
        const double* na = nadj + 6 * (int64_t)i;
        const double2 A = make_double2(na[0], na[1]), B = make_double2(na[2], na[3]), C = make_double2(na[4], na[5]);
        const double2 mk = mt[i], gk = gb[i];
        const int o = perm[i];
        if (gm) {
            // (A^T gb)_k = -A_k + F_k
            gm[o] = make_double2(F.x - A.x, -(F.y - A.y));
        }
        if (gz) {
            const double2 tpart = cmul(gk, make_double2(D.x - C.x, D.y - C.y));
            const double2 spart = cmul(mk, make_double2(B.x + E.x, B.y + E.y));
            gz[o] = make_double2(tpart.x + spart.x, -(tpart.y + spart.y));
        }
    }
}

static void adj_shape(int nt, bool mixed, int* tg, int* sub)
{
    // four lane subgroups; up to 4 (FP32) or 2 (FP64) targets per lane
    const int tgmax = mixed ? 4 : 2;
    int t = 1;
    while (t < tgmax && 4 * t < nt) t <<= 1;
    *sub = 4;
    *tg = t;
}

template <class R, int TG, int SUB, bool DER>
static void launch_adj_one(const P2PItemA* items, int item_base, const int2* xitems, int nx, const int32_t* icnt,
                           const int32_t* ioff, double* partial, const int32_t* bstart,
                           const int32_t* bcount, const int32_t* s_beg, const int32_t* s_cnt, const int32_t* s_ids,
                           const double* X, const double* Y, const double* mt, const double* gb, double* out,
                           hipStream_t s)
{
    k_p2p_adj<R, TG, SUB, DER><<<(nx + 3) / 4, 256, 0, s>>>(items, item_base, xitems, nx, icnt, ioff, partial,
                                                       bstart, bcount, s_beg, s_cnt, s_ids, X, Y,
                                                       (const double2*)mt, (const double2*)gb, out);
}

void balance_launch(Plan::Balance& b, const void* items, int n, const std::vector<P2PClass>& cls,
                    const int32_t* s_cnt, const int32_t* bcount, hipStream_t s);
void balance_finish(Plan::Balance& b, int n, int vals, hipStream_t s);
void combine_chunks(const Plan::Balance& b, const void* items, int n, const int32_t* bstart, double* out,
                    hipStream_t s);

// Near-field sums of the transposed chain for the weights gb (tree order),
// into pl.near_d (6 doubles per point, see k_p2p_adj; with der only the
// derivative sum C, in entries 4 and 5, and gb unused), in source chunks when
// some strong list is long (the chunk lists of the adjoint items are made
// once per plan).  pl.mtree holds the strengths in tree order.
static void adjoint_near(Plan& pl, const double* gb_tree, bool der, hipStream_t s)
{
    Tree& t = *pl.tree;
    TreeSchedule& sc = *t.sched;
    PlanExtra& ex = *pl.ex;
    const bool mixed = pl.precision == FMM_MIXED;
    if (pl.near_d.n < (size_t)(6 * sc.n)) pl.near_d.alloc(6 * sc.n, s);
    const P2PItemA* items = (const P2PItemA*)ex.adj_items.p;
    int nadj = 0;
    for (auto& c : ex.adj_class) nadj = std::max<int>(nadj, (int)(c.off + c.n));
    Plan::Balance& ba = pl.bal_adj;
    if (ba.cls.empty()) {
        if (pl.split_p2p) {
            balance_launch(ba, items, nadj, ex.adj_class, pl.s_cnt.p, sc.d_box_count.p, s);
            FMM_HIP(hipStreamSynchronize(s));
            balance_finish(ba, nadj, 6, s);
        } else {
            for (auto& c : ex.adj_class) ba.cls.push_back(c.off);
            ba.cls.push_back(nadj);
            ba.total = nadj;
        }
    }
    for (size_t ci = 0; ci < ex.adj_class.size(); ++ci) {
        const P2PClass& c = ex.adj_class[ci];
        const int64_t x0 = ba.cls[ci], x1 = ba.cls[ci + 1];
        const int2* xit = ba.xitems.p ? ba.xitems.p + x0 : nullptr;
        const int nx = (int)(x1 - x0);
#define ACASE(R_, TG_, SUB_)                                                                                  \
    if (c.tg == TG_ && c.sub == SUB_) {                                                                       \
        (der ? launch_adj_one<R_, TG_, SUB_, true> : launch_adj_one<R_, TG_, SUB_, false>)(                   \
                                      items, (int)x0, xit, nx, ba.icnt.p, ba.ioff.p, ba.partial.p,            \
                                      sc.d_box_start.p, sc.d_box_count.p, pl.s_beg.p, pl.s_cnt.p, pl.s_ids.p,  \
                                      t.x.p, t.y.p, pl.mtree.p, gb_tree, pl.near_d.p, s);                  \
        check_launch("p2p adjoint");                                                                          \
        continue;                                                                                             \
    }
        if (mixed) {
            ACASE(float, 1, 4) ACASE(float, 2, 4) ACASE(float, 4, 4)
        } else {
            ACASE(double, 1, 4) ACASE(double, 2, 4)
        }
#undef ACASE
        throw Error(FMM_EDEVICE, "unsupported adjoint P2P shape");
    }
    combine_chunks(ba, items, nadj, sc.d_box_start.p, pl.near_d.p, s);
}

void adjoint_device(Plan& pl, const double* m, const double* gphi, double* gm, double* gz, hipStream_t s)
{
    Tree& t = *pl.tree;
    TreeSchedule& sc = *t.sched;
    PlanExtra& ex = *pl.ex;
    const bool mixed = pl.precision == FMM_MIXED;
    const int64_t n = sc.n;
    const size_t cs = mixed ? sizeof(float) : sizeof(double);
    if (pl.gtree.n < (size_t)(2 * n)) pl.gtree.alloc(2 * n, s);
    DBuf<double> ngb;
    ngb.alloc(2 * n, s);
    if (pl.amp.n < 2 * cs * sc.nbox * pl.p) pl.amp.alloc(2 * cs * sc.nbox * pl.p, s);
    if (pl.aloc.n < 2 * cs * sc.nbox * pl.p) pl.aloc.alloc(2 * cs * sc.nbox * pl.p, s);
    // strengths m in tree order (the forward's gather, repeated for safety)
    launch_gather(n, t.perm.p, m, pl.mtree.p, s);
    k_gather_adj<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, t.perm.p, (const double2*)gphi,
                                                             (double2*)pl.gtree.p, (double2*)ngb.p, nullptr);
    check_launch("gather adjoint");
    // far chain on -gb: L2P^T (= P2M), L2L^T (= M2M), M2L^T (= -M2L), M2M^T (= L2L)
    const int nleaf = (int)sc.nleaf;
    auto far = [&](auto tag) {
        using T = decltype(tag);
        launch_p2m<T>(ex.leaves.p, nleaf, sc.d_box_start.p, sc.d_box_count.p, ex.leaf_max, t.geom.p, t.x.p, t.y.p, ngb.p, pl.p,
                      pl.amp.p, s);
        for (int l = sc.max_levels - 2; l >= 1; --l) {
            int nn = (int)(ex.m2m_off[l + 1] - ex.m2m_off[l]);
            launch_m2m<T>(ex.d_m2m.p + ex.m2m_off[l], nn, ex.child0.p, t.geom.p, ex.binom.p, pl.p, pl.amp.p, s);
        }
        const Plan::Balance& bm = pl.bal_m2l;
        launch_m2l<T>(nullptr, (int)sc.nbox, bm.xitems.p, (int)bm.total, bm.icnt.p, bm.ioff.p, bm.partial.p,
                      bm.total > sc.nbox, pl.w_beg.p, pl.w_cnt.p, pl.w_ids.p, t.geom.p, ex.binom.p, pl.p, pl.amp.p,
                      pl.aloc.p, s, pl.tune.m2l_batch, nullptr);
        for (int l = 1; l + 1 < sc.max_levels; ++l) {
            int nn = (int)(ex.m2m_off[l + 1] - ex.m2m_off[l]);
            launch_l2l<T>(ex.d_m2m.p + ex.m2m_off[l], nn, ex.child0.p, t.geom.p, ex.binom.p, pl.p, pl.aloc.p, s);
        }
    };
    if (mixed) far(float()); else far(double());
    adjoint_near(pl, pl.gtree.p, false, s);
    // combination and scatter: G lanes per leaf, P terms held per lane
    const int G = ex.leaf_max <= 16 ? 16 : (ex.leaf_max <= 32 ? 32 : 64);
    const int P = pl.p <= 16 ? 16 : (pl.p <= 32 ? 32 : 64);
    const unsigned gridf = (unsigned)((nleaf + 256 / G - 1) / (256 / G));
    auto fin = [&](auto tag, auto gtag, auto ptag) {
        using T = decltype(tag);
        constexpr int G_ = decltype(gtag)::value, P_ = decltype(ptag)::value;
        k_adj_final<T, G_, P_><<<gridf, 256, 0, s>>>(ex.leaves.p, nleaf, sc.d_box_start.p, sc.d_box_count.p, t.geom.p,
                                                      t.x.p, t.y.p, (const T*)pl.local.p, (const T*)pl.aloc.p, pl.p,
                                                      pl.near_d.p, (const double2*)pl.mtree.p,
                                                      (const double2*)pl.gtree.p, t.perm.p, (double2*)gm,
                                                      (double2*)gz);
    };
    auto fin_g = [&](auto tag, auto ptag) {
        if (G == 16) fin(tag, std::integral_constant<int, 16>{}, ptag);
        else if (G == 32) fin(tag, std::integral_constant<int, 32>{}, ptag);
        else fin(tag, std::integral_constant<int, 64>{}, ptag);
    };
    auto fin_p = [&](auto tag) {
        if (P == 16) fin_g(tag, std::integral_constant<int, 16>{});
        else if (P == 32) fin_g(tag, std::integral_constant<int, 32>{});
        else fin_g(tag, std::integral_constant<int, 64>{});
    };
    if (mixed) fin_p(float{});
    else fin_p(double{});
    check_launch("adjoint final");
}

// Derivative of the field at the points: the derivative of the forward local
// expansion of the point's leaf (d/dz = (1/rs) d/dv, Horner in v) minus the
// near-field sum sum_j m_j / (z_i - z_j)^2, written in input order.  G lanes
// per leaf, the leaf's expansion in LDS (FP64).
template <class T, int G, int P>
__global__ void __launch_bounds__(256)
k_field_final(const int32_t* __restrict__ leaves, int nleaf, const int32_t* __restrict__ bstart,
              const int32_t* __restrict__ bcount, const double* __restrict__ geom, const double* __restrict__ X,
              const double* __restrict__ Y, const T* __restrict__ loc, int p, const double* __restrict__ nadj,
              const int32_t* __restrict__ perm, double2* dphi)
{
    using T2 = typename Vec2<T>::type;
    constexpr int NLEAF = 256 / G;
    __shared__ double2 sbl[NLEAF][P];
    const int lane = threadIdx.x & 63;
    const int slot = threadIdx.x / G;
    const int li = blockIdx.x * NLEAF + slot;
    const int sl = lane % G;
    const bool valid = li < nleaf;
    int st = 0, n = 0;
    double cx = 0.0, cy = 0.0, inv = 0.0;
    if (valid) {
        const int g = leaves[li];
        st = bstart[g];
        n = bcount[g];
        cx = geom[4 * (int64_t)g];
        cy = geom[4 * (int64_t)g + 1];
        inv = 1.0 / geom[4 * (int64_t)g + 3];
        const T2* bsrc = reinterpret_cast<const T2*>(loc) + (int64_t)g * p;
        for (int k = sl; k < P; k += G) {
            const T2 zero = {(T)0, (T)0};
            const T2 b = k < p ? bsrc[k] : zero;
            sbl[slot][k] = make_double2((double)b.x, (double)b.y);
        }
    }
    __syncthreads();
    const double2* bl = sbl[slot];
    for (int j = sl; j < n; j += G) {
        const int i = st + j;
        const double2 v = make_double2((X[i] - cx) * inv, (Y[i] - cy) * inv);
        double2 bv = bl[P - 1], bd = make_double2(0, 0);
#pragma unroll 2
        for (int l = P - 2; l >= 0; --l) {
            bd = cmul(bd, v); bd.x += bv.x; bd.y += bv.y;
            bv = cmul(bv, v); bv.x += bl[l].x; bv.y += bl[l].y;
        }
        const double* na = nadj + 6 * (int64_t)i;
        dphi[perm[i]] = make_double2(bd.x * inv - na[4], bd.y * inv - na[5]);
    }
}

void field_device(Plan& pl, const double* m, double* phi, double* dphi, hipStream_t s)
{
    Tree& t = *pl.tree;
    TreeSchedule& sc = *t.sched;
    PlanExtra& ex = *pl.ex;
    const bool mixed = pl.precision == FMM_MIXED;
    // the forward evaluation: phi, the local expansions and m in tree order
    evaluate_device(pl, m, phi, nullptr, nullptr, s);
    // near-field derivative sums: near_d[4..5] = sum m_j w^2
    adjoint_near(pl, pl.mtree.p, true, s);
    const int nleaf = (int)sc.nleaf;
    const int G = ex.leaf_max <= 16 ? 16 : (ex.leaf_max <= 32 ? 32 : 64);
    const int P = pl.p <= 16 ? 16 : (pl.p <= 32 ? 32 : 64);
    const unsigned grid = (unsigned)((nleaf + 256 / G - 1) / (256 / G));
    auto fin = [&](auto tag, auto gtag, auto ptag) {
        using T = decltype(tag);
        constexpr int G_ = decltype(gtag)::value, P_ = decltype(ptag)::value;
        k_field_final<T, G_, P_><<<grid, 256, 0, s>>>(ex.leaves.p, nleaf, sc.d_box_start.p, sc.d_box_count.p,
                                                      t.geom.p, t.x.p, t.y.p, (const T*)pl.local.p, pl.p,
                                                      pl.near_d.p, t.perm.p, (double2*)dphi);
    };
    auto fin_g = [&](auto tag, auto ptag) {
        if (G == 16) fin(tag, std::integral_constant<int, 16>{}, ptag);
        else if (G == 32) fin(tag, std::integral_constant<int, 32>{}, ptag);
        else fin(tag, std::integral_constant<int, 64>{}, ptag);
    };
    auto fin_p = [&](auto tag) {
        if (P == 16) fin_g(tag, std::integral_constant<int, 16>{});
        else if (P == 32) fin_g(tag, std::integral_constant<int, 32>{});
        else fin_g(tag, std::integral_constant<int, 64>{});
    };
    if (mixed) fin_p(float{});
    else fin_p(double{});
    check_launch("field final");
}

// adjoint P2P work items (leaf, target chunk) grouped by shape; host side
void prepare_adjoint_items(Plan& pl, PlanExtra& ex, const std::vector<int32_t>& leaves, hipStream_t s)
{
    TreeSchedule& sc = *pl.tree->sched;
    const bool mixed = pl.precision == FMM_MIXED;
    std::map<std::pair<int, int>, std::vector<P2PItemA>> cls;
    for (int32_t g : leaves) {
        int nt = sc.box_count[g];
        int tg, sub;
        adj_shape(nt, mixed, &tg, &sub);
        int chunk = tg * sub;
        for (int t0 = 0; t0 < nt; t0 += chunk) cls[{tg, sub}].push_back(P2PItemA{g, t0, std::min(chunk, nt - t0), 0});
    }
    std::vector<P2PItemA> items;
    ex.adj_class.clear();
    for (auto& kv : cls) {
        ex.adj_class.push_back({kv.first.first, kv.first.second, (int64_t)items.size(), (int64_t)kv.second.size()});
        items.insert(items.end(), kv.second.begin(), kv.second.end());
    }
    ex.adj_items.alloc(std::max<size_t>(items.size() * sizeof(P2PItemA), 1), s);
    if (!items.empty())
        FMM_HIP(hipMemcpyAsync(ex.adj_items.p, items.data(), items.size() * sizeof(P2PItemA), hipMemcpyHostToDevice, s));
    FMM_HIP(hipStreamSynchronize(s));
}

}  // namespace fmm
