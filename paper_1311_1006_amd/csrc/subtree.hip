// subtree.hip -- the upward and downward passes of the far field (Sec. 2.1,
// Fig. 2.2) by subtrees, for trees whose problems all have the same depth
// L >= 3 and expansions of at most 32 terms.
//
// Expansions are the scaled ones of expansions.hip (multipole a_k and local
// b_l in powers of (z - c)/rs); the shifts are the same exact re-centrings:
//     M2M  a^P_k = sum_{l<=k} C(k,l) rho^l tau^(k-l) a^C_l
//     L2L  b^C_l = rho^l sum_{k>=l} C(k,l) tau^(k-l) b^P_k
// with rho = rs_C / rs_P and tau = (c_C - c_P) / rs_P, computed in FP64 (the
// storage type T of the coefficients is float for mixed precision).
//
// Upward: one workgroup per box R of level L-3 forms the multipoles of its 16
// leaves (P2M, with the gather of the strengths into tree order, which the
// near field reads), of its 4 children and of R itself, all from LDS; then one
// workgroup per box of level a forms the 3 levels a+2, a+1, a above the
// level a+3 the previous launch wrote, until the root.  Three launches at
// L = 9 instead of one per level.
//
// Downward: the local expansion of a box is its own M2L sum plus the L2L
// image of its parent's complete expansion, hence plus the images, shifted
// directly into the box, of the M2L sums of all its ancestors (the shifts
// are exact, so the two forms agree up to rounding).  One workgroup per box R
// of level L-3 shifts the M2L sums of R's ancestors (levels 0 .. L-4) into R,
// one 16-lane group per ancestor, adds them to R's own, hands the result
// down to R's 4 children and 16 leaves in LDS, stores every leaf's complete
// expansion and evaluates it at the leaf's points (L2P), adding the near
// field and scattering to input order.  There is no L2L launch.
#include <type_traits>

#include "fmm_internal.h"
#include "kernels_common.h"

namespace fmm {

// b^e, e >= 0, by repeated squaring (the operations of the shift tables of
// expansions.hip)
__device__ __forceinline__ double2 sub_cpow(double2 b, int e)
{
    double2 r = make_double2(1.0, 0.0);
    while (e) {
        if (e & 1) r = cmul(r, b);
        b = cmul(b, b);
        e >>= 1;
    }
    return r;
}
__device__ __forceinline__ double sub_rpow(double b, int e)
{
    double r = 1.0;
    while (e) {
        if (e & 1) r *= b;
        b *= b;
        e >>= 1;
    }
    return r;
}

// id of box j of level l of problem b, every problem holding NB boxes
__device__ __forceinline__ int sub_box(int b, int64_t NB, int l, int64_t j)
{
    return (int)((int64_t)b * NB + level_base(l) + j);
}

// The binomial table C(k, l), k, l < P, into LDS (row k, column l), in two
// steps so that other loads can be issued between them: the loads into
// registers (all in flight before the first store), then the stores
template <int P>
struct BinomRegs {
    static constexpr int R = (P * P + 255) / 256;   // blocks of 256 threads
    double v[R];
};
template <int P>
__device__ __forceinline__ BinomRegs<P> binom_load(const double* __restrict__ binom)
{
    BinomRegs<P> b;
#pragma unroll
    for (int r = 0; r < BinomRegs<P>::R; ++r) {
        const int i = threadIdx.x + 256 * r;
        b.v[r] = binom[(i < P * P ? i / P : 0) * kBinomStride + (i < P * P ? i % P : 0)];
    }
    return b;
}
template <int P>
__device__ __forceinline__ void binom_store(double (*sb)[P], const BinomRegs<P>& b)
{
#pragma unroll
    for (int r = 0; r < BinomRegs<P>::R; ++r) {
        const int i = threadIdx.x + 256 * r;
        if (i < P * P) sb[i / P][i % P] = b.v[r];
    }
}
template <int P>
__device__ __forceinline__ void load_binom(double (*sb)[P], const double* __restrict__ binom)
{
    binom_store<P>(sb, binom_load<P>(binom));
}

// M2M into one parent by one wavefront: lane (c, j), c = lane/16 the child,
// forms child c's contribution to the coefficients k = j, j + 16 of the
// parent; co[c] holds child c's coefficients (as stored, in FP64).  The
// contributions land in part[c][k]; the caller adds them in child order.
// The geometry an M2M step needs (centre and scaling radius of the parent
// and of the lane's child), loaded ahead of the step.
struct M2MGeo {
    double px, py, prs, cx, cy, crs;
};
__device__ __forceinline__ M2MGeo m2m_geo(const double* __restrict__ geom, int par, int child)
{
    const double* gp = geom + 4 * (int64_t)par;
    const double* gc = geom + 4 * (int64_t)child;
    return M2MGeo{gp[0], gp[1], gp[3], gc[0], gc[1], gc[3]};
}

template <int P>
__device__ __forceinline__ void m2m_wave(int p, const M2MGeo& g, const double2 (*co)[P], double2 (*tau)[P],
                                         double (*rho)[P], double2 (*part)[P], const double (*sb)[P])
{
    const int lane = threadIdx.x & 63, c = lane >> 4, j = lane & 15;
    const double prs = g.prs;
    const double r = g.crs / prs;
    const double2 t = make_double2((g.cx - g.px) / prs, (g.cy - g.py) / prs);
    for (int jj = j; jj < p; jj += 16) {
        tau[c][jj] = sub_cpow(t, jj);
        rho[c][jj] = sub_rpow(r, jj);
    }
    wave_sync();
    // the sums run over the compile-time bound P (terms past k are skipped),
    // so that their LDS loads are all issued before the first is used
    for (int k = j; k < p; k += 16) {
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int l = 0; l < P; ++l) {
            if (l <= k) {
                const double s = sb[k][l] * rho[c][l];
                const double2 v = cmul(co[c][l], tau[c][k - l]);
                acc.x += s * v.x;
                acc.y += s * v.y;
            }
        }
        part[c][k] = acc;
    }
    wave_sync();
}

// The parent's coefficient k (lane k < p) from the four contributions
template <int P>
__device__ __forceinline__ double2 m2m_sum(const double2 (*part)[P], int k)
{
    const double2 v0 = part[0][k], v1 = part[1][k], v2 = part[2][k], v3 = part[3][k];
    return make_double2(((v0.x + v1.x) + v2.x) + v3.x, ((v0.y + v1.y) + v2.y) + v3.y);
}

template <class T>
__device__ __forceinline__ void store_coef(T* dst, int64_t box, int p, int k, double2 v, double2* mirror)
{
    const T tx = (T)v.x, ty = (T)v.y;
    dst[2 * (box * p + k)] = tx;
    dst[2 * (box * p + k) + 1] = ty;
    if (mirror) *mirror = make_double2((double)tx, (double)ty);
}

// ------------------------------------------------------------------ upward

// One workgroup per box R of level L-3 (nroot per problem): P2M of its 16
// leaves (16 lanes per leaf, the transposing butterfly of k_p2m), M2M into
// its 4 children (one wavefront each) and into R (wavefront 0).
template <class T, int P, bool GATHER>
__global__ void __launch_bounds__(256)
k_up_leaf(int L, int64_t NB, int nroot, const int32_t* __restrict__ bstart, const int32_t* __restrict__ bcount,
          const double* __restrict__ geom, const double* __restrict__ X, const double* __restrict__ Y,
          const double2* __restrict__ mt, int p, T* mp, const double* __restrict__ binom, GatherOut go)
{
    constexpr int V = 2 * P;
    __shared__ double sb[P][P];
    __shared__ double2 sco[16][P];        // the leaves' coefficients (as stored)
    __shared__ double2 spar[4][P];        // the children of R (as stored)
    __shared__ double2 stau[4][4][P];     // per wavefront: tau^j of its four children
    __shared__ double srho[4][4][P];
    __shared__ double2 spart[4][4][P];    // per wavefront: the children's contributions
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int gl = threadIdx.x >> 4, sl = threadIdx.x & 15;
    const int b = blockIdx.x / nroot;
    const int64_t jR = blockIdx.x % nroot;
    const int R = sub_box(b, NB, L - 3, jR);
    const int leaf = sub_box(b, NB, L - 1, 16 * jR + gl);
    const BinomRegs<P> bin = binom_load<P>(binom);   // stored to LDS after P2M
    const int st = bstart[leaf], n = bcount[leaf];
    const double cx = geom[4 * (int64_t)leaf], cy = geom[4 * (int64_t)leaf + 1];
    const double inv = 1.0 / geom[4 * (int64_t)leaf + 3];
    double v[V];
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] = 0.0;
    for (int j = sl; j < n; j += 16) {
        const int i = st + j;
        double2 z, t;
        if constexpr (GATHER) {
            const double2 mm = go.m[go.perm[i]];
            const double x = X[i], y = Y[i];
            go.mtree[i] = mm;
            z = make_double2((x - cx) * inv, (y - cy) * inv);
            t = mm;
        } else {
            z = make_double2((X[i] - cx) * inv, (Y[i] - cy) * inv);
            t = mt[i];
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            v[2 * k] += t.x;
            v[2 * k + 1] += t.y;
            if (k + 1 < P) t = cmul(t, z);
        }
    }
    treduce<V, 16>(v, lane);
    const int base = treduce_base<V, 16>(sl);
#pragma unroll
    for (int i = 0; i < V / 16; ++i) {
        const int idx = base + i, k = idx >> 1;
        if (k < p) {
            const T tv = (T)v[i];
            mp[2 * ((int64_t)leaf * p + k) + (idx & 1)] = tv;
            if (idx & 1) sco[gl][k].y = (double)tv;
            else sco[gl][k].x = (double)tv;
        }
    }
    binom_store<P>(sb, bin);
    __syncthreads();   // the binomial table; the leaves of each wavefront are its own lanes'
    // the children of R: wavefront w forms child w from leaves 4w .. 4w+3
    const int cw = sub_box(b, NB, L - 2, 4 * jR + w);
    m2m_wave<P>(p, m2m_geo(geom, cw, sub_box(b, NB, L - 1, 16 * jR + 4 * w + (lane >> 4))), sco + 4 * w, stau[w],
                srho[w], spart[w], sb);
    for (int k = lane; k < p; k += 64) store_coef<T>(mp, cw, p, k, m2m_sum<P>(spart[w], k), &spar[w][k]);
    __syncthreads();
    if (w == 0) {
        m2m_wave<P>(p, m2m_geo(geom, R, sub_box(b, NB, L - 2, 4 * jR + (lane >> 4))), spar, stau[0], srho[0],
                    spart[0], sb);
        for (int k = lane; k < p; k += 64) store_coef<T>(mp, R, p, k, m2m_sum<P>(spart[0], k), nullptr);
    }
}

// One workgroup per box A of level a (nper per problem): the multipoles of
// levels a+D-1 .. a of A's subtree from those of level a+D (D <= 3).
template <class T, int P>
__global__ void __launch_bounds__(256)
k_up_mid(int a, int D, int64_t NB, int nper, const double* __restrict__ geom, int p, T* mp,
         const double* __restrict__ binom)
{
    __shared__ double sb[P][P];
    __shared__ double2 sc0[64][P];
    __shared__ double2 sc1[16][P];
    __shared__ double2 stau[4][4][P];
    __shared__ double srho[4][4][P];
    __shared__ double2 spart[4][4][P];
    __shared__ double sg[85][3];          // centre and scaling radius of the boxes under A
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int b = blockIdx.x / nper;
    const int64_t jA = blockIdx.x % nper;
    const BinomRegs<P> bin = binom_load<P>(binom);
    // the geometry of A's subtree, levels a .. a+D (at most 85 boxes), loaded
    // once for all the M2M steps: slot t = (4^d - 1)/3 + i holds box i of
    // level a+d under A (a thread past the last slot loads the last again)
    const int ngeo = ((4 << (2 * D)) - 1) / 3;
    double gv[3];
    {
        const int t = min((int)threadIdx.x, ngeo - 1);
        int d = 0, base = 0;
        while (t >= base + (1 << (2 * d))) {
            base += 1 << (2 * d);
            ++d;
        }
        const int64_t box = sub_box(b, NB, a + d, ((int64_t)jA << (2 * d)) + (t - base));
        gv[0] = geom[4 * box];
        gv[1] = geom[4 * box + 1];
        gv[2] = geom[4 * box + 3];
    }
    // level a+D: 4^D <= 64 boxes, all loads in flight before the first store
    const int nin = 1 << (2 * D);
    constexpr int R = 64 * P / 256;
    double2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = threadIdx.x + 256 * r;
        const int c = i / P, k = i % P;
        v[r] = make_double2(0.0, 0.0);
        if (c < nin && k < p) {
            const int64_t box = sub_box(b, NB, a + D, ((int64_t)jA << (2 * D)) + c);
            v[r] = make_double2((double)mp[2 * (box * p + k)], (double)mp[2 * (box * p + k) + 1]);
        }
    }
    binom_store<P>(sb, bin);
    if ((int)threadIdx.x < ngeo)
        for (int e = 0; e < 3; ++e) sg[threadIdx.x][e] = gv[e];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = threadIdx.x + 256 * r;
        const int c = i / P, k = i % P;
        if (c < nin && k < p) sc0[c][k] = v[r];
    }
    __syncthreads();
    double2 (*cur)[P] = sc0;
    double2 (*nxt)[P] = sc1;
    for (int d = D - 1; d >= 0; --d) {
        const int lv = a + d, np = 1 << (2 * d);   // parents at level lv under A
        for (int q = w; q < np; q += 4) {
            const int par = sub_box(b, NB, lv, ((int64_t)jA << (2 * d)) + q);
            const double* gp = sg[((1 << (2 * d)) - 1) / 3 + q];
            const double* gc = sg[((4 << (2 * d)) - 1) / 3 + 4 * q + (lane >> 4)];
            m2m_wave<P>(p, M2MGeo{gp[0], gp[1], gp[2], gc[0], gc[1], gc[2]}, cur + 4 * q, stau[w], srho[w], spart[w],
                        sb);
            for (int k = lane; k < p; k += 64) store_coef<T>(mp, par, p, k, m2m_sum<P>(spart[w], k), &nxt[q][k]);
            wave_sync();   // spart is rewritten by the next parent of this wavefront
        }
        __syncthreads();
        double2 (*tmp)[P] = cur;
        cur = nxt;
        nxt = tmp;
    }
}

// ---------------------------------------------------------------- downward

// One workgroup per box R of level L-3.  See the file header.
// Every global load that does not depend on a computed value (the geometry
// and the M2L sums of R, of its ancestors, of its children and of the leaf
// of each 16-lane group, the leaf's first 32 points with their near field)
// is issued at the start, so the workgroup waits for memory twice (the
// points' loads need the leaf's start) instead of once per phase.
template <class T, int P>
__global__ void __launch_bounds__(256)
k_down_leaf(int L, int64_t NB, int nroot, const int32_t* __restrict__ bstart, const int32_t* __restrict__ bcount,
            const double* __restrict__ geom, const double* __restrict__ X, const double* __restrict__ Y, T* loc,
            int p, const double2* __restrict__ nearf, const int32_t* __restrict__ perm, double2* phi,
            double2* phi_near, double2* phi_far, const long long* __restrict__ guard, const double* __restrict__ binom)
{
    if (guard != nullptr && *guard != 0) return;   // lists flagged: this launch is void
    using T2 = typename Vec2<T>::type;
    constexpr int KP = P / 16;          // coefficients per lane of a 16-lane group
    constexpr int NPT = 2;              // points per lane loaded ahead (a leaf's first 32)
    __shared__ double sb[P][P];
    __shared__ double2 sanc[16][P];     // ancestor coefficients (their M2L sums), then the leaves' expansions
    __shared__ double2 stab[16][P];     // tau powers, one table per 16-lane group
    __shared__ double2 spart[16][P];    // the ancestors' images in R
    __shared__ double2 sR[P];           // R's complete expansion
    __shared__ double2 sC[4][P];        // the children's complete expansions
    const int gl = threadIdx.x >> 4, sl = threadIdx.x & 15, w = threadIdx.x >> 6;
    const int b = blockIdx.x / nroot;
    const int64_t jR = blockIdx.x % nroot;
    const int lR = L - 3;
    const int R = sub_box(b, NB, lR, jR);
    const int leaf = sub_box(b, NB, L - 1, 16 * jR + gl);
    const T2* lo = reinterpret_cast<const T2*>(loc);
    const BinomRegs<P> bin = binom_load<P>(binom);
    // ---- loads: every one unconditional, at an index clamped into range (a
    // load under a branch would be waited for where the branch ends); the
    // lanes that have no use for a value never read it
    const int st = bstart[leaf], n = bcount[leaf];
    const double lcx = geom[4 * (int64_t)leaf], lcy = geom[4 * (int64_t)leaf + 1], lrs = geom[4 * (int64_t)leaf + 3];
    const double Rx = geom[4 * (int64_t)R], Ry = geom[4 * (int64_t)R + 1], Rrs = geom[4 * (int64_t)R + 3];
    // group gl < nanc: the ancestor of level gl
    const int nanc = lR;
    const bool anc = gl < nanc;
    const int A = anc ? sub_box(b, NB, gl, jR >> (2 * (lR - gl))) : R;
    const double ax = geom[4 * (int64_t)A], ay = geom[4 * (int64_t)A + 1], ars = geom[4 * (int64_t)A + 3];
    T2 ca[KP];
#pragma unroll
    for (int q = 0; q < KP; ++q) ca[q] = lo[(int64_t)A * p + min(sl + 16 * q, p - 1)];
    // thread l < p: R's own sum
    const T2 cR = lo[(int64_t)R * p + min((int)threadIdx.x, p - 1)];
    // group c of wavefront 0 (every wavefront loads it; only wavefront 0
    // uses it): child c of R
    const int Cg = sub_box(b, NB, L - 2, 4 * jR + (gl & 3));
    const double cgx = geom[4 * (int64_t)Cg], cgy = geom[4 * (int64_t)Cg + 1], cgrs = geom[4 * (int64_t)Cg + 3];
    T2 cc[KP];
#pragma unroll
    for (int q = 0; q < KP; ++q) cc[q] = lo[(int64_t)Cg * p + min(sl + 16 * q, p - 1)];
    // wavefront w: child w of R, the parent of its four leaves; the leaf's own sum
    const int Cw = sub_box(b, NB, L - 2, 4 * jR + w);
    const double cwx = geom[4 * (int64_t)Cw], cwy = geom[4 * (int64_t)Cw + 1], cwrs = geom[4 * (int64_t)Cw + 3];
    T2 cl[KP];
#pragma unroll
    for (int q = 0; q < KP; ++q) cl[q] = lo[(int64_t)leaf * p + min(sl + 16 * q, p - 1)];
    // the leaf's first points (a lane past the leaf's end reads point 0)
    double px[NPT], py[NPT];
    double2 pn[NPT];
    int po[NPT];
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
        const int j = sl + 16 * q;
        const int i = j < n ? st + j : 0;
        px[q] = X[i];
        py[q] = Y[i];
        pn[q] = nearf[i];
        po[q] = perm[i];
    }
    binom_store<P>(sb, bin);
    __syncthreads();   // every wavefront reads rows of the table the others wrote
    // ---- the ancestors (levels 0 .. lR-1) into R: group gl takes level gl
    if (anc) {
        const double2 t = make_double2((Rx - ax) / ars, (Ry - ay) / ars);
        const double rho = Rrs / ars;
#pragma unroll
        for (int q = 0; q < KP; ++q) {
            const int k = sl + 16 * q;
            if (k < p) {
                sanc[gl][k] = make_double2((double)ca[q].x, (double)ca[q].y);
                stab[gl][k] = sub_cpow(t, k);
            }
        }
        wave_sync();
        for (int l = sl; l < p; l += 16) {
            double2 acc = make_double2(0.0, 0.0);
#pragma unroll
            for (int k = 0; k < P; ++k) {
                if (k >= l && k < p) {
                    const double s = sb[k][l];
                    const double2 v = cmul(sanc[gl][k], stab[gl][k - l]);
                    acc.x += s * v.x;
                    acc.y += s * v.y;
                }
            }
            const double rl = sub_rpow(rho, l);
            spart[gl][l] = make_double2(rl * acc.x, rl * acc.y);
        }
    }
    __syncthreads();
    // R's complete expansion: its own M2L sum, then the ancestors top-down
    if ((int)threadIdx.x < p) {
        const int l = threadIdx.x;
        double2 acc = make_double2((double)cR.x, (double)cR.y);
        for (int a = 0; a < nanc; ++a) {
            acc.x += spart[a][l].x;
            acc.y += spart[a][l].y;
        }
        sR[l] = acc;
    }
    __syncthreads();
    // ---- R into its four children: wavefront 0, lane (c, l)
    if (w == 0) {
        const int c = gl;
        const double2 t = make_double2((cgx - Rx) / Rrs, (cgy - Ry) / Rrs);
        const double rho = cgrs / Rrs;
        for (int k = sl; k < p; k += 16) stab[c][k] = sub_cpow(t, k);
        wave_sync();
#pragma unroll
        for (int q = 0; q < KP; ++q) {
            const int l = sl + 16 * q;
            if (l >= p) continue;
            double2 acc = make_double2(0.0, 0.0);
#pragma unroll
            for (int k = 0; k < P; ++k) {
                if (k >= l && k < p) {
                    const double s = sb[k][l];
                    const double2 v = cmul(sR[k], stab[c][k - l]);
                    acc.x += s * v.x;
                    acc.y += s * v.y;
                }
            }
            const double rl = sub_rpow(rho, l);
            sC[c][l] = make_double2((double)cc[q].x + rl * acc.x, (double)cc[q].y + rl * acc.y);
        }
    }
    __syncthreads();
    // ---- child w into its four leaves (wavefront w, group gl = leaf 4w + m):
    // the leaf's complete expansion, stored (the storage type) and kept for L2P
    {
        const double2 t = make_double2((lcx - cwx) / cwrs, (lcy - cwy) / cwrs);
        const double rho = lrs / cwrs;
        for (int k = sl; k < p; k += 16) stab[gl][k] = sub_cpow(t, k);
        wave_sync();
        T2* lw = reinterpret_cast<T2*>(loc);
#pragma unroll
        for (int q = 0; q < KP; ++q) {
            const int l = sl + 16 * q;
            if (l >= p) {
                sanc[gl][l] = make_double2(0.0, 0.0);
                continue;
            }
            double2 acc = make_double2(0.0, 0.0);
#pragma unroll
            for (int k = 0; k < P; ++k) {
                if (k >= l && k < p) {
                    const double s = sb[k][l];
                    const double2 v = cmul(sC[w][k], stab[gl][k - l]);
                    acc.x += s * v.x;
                    acc.y += s * v.y;
                }
            }
            const double rl = sub_rpow(rho, l);
            const T tx = (T)((double)cl[q].x + rl * acc.x), ty = (T)((double)cl[q].y + rl * acc.y);
            lw[(int64_t)leaf * p + l] = T2{tx, ty};
            sanc[gl][l] = make_double2((double)tx, (double)ty);
        }
        wave_sync();
    }
    // ---- L2P at the leaf's points (Horner), plus the near field, to input order
    const double inv = 1.0 / lrs;
    const double2* co = sanc[gl];
    for (int j = sl, q = 0; j < n; j += 16, ++q) {
        const int i = st + j;
        double x, y, nfx, nfy;
        int o;
        if (q < NPT) {
            // (a run-time index into the arrays would move them to scratch)
            x = q == 0 ? px[0] : px[NPT - 1];
            y = q == 0 ? py[0] : py[NPT - 1];
            nfx = q == 0 ? pn[0].x : pn[NPT - 1].x;
            nfy = q == 0 ? pn[0].y : pn[NPT - 1].y;
            o = q == 0 ? po[0] : po[NPT - 1];
        } else {
            x = X[i]; y = Y[i];
            const double2 nf = nearf[i];
            nfx = nf.x; nfy = nf.y;
            o = perm[i];
        }
        const double2 z = make_double2((x - lcx) * inv, (y - lcy) * inv);
        double2 acc = co[P - 1];
#pragma unroll
        for (int l = P - 2; l >= 0; --l) {
            acc = cmul(acc, z);
            acc.x += co[l].x;
            acc.y += co[l].y;
        }
        if (phi) phi[o] = make_double2(acc.x + nfx, acc.y + nfy);
        if (phi_near) phi_near[o] = make_double2(nfx, nfy);
        if (phi_far) phi_far[o] = acc;
    }
}

// ---------------------------------------------------------------- launchers

bool subtree_ok(int L, int p) { return L >= 3 && p <= 32; }

template <class T>
void launch_up_subtree(int nprob, int L, const int32_t* bstart, const int32_t* bcount, const double* geom,
                       const double* X, const double* Y, const double* mt, int p, void* mp, const double* binom,
                       const GatherOut* go, hipStream_t s, hipEvent_t after_leaves)
{
    const GatherOut none{};
    const GatherOut& gg = go ? *go : none;
    const int64_t NB = nbox_levels(L);
    const int nroot = 1 << (2 * (L - 3));
    const unsigned grid = (unsigned)(nprob * nroot);
#define UP_CASE(P_)                                                                                        \
    if (go)                                                                                                \
        k_up_leaf<T, P_, true><<<grid, 256, 0, s>>>(L, NB, nroot, bstart, bcount, geom, X, Y,             \
                                                    (const double2*)mt, p, (T*)mp, binom, gg);             \
    else                                                                                                   \
        k_up_leaf<T, P_, false><<<grid, 256, 0, s>>>(L, NB, nroot, bstart, bcount, geom, X, Y,            \
                                                     (const double2*)mt, p, (T*)mp, binom, gg);
    if (p <= 16) { UP_CASE(16) }
    else if (p <= 32) { UP_CASE(32) }
    else throw Error(FMM_EINVAL, "subtree upward pass needs p <= 32");
#undef UP_CASE
    check_launch("upward leaves");
    // the gather is complete here: work that needs only the strengths in tree
    // order (the near field) may start
    if (after_leaves) FMM_HIP(hipEventRecord(after_leaves, s));
    // levels L-4 .. 0 in subtrees of at most three levels
    for (int lv = L - 3; lv > 0;) {
        const int D = lv < 3 ? lv : 3;
        const int a = lv - D;
        const int nper = 1 << (2 * a);
        const unsigned g2 = (unsigned)(nprob * nper);
        if (p <= 16) k_up_mid<T, 16><<<g2, 256, 0, s>>>(a, D, NB, nper, geom, p, (T*)mp, binom);
        else k_up_mid<T, 32><<<g2, 256, 0, s>>>(a, D, NB, nper, geom, p, (T*)mp, binom);
        check_launch("upward subtrees");
        lv = a;
    }
}

template <class T>
void launch_down_subtree(int nprob, int L, const int32_t* bstart, const int32_t* bcount, const double* geom,
                         const double* X, const double* Y, void* loc, int p, const double* nearf,
                         const int32_t* perm, double* phi, double* phi_near, double* phi_far, const long long* guard,
                         const double* binom, hipStream_t s)
{
    const int64_t NB = nbox_levels(L);
    const int nroot = 1 << (2 * (L - 3));
    const unsigned grid = (unsigned)(nprob * nroot);
#define DOWN_ARGS L, NB, nroot, bstart, bcount, geom, X, Y, (T*)loc, p, (const double2*)nearf, perm, (double2*)phi, \
                  (double2*)phi_near, (double2*)phi_far, guard, binom
    if (p <= 16) k_down_leaf<T, 16><<<grid, 256, 0, s>>>(DOWN_ARGS);
    else if (p <= 32) k_down_leaf<T, 32><<<grid, 256, 0, s>>>(DOWN_ARGS);
    else throw Error(FMM_EINVAL, "subtree downward pass needs p <= 32");
#undef DOWN_ARGS
    check_launch("downward leaves");
}

#define INST(T)                                                                                           \
    template void launch_up_subtree<T>(int, int, const int32_t*, const int32_t*, const double*, const double*, \
                                       const double*, const double*, int, void*, const double*,          \
                                       const GatherOut*, hipStream_t, hipEvent_t);                       \
    template void launch_down_subtree<T>(int, int, const int32_t*, const int32_t*, const double*,          \
                                         const double*, const double*, void*, int, const double*,          \
                                         const int32_t*, double*, double*, double*, const long long*,      \
                                         const double*, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace fmm
