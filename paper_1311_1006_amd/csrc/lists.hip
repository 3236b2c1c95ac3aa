// lists.hip -- strong / weak connectivity of Sec. 2.1 on gfx950.
//
// Level by level (all problems of a batch at once): the candidates of a box
// are the children of the boxes strongly coupled to its parent; a candidate
// is weak (an M2L partner at this level) when the theta-criterion (2.3)
// R + theta r <= theta d holds and strong otherwise; a box is always strong
// with itself.  Each level is three kernels: count, exclusive scan (one
// workgroup; it also offsets the level into the id pools), fill.  Fills are
// bounds-checked against the pool capacity; an overflow flag makes the host
// grow the pools and run the build again.
#include "fmm_internal.h"

// Box geometry, split axes and the theta-criterion must round every product
// and sum on its own (no fused multiply-add), like a plain IEEE evaluation.
#pragma clang fp contract(off)

namespace fmm {

// theta-criterion, squared, every product and sum rounded alone
__device__ __forceinline__ bool well_separated(const double* gb, const double* gc, double theta)
{
    double R = gb[2] > gc[2] ? gb[2] : gc[2];
    double rr = gb[2] > gc[2] ? gc[2] : gb[2];
    double dx = (gb[0] - gc[0]), dy = (gb[1] - gc[1]);
    double s = ((dx * dx) + (dy * dy));
    double t = (R + (theta * rr));
    double tt = (t * t);
    double rhs = ((theta * theta) * s);
    return (s > 0.0) && (tt <= rhs);
}

struct LevelCtx {
    const int32_t* boxes;     // global ids of this level's boxes
    int n;
    const int32_t* parent;
    const int32_t* prob;
    const int64_t* pbox;      // first box id per problem
    int64_t lb, lbp;          // level_base(l), level_base(l-1)
    const double* geom;       // [nbox][4] cx cy r rs
    double theta;
};

template <bool FILL>
__global__ void k_level(LevelCtx c, int32_t* s_beg, int32_t* s_cnt, int32_t* w_beg, int32_t* w_cnt,
                        int32_t* s_ids, int32_t* w_ids, int64_t cap_s, int64_t cap_w)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= c.n) return;
    int32_t g = c.boxes[i];
    int32_t P = c.parent[g];
    int64_t pb = c.pbox[c.prob[g]];
    const double* gg = c.geom + 4 * (int64_t)g;
    int32_t ps = s_beg[P], pn = s_cnt[P];
    int ns = 0, nw = 0;
    int64_t sb = 0, wb = 0;
    if (FILL) { sb = s_beg[g]; wb = w_beg[g]; }
    for (int e = 0; e < pn; ++e) {
        if ((int64_t)ps + e >= cap_s) break;   // pools overflowed at an earlier level
        int32_t q = s_ids[ps + e];
        int64_t c0 = pb + c.lb + 4 * ((int64_t)q - pb - c.lbp);
        for (int k = 0; k < 4; ++k) {
            int32_t cc = (int32_t)(c0 + k);
            bool weak = (cc != g) && well_separated(gg, c.geom + 4 * (int64_t)cc, c.theta);
            if (weak) {
                if (FILL && wb + nw < cap_w) w_ids[wb + nw] = cc;
                ++nw;
            } else {
                if (FILL && sb + ns < cap_s) s_ids[sb + ns] = cc;
                ++ns;
            }
        }
    }
    if (!FILL) { s_cnt[g] = ns; w_cnt[g] = nw; }
}

// exclusive scan of the level's counts into pool offsets; totals[0..1] hold
// the running pool sizes (strong, weak), totals[2] an overflow flag
__global__ void __launch_bounds__(1024)
k_level_scan(const int32_t* boxes, int n, const int32_t* s_cnt, const int32_t* w_cnt, int32_t* s_beg,
             int32_t* w_beg, long long* totals, int64_t cap_s, int64_t cap_w)
{
    __shared__ long long sh[2][16];
    long long bs = totals[0], bw = totals[1];
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int c0 = 0; c0 < n; c0 += 1024) {
        int i = c0 + threadIdx.x;
        long long vs = 0, vw = 0;
        if (i < n) { vs = s_cnt[boxes[i]]; vw = w_cnt[boxes[i]]; }
        long long xs = vs, xw = vw;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            long long ys = __shfl_up(xs, o, 64), yw = __shfl_up(xw, o, 64);
            if (lane >= o) { xs += ys; xw += yw; }
        }
        if (lane == 63) { sh[0][wid] = xs; sh[1][wid] = xw; }
        __syncthreads();
        long long ps = 0, pw = 0, ts = 0, tw = 0;
        for (int w = 0; w < 16; ++w) {
            if (w < wid) { ps += sh[0][w]; pw += sh[1][w]; }
            ts += sh[0][w]; tw += sh[1][w];
        }
        if (i < n) {
            s_beg[boxes[i]] = (int32_t)(bs + ps + xs - vs);
            w_beg[boxes[i]] = (int32_t)(bw + pw + xw - vw);
        }
        bs += ts; bw += tw;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        totals[0] = bs; totals[1] = bw;
        if (bs > cap_s || bw > cap_w) totals[2] = 1;
    }
}

__global__ void k_root_lists(const int32_t* roots, int n, int32_t* s_beg, int32_t* s_cnt, int32_t* w_beg,
                             int32_t* w_cnt, int32_t* s_ids, long long* totals)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        int32_t r = roots[i];
        s_beg[r] = i; s_cnt[r] = 1; s_ids[i] = r;
        w_beg[r] = 0; w_cnt[r] = 0;
    }
    if (i == 0) { totals[0] = n; totals[1] = 0; totals[2] = 0; totals[3] = 0; }
}

// pairs of the near field: sum over leaves of n_T * (points of its strong list)
__global__ void k_count_p2p(const int32_t* leaves, int n, const int32_t* box_count, const int32_t* s_beg,
                            const int32_t* s_cnt, const int32_t* s_ids, long long* totals, int64_t cap_s)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    long long v = 0;
    if (i < n) {
        int32_t g = leaves[i];
        long long src = 0;
        for (int e = 0; e < s_cnt[g] && (int64_t)s_beg[g] + e < cap_s; ++e)
            src += box_count[s_ids[s_beg[g] + e]];
        v = src * box_count[g];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd((unsigned long long*)&totals[3], (unsigned long long)v);
}

void build_lists_device(Plan& pl, hipStream_t s)
{
    Tree& t = *pl.tree;
    TreeSchedule& sc = *t.sched;
    int64_t nb = sc.nbox;
    pl.s_beg.alloc(nb, s); pl.s_cnt.alloc(nb, s); pl.w_beg.alloc(nb, s); pl.w_cnt.alloc(nb, s);
    DBuf<int64_t> pbox; pbox.alloc(sc.nprob, s);
    FMM_HIP(hipMemcpyAsync(pbox.p, sc.pbox.data(), sizeof(int64_t) * sc.nprob, hipMemcpyHostToDevice, s));
    DBuf<long long> totals; totals.alloc(4, s);
    int64_t cap_s = std::max<int64_t>(pl.n_strong, 24 * nb + 1024);
    int64_t cap_w = std::max<int64_t>(pl.n_weak, 64 * nb + 1024);
    for (int attempt = 0; attempt < 3; ++attempt) {
        pl.s_ids.alloc(cap_s, s);
        pl.w_ids.alloc(cap_w, s);
        const int32_t* lv = pl.d_level_boxes.p;
        int nroot = (int)pl.level_boxes[0].size();
        k_root_lists<<<(nroot + 255) / 256, 256, 0, s>>>(lv, nroot, pl.s_beg.p, pl.s_cnt.p, pl.w_beg.p,
                                                         pl.w_cnt.p, pl.s_ids.p, totals.p);
        check_launch("root lists");
        for (int l = 1; l < sc.max_levels; ++l) {
            LevelCtx c;
            c.boxes = lv + pl.level_boxes_off[l];
            c.n = (int)pl.level_boxes[l].size();
            if (c.n == 0) continue;
            c.parent = sc.d_box_parent.p; c.prob = sc.d_box_prob.p; c.pbox = pbox.p;
            c.lb = level_base(l); c.lbp = level_base(l - 1);
            c.geom = t.geom.p; c.theta = pl.theta;
            int g = (c.n + 255) / 256;
            k_level<false><<<g, 256, 0, s>>>(c, pl.s_beg.p, pl.s_cnt.p, pl.w_beg.p, pl.w_cnt.p, pl.s_ids.p,
                                             pl.w_ids.p, cap_s, cap_w);
            k_level_scan<<<1, 1024, 0, s>>>(c.boxes, c.n, pl.s_cnt.p, pl.w_cnt.p, pl.s_beg.p, pl.w_beg.p,
                                            totals.p, cap_s, cap_w);
            k_level<true><<<g, 256, 0, s>>>(c, pl.s_beg.p, pl.s_cnt.p, pl.w_beg.p, pl.w_cnt.p, pl.s_ids.p,
                                            pl.w_ids.p, cap_s, cap_w);
            check_launch("level lists");
        }
        int nl = (int)sc.nleaf;
        k_count_p2p<<<(nl + 255) / 256, 256, 0, s>>>(pl.leaves.p, nl, sc.d_box_count.p, pl.s_beg.p,
                                                     pl.s_cnt.p, pl.s_ids.p, totals.p, cap_s);
        check_launch("count p2p");
        long long h[4];
        FMM_HIP(hipMemcpyAsync(h, totals.p, sizeof(h), hipMemcpyDeviceToHost, s));
        FMM_HIP(hipStreamSynchronize(s));
        pl.n_strong = h[0];
        pl.n_weak = h[1];
        pl.n_p2p_pairs = h[3];
        if (!h[2]) return;
        cap_s = h[0] + h[0] / 4 + 1024;
        cap_w = h[1] + h[1] / 4 + 1024;
    }
    throw Error(FMM_EDEVICE, "connectivity lists did not fit after growing the pools");
}

}  // namespace fmm
