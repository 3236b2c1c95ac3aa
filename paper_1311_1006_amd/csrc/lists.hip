// lists.hip -- strong / weak connectivity of Sec. 2.1 on gfx950.
//
// Level by level (all problems of a batch at once): the candidates of a box
// are the children of the boxes strongly coupled to its parent; a candidate
// is weak (an M2L partner at this level) when the theta-criterion (2.3)
// R + theta r <= theta d holds and strong otherwise; a box is always strong
// with itself.  The usual build is one pass with fixed per-box capacities;
// otherwise every pass (a range of levels, or one level) is three kernels:
// count, exclusive scan (it also offsets the pass into the id pools), fill.
// Fills are bounds-checked against the pool capacity; an overflow flag makes
// the host grow the pools and run the build again.
#include <algorithm>
#include <climits>
#include <utility>
#include <vector>

#include "fmm_internal.h"
#include "kernels_common.h"
#include "plan_extra.h"

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

// Exclusive scan of the level's counts into pool offsets, in two passes over
// blocks of 1024 boxes: per-block sums, then every block adds the sums of
// the blocks before it.  totals[0..1] hold the running pool sizes (strong,
// weak), totals[2] an overflow flag; snap[0..1] keep the sizes before this
// level so that the second pass can update totals without a race.
__device__ __forceinline__ void block_sum2(long long& a, long long& b, long long (*sh)[16])
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) { a += __shfl_xor(a, o, 64); b += __shfl_xor(b, o, 64); }
    if (lane == 0) { sh[0][wid] = a; sh[1][wid] = b; }
    __syncthreads();
    a = 0; b = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { a += sh[0][w]; b += sh[1][w]; }
    __syncthreads();
}

__global__ void __launch_bounds__(1024)
k_scan_reduce(const int32_t* boxes, int n, const int32_t* s_cnt, const int32_t* w_cnt, long long* bsum,
              const long long* totals, long long* snap)
{
    __shared__ long long sh[2][16];
    const int i = blockIdx.x * 1024 + threadIdx.x;
    long long vs = 0, vw = 0;
    if (i < n) { const int32_t g = boxes[i]; vs = s_cnt[g]; vw = w_cnt[g]; }
    block_sum2(vs, vw, sh);
    if (threadIdx.x == 0) {
        bsum[2 * blockIdx.x] = vs;
        bsum[2 * blockIdx.x + 1] = vw;
        if (blockIdx.x == 0) { snap[0] = totals[0]; snap[1] = totals[1]; }
    }
}

__global__ void __launch_bounds__(1024)
k_scan_apply(const int32_t* boxes, int n, const int32_t* s_cnt, const int32_t* w_cnt, const long long* bsum,
             const long long* snap, int32_t* s_beg, int32_t* w_beg, long long* totals, int64_t cap_s,
             int64_t cap_w)
{
    __shared__ long long sh[2][16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    // offset of this block: sum of the block sums before it
    long long os = 0, ow = 0;
    for (int b = threadIdx.x; b < (int)blockIdx.x; b += 1024) { os += bsum[2 * b]; ow += bsum[2 * b + 1]; }
    block_sum2(os, ow, sh);
    const int i = blockIdx.x * 1024 + threadIdx.x;
    long long vs = 0, vw = 0;
    int32_t g = 0;
    if (i < n) { g = boxes[i]; vs = s_cnt[g]; vw = w_cnt[g]; }
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
    const long long bs0 = snap[0] + os, bw0 = snap[1] + ow;
    if (i < n) {
        s_beg[g] = (int32_t)(bs0 + ps + xs - vs);
        w_beg[g] = (int32_t)(bw0 + pw + xw - vw);
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        totals[0] = bs0 + ts;
        totals[1] = bw0 + tw;
        if (bs0 + ts > cap_s || bw0 + tw > cap_w) totals[2] |= 1;
    }
}

// pairs of the near field: sum over leaves of n_T * (points of its strong
// list); one wavefront per leaf, lanes over the list
__global__ void __launch_bounds__(256)
k_count_p2p(const int32_t* leaves, int n, const int32_t* box_count, const int32_t* s_beg, const int32_t* s_cnt,
            const int32_t* s_ids, long long* totals, int64_t cap_s)
{
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const int32_t g = leaves[i];
    const int64_t b0 = s_beg[g];
    const int cnt = s_cnt[g];
    long long src = 0;
    for (int e0 = lane; e0 < cnt; e0 += 256) {
        int32_t id[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + 64 * u;
            id[u] = (e < cnt && b0 + e < cap_s) ? s_ids[b0 + e] : -1;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (id[u] >= 0) src += box_count[id[u]];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) src += __shfl_xor(src, o, 64);
    if (lane == 0 && src) atomicAdd((unsigned long long*)&totals[3], (unsigned long long)(src * box_count[g]));
}

// ----------------------------------------------------------------------------
// Several levels per pass: for the boxes of levels l0..l1 together, one
// wavefront per box walks down from its ancestor at level l0-1 (whose strong
// list is already in the pool; from the root itself when l0 = 0) to the box,
// keeping the strong list of the ancestor at each level in an LDS frontier.
// The frontier of the box's own level is its strong list, the candidates
// rejected there its weak list; ballots keep both in the order the
// level-by-level build gives.  A pass is count, scan, fill, so a few passes
// replace four launches per level; a deeper pass repeats the upper levels of
// its range once per box, so the passes are kept short near the leaves.  A
// frontier larger than kFrontCap sets bit 1 of the overflow word; the layout
// is then built one level per pass (k_traverse_sib below the root).
constexpr int kFrontCap = 1024;

struct TravCtx {
    const int32_t* boxes;     // global ids of the pass's boxes (levels l0..l1)
    int n;
    int l0;
    int64_t first = -1;       // >= 0: a single problem, and box i of the pass is box first + i
                              // of level l0 (no id, level or problem loads)
    int32_t* long_q = nullptr;   // count and fill passes by sibling groups: the groups whose
    int32_t* long_n = nullptr;   // parent list is long, queued for k_traverse_long (and their count)
    int cs, cw;               // per-box list capacities of the one-pass build
    const int32_t* prob;
    const int8_t* level;
    const int64_t* pbox;
    const double* geom;
    double theta;
    // one-pass mode: per-leaf source counts of the near field, and flags for
    // lists long enough to be split into work chunks
    const int32_t* child0;    // -1 for leaves
    const int32_t* box_count;
    int32_t* nsrc;
};

__device__ __forceinline__ void wave_sync_l()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// MODE 0 counts, MODE 1 fills at the offsets of the scan, MODE 2 does both in
// one pass with fixed per-box capacities: the strong list of box g starts at
// g * cs and its weak list at g * cw (bit 0 of the overflow word when a list
// does not fit; the compact build then runs instead).
template <int MODE>
__global__ void __launch_bounds__(256)
k_traverse(TravCtx c, int32_t* s_beg, int32_t* s_cnt, int32_t* w_beg, int32_t* w_cnt, int32_t* s_ids,
           int32_t* w_ids, int64_t cap_s, int64_t cap_w, long long* totals)
{
    constexpr bool FILL = MODE != 0;
    __shared__ int32_t front_all[4][2][kFrontCap];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + wv);   // one box per wavefront: uniform
    if (i >= c.n) return;
    int32_t* fa = front_all[wv][0];
    int32_t* fb = front_all[wv][1];
    const int64_t g = c.boxes[i];
    const int L = c.level[g];
    const int64_t pb = c.pbox[c.prob[g]];
    const int64_t jl = g - pb - level_base(L);        // index of the box within its level
    bool overflow = false, cap_overflow = false;
    long long src = 0;                                // near-field sources (one-pass mode)
    int nf;
    if (c.l0 == 0) {
        nf = 1;
        if (lane == 0) fa[0] = (int32_t)pb;           // the root is strong with itself
    } else {
        // the ancestor's strong list from the pool: only the entries that
        // were written (at most cs in the one-pass mode, where a longer list
        // is truncated and flagged)
        const int64_t a0 = pb + level_base(c.l0 - 1) + (jl >> (2 * (L - c.l0 + 1)));
        const int64_t ab = s_beg[a0];
        nf = s_cnt[a0];
        if (MODE == 2 && nf > c.cs) { cap_overflow = true; nf = c.cs; }
        if (nf > kFrontCap) { overflow = true; nf = kFrontCap; }
        for (int e = lane; e < nf; e += 64) fa[e] = (ab + e < cap_s) ? s_ids[ab + e] : (int32_t)pb;
    }
    wave_sync_l();
    int64_t sb = 0, wb = 0, lim_s = cap_s, lim_w = cap_w;
    if (MODE == 1) { sb = s_beg[g]; wb = w_beg[g]; }
    if (MODE == 2) { sb = g * c.cs; wb = g * c.cw; lim_s = sb + c.cs; lim_w = wb + c.cw; }
    int nw = 0;
    for (int k = (c.l0 == 0 ? 1 : c.l0); k <= L; ++k) {
        const int64_t anc = pb + level_base(k) + (jl >> (2 * (L - k)));
        const double* ga = c.geom + 4 * anc;
        const int64_t lb = level_base(k), lbp = level_base(k - 1);
        const int ncand = 4 * nf;
        const bool last = k == L;
        int nn = 0;
        for (int c0 = 0; c0 < ncand; c0 += 64) {
            const int idx = c0 + lane;
            bool valid = idx < ncand;
            bool weak = false;
            int32_t cc = 0;
            if (valid) {
                const int32_t q = fa[idx >> 2];
                const int64_t qj = (int64_t)q - pb - lbp;   // index of q within level k-1
                if (qj < 0 || qj >= (int64_t(1) << (2 * (k - 1)))) {
                    valid = false;                          // not a box of that level: never
                    overflow = true;                        // dereferenced, list rebuilt
                } else {
                    cc = (int32_t)(pb + lb + 4 * qj + (idx & 3));
                    weak = (cc != anc) && well_separated(ga, c.geom + 4 * (int64_t)cc, c.theta);
                }
            }
            const unsigned long long bs = __ballot(valid && !weak), bw = __ballot(valid && weak);
            const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
            if (valid && !weak) {
                const int o = nn + __popcll(bs & below);
                if (!last && o < kFrontCap) fb[o] = cc;
                if (FILL && last && sb + o < lim_s) s_ids[sb + o] = cc;
                if (MODE == 2 && last) src += c.box_count[cc];
            }
            if (FILL && last && valid && weak) {
                const int64_t o = wb + nw + __popcll(bw & below);
                if (o < lim_w) w_ids[o] = cc;
            }
            nn += __popcll(bs);
            if (last) nw += __popcll(bw);
        }
        if (!last && nn > kFrontCap) { overflow = true; nn = kFrontCap; }
        wave_sync_l();
        int32_t* t = fa; fa = fb; fb = t;
        nf = nn;
    }
    if (MODE == 2) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) src += __shfl_xor(src, o, 64);
    }
    // flags raised by any lane
    cap_overflow = __ballot(cap_overflow) != 0ull;
    overflow = __ballot(overflow) != 0ull;
    if (lane == 0) {
        if (L == 0) {                                  // a root (only in a pass with l0 = 0)
            nf = 1;
            nw = 0;
            if (FILL && sb < lim_s) s_ids[sb] = (int32_t)g;
        }
        if (MODE != 1) { s_cnt[g] = nf; w_cnt[g] = nw; }
        if (MODE == 2) {
            s_beg[g] = (int32_t)sb;
            w_beg[g] = (int32_t)wb;
            if (nf > c.cs || nw > c.cw) cap_overflow = true;
            if (nw > kChunkPairs) atomicOr((unsigned long long*)&totals[2], 8ull);
            if (L == 0) src = c.box_count[g];
            if (c.child0[g] < 0) {                      // a leaf: its near-field source count
                c.nsrc[g] = (int32_t)(src < INT32_MAX ? src : INT32_MAX);
                if (src > kChunkSrc) atomicOr((unsigned long long*)&totals[2], 4ull);
            }
        }
        if (cap_overflow) atomicOr((unsigned long long*)&totals[2], 1ull);
        if (overflow) atomicOr((unsigned long long*)&totals[2], 2ull);
    }
}

// totals cleared; the tree's error word (non-finite positions) becomes flag 16
__global__ void k_totals_init(long long* totals, const uint32_t* tree_err)
{
    if (threadIdx.x == 0) {
        totals[0] = 0; totals[1] = 0; totals[3] = 0;
        totals[2] = *tree_err ? 16 : 0;
    }
}

static void check_tree_flag(long long flag)
{
    if (flag & 16) throw Error(FMM_EINVAL, "non-finite position");
}

// Level ranges of the passes: the three deepest levels one at a time (by
// sibling groups), everything above them in one pass from the root; or, for
// a layout whose frontiers overflowed, every level on its own.
static std::vector<std::pair<int, int>> traversal_passes(int levels, bool single = false)
{
    std::vector<std::pair<int, int>> r;
    const int top = levels - 1;
    if (single) {
        // one level per pass (sibling groups below the root): no frontier,
        // lists of any length
        for (int l = 0; l <= top; ++l) r.push_back({l, l});
        return r;
    }
    if (levels <= 4) { r.push_back({0, top}); return r; }
    r.push_back({0, top - 3});
    for (int l = top - 2; l <= top; ++l) r.push_back({l, l});
    return r;
}

// A sibling group whose parent's strong list is longer than this is handled
// by a whole workgroup (k_traverse_long) in the count and fill passes: one
// wavefront walking a list of thousands of boxes (clustered points, where a
// leaf holding a point far from the others is strong with most of its level)
// took milliseconds alone.
constexpr int kLongList = 1024;
constexpr int kLongWaves = 16;      // wavefronts of a k_traverse_long workgroup
constexpr int kLongGroups = 4;      // runs of 64 candidates per wavefront and loop trip
constexpr int kLongGrid = 256;      // its workgroups (they take the work units in turn)
constexpr int kLongUnits = 16;      // work units of a split group (runs of consecutive trips)
constexpr int kLongSplitCap = 4096; // queued groups split into units (later ones are one unit)
constexpr int kLongFromLevel = 6;   // a parent level of fewer than kLongList boxes has no long list

// Candidates taken per loop trip of k_traverse_sib: four groups of 64 whose
// id and geometry loads are all issued before the first test, so a long
// parent list costs one memory round trip per 256 candidates.
constexpr int kCandGroups = 4;

// A single level l >= 1, one wavefront per group of four siblings: every
// candidate (a child of an entry of the parent's strong list, read from the
// pool, so the list may have any length) is loaded once and tested against
// the four siblings; each sibling's strong and weak lists are compacted by
// ballots in candidate order, as in k_traverse.  MODE 0 counts, MODE 1 fills
// at the scanned offsets, MODE 2 fills at fixed per-box capacities and also
// counts each leaf's near-field sources and raises the chunk flags.

template <int MODE>
__global__ void __launch_bounds__(256)
k_traverse_sib(TravCtx c, int32_t* s_beg, int32_t* s_cnt, int32_t* w_beg, int32_t* w_cnt, int32_t* s_ids,
               int32_t* w_ids, int64_t cap_s, int64_t cap_w, long long* totals)
{
    constexpr bool FILL = MODE != 0;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // one sibling group per wavefront: its values are uniform (scalar registers)
    const int i = __builtin_amdgcn_readfirstlane((blockIdx.x * 4 + wv) * 4);
    if (i >= c.n) return;
    int64_t g0, pb;                                   // first of four siblings, its problem's base
    int L;
    if (c.first >= 0) {
        g0 = c.first + i;
        L = c.l0;
        pb = 0;
    } else {
        g0 = c.boxes[i];
        L = c.level[g0];
        pb = c.pbox[c.prob[g0]];
    }
    const int64_t jl = g0 - pb - level_base(L);
    bool overflow = false, cap_overflow = false;
    const int64_t a0 = pb + level_base(L - 1) + (jl >> 2);
    // the parent's strong list: with fixed capacities it starts at a0 * cs,
    // so the ids of the first loop trip are loaded beside its length (the
    // entries past the length are loaded but never used)
    const int64_t ab = MODE == 2 ? a0 * c.cs : (int64_t)s_beg[a0];
    int32_t q_first[kCandGroups];
    if constexpr (MODE == 2) {
#pragma unroll
        for (int u = 0; u < kCandGroups; ++u) {
            const int64_t e = ab + ((64 * u + lane) >> 2);
            q_first[u] = s_ids[e < cap_s ? e : cap_s - 1];
        }
    }
    int nf = s_cnt[a0];
    if (MODE == 2 && nf > c.cs) { cap_overflow = true; nf = c.cs; }
    // a long parent list: the count pass queues the group for
    // k_traverse_long, the fill pass finds it queued
    if (MODE != 2 && c.long_q != nullptr && nf > kLongList) {
        if (MODE == 0 && lane == 0) c.long_q[atomicAdd(c.long_n, 1)] = i;
        return;
    }
    double gx[4], gy[4], gr[4];
    int64_t sb[4], wb[4], ls[4], lw[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int64_t g = g0 + t;
        const double* gg = c.geom + 4 * g;
        gx[t] = gg[0]; gy[t] = gg[1]; gr[t] = gg[2];
        sb[t] = 0; wb[t] = 0; ls[t] = cap_s; lw[t] = cap_w;
        if (MODE == 1) { sb[t] = s_beg[g]; wb[t] = w_beg[g]; }
        if (MODE == 2) { sb[t] = g * c.cs; wb[t] = g * c.cw; ls[t] = sb[t] + c.cs; lw[t] = wb[t] + c.cw; }
    }
    const int64_t lb = level_base(L), lbp = level_base(L - 1);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int ns[4] = {0, 0, 0, 0}, nw[4] = {0, 0, 0, 0};
    long long src[4] = {0, 0, 0, 0};
    const int64_t ncand = 4 * (int64_t)nf;
    for (int64_t c0 = 0; c0 < ncand; c0 += 64 * kCandGroups) {
        bool valid[kCandGroups];
        int32_t cc[kCandGroups];
        double cg[kCandGroups][4];
        long long cnt[kCandGroups];
#pragma unroll
        for (int u = 0; u < kCandGroups; ++u) {
            const int64_t idx = c0 + 64 * u + lane;
            valid[u] = idx < ncand;
            const int64_t e = ab + (idx >> 2);
            int32_t q = (int32_t)(pb + lbp);
            if (valid[u]) {
                if (MODE == 2 && c0 == 0) q = e < cap_s ? q_first[u] : (int32_t)pb;
                else q = e < cap_s ? s_ids[e] : (int32_t)pb;
            }
            const int64_t qj = (int64_t)q - pb - lbp;
            if (valid[u] && (qj < 0 || qj >= (int64_t(1) << (2 * (L - 1))))) {
                valid[u] = false;                       // not a box of that level: never
                overflow = true;                        // dereferenced, list rebuilt
            }
            cc[u] = valid[u] ? (int32_t)(pb + lb + 4 * qj + (idx & 3)) : (int32_t)g0;
        }
#pragma unroll
        for (int u = 0; u < kCandGroups; ++u) {
            const double* gc = c.geom + 4 * (int64_t)(valid[u] ? cc[u] : (int32_t)g0);
            cg[u][0] = gc[0]; cg[u][1] = gc[1]; cg[u][2] = gc[2]; cg[u][3] = 0.0;
            cnt[u] = MODE == 2 && valid[u] ? c.box_count[cc[u]] : 0;
        }
#pragma unroll
        for (int u = 0; u < kCandGroups; ++u) {
            if (c0 + 64 * u >= ncand) break;       // uniform: no candidate left
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const double gb[4] = {gx[t], gy[t], gr[t], 0.0};
                const bool weak = valid[u] && (cc[u] != g0 + t) && well_separated(gb, cg[u], c.theta);
                const bool strong = valid[u] && !weak;
                const unsigned long long bs = __ballot(strong), bw = __ballot(weak);
                if (FILL && strong) {
                    const int64_t o = sb[t] + ns[t] + __popcll(bs & below);
                    if (o < ls[t]) s_ids[o] = cc[u];
                }
                if (FILL && weak) {
                    const int64_t o = wb[t] + nw[t] + __popcll(bw & below);
                    if (o < lw[t]) w_ids[o] = cc[u];
                }
                if (MODE == 2 && strong) src[t] += cnt[u];
                ns[t] += __popcll(bs);
                nw[t] += __popcll(bw);
            }
        }
    }
    if (MODE == 2) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) src[t] += __shfl_xor(src[t], o, 64);
    }
    cap_overflow = __ballot(cap_overflow) != 0ull;
    overflow = __ballot(overflow) != 0ull;
    if (lane == 0) {
        unsigned long long fl = 0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t g = g0 + t;
            if (MODE != 1) { s_cnt[g] = ns[t]; w_cnt[g] = nw[t]; }
            if (MODE == 2) {
                s_beg[g] = (int32_t)sb[t];
                w_beg[g] = (int32_t)wb[t];
                if (ns[t] > c.cs || nw[t] > c.cw) cap_overflow = true;
                if (nw[t] > kChunkPairs) fl |= 8ull;
                if (c.child0[g] < 0) {                  // a leaf: its near-field source count
                    c.nsrc[g] = (int32_t)(src[t] < INT32_MAX ? src[t] : INT32_MAX);
                    if (src[t] > kChunkSrc) fl |= 4ull;
                }
            }
        }
        if (cap_overflow) fl |= 1ull;
        if (overflow) fl |= 2ull;
        if (fl) atomicOr((unsigned long long*)&totals[2], fl);
    }
}

// The count (MODE 0) and fill (MODE 1) passes of the sibling groups that
// k_traverse_sib queued, by a workgroup of kLongWaves wavefronts per work
// unit, kLongGroups * 64 * kLongWaves candidates per loop trip (run r = u *
// kLongWaves + w of 64 belongs to wavefront w, u < kLongGroups; every load of
// a trip is issued before its first test).  The strong and weak counts of
// every run go through LDS and are scanned over the runs, so the lists are
// written in candidate order, as k_traverse_sib writes them.  The first
// kLongSplitCap queued groups are split into kLongUnits units of consecutive
// trips: the count pass writes each unit's counts to ucnt, k_long_finish
// turns them into offsets (exclusive prefixes in unit order) and the
// siblings' list lengths, and the fill pass starts each unit at its offset.
// Later queued groups are one unit.  The workgroups take the units in turn.
template <int MODE>
__global__ void __launch_bounds__(1024)
k_traverse_long(TravCtx c, const int32_t* __restrict__ queue, const int32_t* __restrict__ qn, int32_t* ucnt,
                int32_t* s_beg, int32_t* s_cnt, int32_t* w_beg, int32_t* w_cnt, int32_t* s_ids, int32_t* w_ids,
                int64_t cap_s, int64_t cap_w, long long* totals)
{
    static_assert(MODE == 0 || MODE == 1, "count or fill");
    constexpr int G = kLongGroups, NR = kLongGroups * kLongWaves;   // runs of 64 per trip
    static_assert(NR == 64, "one run per lane in the scan of a trip's counts");
    constexpr int64_t kTrip = 64 * NR;                               // candidates per trip
    __shared__ int cnt_s[4][NR], cnt_w[4][NR];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int nq = *qn;
    const int ks = min(nq, kLongSplitCap);                           // split groups
    const int64_t nunits = (int64_t)ks * kLongUnits + (nq - ks);
    bool overflow = false;
    for (int64_t unit = blockIdx.x; unit < nunits; unit += gridDim.x) {
        const bool split = unit < (int64_t)ks * kLongUnits;
        const int k = split ? (int)(unit / kLongUnits) : ks + (int)(unit - (int64_t)ks * kLongUnits);
        const int j = split ? (int)(unit % kLongUnits) : 0;
        const int i = queue[k];
        int64_t g0, pb;
        int L;
        if (c.first >= 0) {
            g0 = c.first + i;
            L = c.l0;
            pb = 0;
        } else {
            g0 = c.boxes[i];
            L = c.level[g0];
            pb = c.pbox[c.prob[g0]];
        }
        const int64_t jl = g0 - pb - level_base(L);
        const int64_t a0 = pb + level_base(L - 1) + (jl >> 2);
        const int64_t ab = s_beg[a0];
        const int nf = s_cnt[a0];
        const int64_t ncand = 4 * (int64_t)nf;
        const int64_t ntrip = (ncand + kTrip - 1) / kTrip;
        int64_t tr0 = 0, tr1 = ntrip;                                // this unit's trips
        if (split) {
            const int64_t tpu = (ntrip + kLongUnits - 1) / kLongUnits;
            tr0 = min(ntrip, (int64_t)j * tpu);
            tr1 = min(ntrip, tr0 + tpu);
        }
        double gx[4], gy[4], gr[4];
        int64_t sb[4], wb[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const double* gg = c.geom + 4 * (g0 + t);
            gx[t] = gg[0]; gy[t] = gg[1]; gr[t] = gg[2];
            sb[t] = 0;
            wb[t] = 0;
            if (MODE == 1) {
                sb[t] = s_beg[g0 + t];
                wb[t] = w_beg[g0 + t];
                if (split) {                            // the unit's offsets in the lists
                    const int64_t uo = ((int64_t)k * kLongUnits + j) * 8 + 2 * t;
                    sb[t] += ucnt[uo];
                    wb[t] += ucnt[uo + 1];
                }
            }
        }
        const int64_t lb = level_base(L), lbp = level_base(L - 1);
        int ns[4] = {0, 0, 0, 0}, nw[4] = {0, 0, 0, 0};
        for (int64_t tr = tr0; tr < tr1; ++tr) {
            const int64_t c0 = tr * kTrip;
            bool valid[G];
            int32_t cc[G];
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const int64_t idx = c0 + 64 * (u * kLongWaves + wv) + lane;
                valid[u] = idx < ncand;
                const int64_t e = ab + (idx >> 2);
                int32_t q = (int32_t)(pb + lbp);
                if (valid[u]) q = e < cap_s ? s_ids[e] : (int32_t)pb;
                const int64_t qj = (int64_t)q - pb - lbp;
                if (valid[u] && (qj < 0 || qj >= (int64_t(1) << (2 * (L - 1))))) {
                    valid[u] = false;                   // not a box of that level: never
                    overflow = true;                    // dereferenced, list rebuilt
                }
                cc[u] = valid[u] ? (int32_t)(pb + lb + 4 * qj + (idx & 3)) : (int32_t)g0;
            }
            double cg[G][4];
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const double* gc = c.geom + 4 * (int64_t)cc[u];
                cg[u][0] = gc[0]; cg[u][1] = gc[1]; cg[u][2] = gc[2]; cg[u][3] = 0.0;
            }
            // bit 2 (t G + u) strong, the next bit weak
            uint32_t bits = 0;
#pragma unroll
            for (int u = 0; u < G; ++u)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const double gb[4] = {gx[t], gy[t], gr[t], 0.0};
                    const bool weak = valid[u] && (cc[u] != g0 + t) && well_separated(gb, cg[u], c.theta);
                    const bool strong = valid[u] && !weak;
                    bits |= ((uint32_t)strong | ((uint32_t)weak << 1)) << (2 * (t * G + u));
                    const unsigned long long bs = __ballot(strong), bw = __ballot(weak);
                    if (lane == 0) {
                        cnt_s[t][u * kLongWaves + wv] = __popcll(bs);
                        cnt_w[t][u * kLongWaves + wv] = __popcll(bw);
                    }
                }
            __syncthreads();
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                // lane r holds the counts of run r; inclusive scans over the runs
                const int a = cnt_s[t][lane], b = cnt_w[t][lane];
                const int xa = wave_incl_scan(a), xb = wave_incl_scan(b);
                if (MODE == 1) {
                    const int ea = xa - a, eb = xb - b;
#pragma unroll
                    for (int u = 0; u < G; ++u) {
                        const int r = u * kLongWaves + wv;      // this wavefront's run of group u
                        const int ps = __builtin_amdgcn_readlane(ea, r), pw = __builtin_amdgcn_readlane(eb, r);
                        const int sh = 2 * (t * G + u);
                        const bool strong = (bits >> sh) & 1u, weak = (bits >> (sh + 1)) & 1u;
                        const unsigned long long bs = __ballot(strong), bw = __ballot(weak);
                        if (strong) {
                            const int64_t o = sb[t] + ns[t] + ps + __popcll(bs & below);
                            if (o < cap_s) s_ids[o] = cc[u];
                        }
                        if (weak) {
                            const int64_t o = wb[t] + nw[t] + pw + __popcll(bw & below);
                            if (o < cap_w) w_ids[o] = cc[u];
                        }
                    }
                }
                ns[t] += __builtin_amdgcn_readlane(xa, 63);
                nw[t] += __builtin_amdgcn_readlane(xb, 63);
            }
            __syncthreads();   // the counts are rewritten by the next trip
        }
        if (MODE == 0 && threadIdx.x == 0) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (split) {
                    const int64_t uo = ((int64_t)k * kLongUnits + j) * 8 + 2 * t;
                    ucnt[uo] = ns[t];
                    ucnt[uo + 1] = nw[t];
                } else {
                    s_cnt[g0 + t] = ns[t];
                    w_cnt[g0 + t] = nw[t];
                }
            }
        }
    }
    if (__ballot(overflow) != 0ull && lane == 0) atomicOr((unsigned long long*)&totals[2], 2ull);
}

// Between the count and the fill pass: for every split group (thread: group
// k, value v = 2 sibling + strong/weak), its units' counts become exclusive
// prefixes in unit order, and their sum the sibling's list length.
__global__ void k_long_finish(TravCtx c, const int32_t* __restrict__ queue, const int32_t* __restrict__ qn,
                              int32_t* ucnt, int32_t* s_cnt, int32_t* w_cnt)
{
    const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int ks = min(*qn, kLongSplitCap);
    if (x >= (int64_t)ks * 8) return;
    const int k = (int)(x >> 3), v = (int)(x & 7);
    int run = 0;
    for (int jj = 0; jj < kLongUnits; ++jj) {
        int32_t* pv = ucnt + ((int64_t)k * kLongUnits + jj) * 8 + v;
        const int cval = *pv;
        *pv = run;
        run += cval;
    }
    const int i = queue[k];
    const int64_t g0 = c.first >= 0 ? c.first + i : (int64_t)c.boxes[i];
    if (v & 1) w_cnt[g0 + (v >> 1)] = run;
    else s_cnt[g0 + (v >> 1)] = run;
}

__global__ void k_zero_counter(int32_t* p) { if (threadIdx.x == 0) *p = 0; }

static void build_lists_traversal(Plan& pl, hipStream_t s, int64_t cap_s, int64_t cap_w, long long* totals,
                                  const int64_t* pbox, long long* bsum, long long* snap, bool single)
{
    Tree& t = *pl.tree;
    TreeSchedule& sc = *t.sched;
    const PlanExtra& ex = *pl.ex;
    k_totals_init<<<1, 64, 0, s>>>(totals, t.err.p);
    // the queue of sibling groups with long parent lists: its count, then at
    // most one entry per group of the largest sibling pass
    int64_t max_groups = 0;
    for (auto [l0, l1] : traversal_passes(sc.max_levels, single))
        if (l0 == l1 && l0 >= kLongFromLevel)
            max_groups = std::max<int64_t>(max_groups, (ex.level_boxes_off[l1 + 1] - ex.level_boxes_off[l0]) / 4);
    DBuf<int32_t> lq, ucnt;
    if (max_groups > 0) {
        lq.alloc(max_groups + 1, s);
        ucnt.alloc((size_t)std::min<int64_t>(max_groups, kLongSplitCap) * kLongUnits * 8, s);
    }
    for (auto [l0, l1] : traversal_passes(sc.max_levels, single)) {
        TravCtx c;
        c.boxes = ex.d_level_boxes.p + ex.level_boxes_off[l0];
        c.n = (int)(ex.level_boxes_off[l1 + 1] - ex.level_boxes_off[l0]);
        if (c.n == 0) continue;
        c.l0 = l0;
        c.cs = c.cw = 0;
        c.prob = sc.d_box_prob.p; c.level = sc.d_box_level.p; c.pbox = pbox;
        c.geom = t.geom.p; c.theta = pl.theta;
        c.first = sc.nprob == 1 && sc.pbox[0] == 0 && l0 == l1 ? level_base(l0) : -1;
        c.child0 = nullptr; c.box_count = nullptr; c.nsrc = nullptr;
        const bool sib = l0 == l1 && l0 >= 1;   // one level: sibling groups
        const bool longq = sib && l0 >= kLongFromLevel;
        if (longq) {
            c.long_n = lq.p;
            c.long_q = lq.p + 1;
            k_zero_counter<<<1, 64, 0, s>>>(c.long_n);
        }
        const unsigned grid = (unsigned)((c.n + 3) / 4), sgrid = (unsigned)((c.n / 4 + 3) / 4);
        if (sib)
            k_traverse_sib<0><<<sgrid, 256, 0, s>>>(c, pl.s_beg.p, pl.s_cnt.p, pl.w_beg.p, pl.w_cnt.p, pl.s_ids.p,
                                                    pl.w_ids.p, cap_s, cap_w, totals);
        else
            k_traverse<0><<<grid, 256, 0, s>>>(c, pl.s_beg.p, pl.s_cnt.p, pl.w_beg.p, pl.w_cnt.p, pl.s_ids.p,
                                               pl.w_ids.p, cap_s, cap_w, totals);
        if (longq) {
            k_traverse_long<0><<<kLongGrid, 64 * kLongWaves, 0, s>>>(c, c.long_q, c.long_n, ucnt.p, pl.s_beg.p,
                                                                     pl.s_cnt.p, pl.w_beg.p, pl.w_cnt.p, pl.s_ids.p,
                                                                     pl.w_ids.p, cap_s, cap_w, totals);
            k_long_finish<<<(unsigned)(kLongSplitCap * 8 / 256), 256, 0, s>>>(c, c.long_q, c.long_n, ucnt.p,
                                                                              pl.s_cnt.p, pl.w_cnt.p);
        }
        const int nb = (c.n + 1023) / 1024;
        k_scan_reduce<<<nb, 1024, 0, s>>>(c.boxes, c.n, pl.s_cnt.p, pl.w_cnt.p, bsum, totals, snap);
        k_scan_apply<<<nb, 1024, 0, s>>>(c.boxes, c.n, pl.s_cnt.p, pl.w_cnt.p, bsum, snap, pl.s_beg.p,
                                         pl.w_beg.p, totals, cap_s, cap_w);
        if (sib)
            k_traverse_sib<1><<<sgrid, 256, 0, s>>>(c, pl.s_beg.p, pl.s_cnt.p, pl.w_beg.p, pl.w_cnt.p, pl.s_ids.p,
                                                    pl.w_ids.p, cap_s, cap_w, totals);
        else
            k_traverse<1><<<grid, 256, 0, s>>>(c, pl.s_beg.p, pl.s_cnt.p, pl.w_beg.p, pl.w_cnt.p, pl.s_ids.p,
                                               pl.w_ids.p, cap_s, cap_w, totals);
        if (longq)
            k_traverse_long<1><<<kLongGrid, 64 * kLongWaves, 0, s>>>(c, c.long_q, c.long_n, ucnt.p, pl.s_beg.p,
                                                                     pl.s_cnt.p, pl.w_beg.p, pl.w_cnt.p, pl.s_ids.p,
                                                                     pl.w_ids.p, cap_s, cap_w, totals);
        check_launch("traversal lists");
    }
}

// One pass per level range, lists written at fixed per-box capacities (per
// tree layout: they start at kCapStrong / kCapWeak and grow to the longest
// lists seen when a build overflowed them).
constexpr int kCapStrong = 96, kCapWeak = 224;
constexpr int64_t kMaxPaddedPools = int64_t(1) << 30;   // bytes of the fixed-capacity id pools

__global__ void __launch_bounds__(256)
k_max_counts(int64_t n, const int32_t* s_cnt, const int32_t* w_cnt, unsigned int* out)
{
    const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
    int a = i < n ? s_cnt[i] : 0, b = i < n ? w_cnt[i] : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) { a = max(a, __shfl_xor(a, o, 64)); b = max(b, __shfl_xor(b, o, 64)); }
    if ((threadIdx.x & 63) == 0) { atomicMax(&out[0], (unsigned)a); atomicMax(&out[1], (unsigned)b); }
}

static void grow_capacities(Plan& pl, hipStream_t s)
{
    TreeSchedule& sc = *pl.tree->sched;
    DBuf<unsigned int> mx;
    mx.alloc(2, s);
    FMM_HIP(hipMemsetAsync(mx.p, 0, 2 * sizeof(unsigned int), s));
    k_max_counts<<<(unsigned)((sc.nbox + 255) / 256), 256, 0, s>>>(sc.nbox, pl.s_cnt.p, pl.w_cnt.p, mx.p);
    check_launch("max list counts");
    unsigned int h[2];
    FMM_HIP(hipMemcpyAsync(h, mx.p, sizeof(h), hipMemcpyDeviceToHost, s));
    FMM_HIP(hipStreamSynchronize(s));
    PlanExtra& ex = *pl.ex;
    ex.cap_strong = std::max<int>(ex.cap_strong, (int)((h[0] + 31) / 32 * 32));
    ex.cap_weak = std::max<int>(ex.cap_weak, (int)((h[1] + 31) / 32 * 32));
    // a few very long lists (clustered points) would make the padded pools
    // huge: this layout then keeps the compact build
    if ((int64_t)sc.nbox * (ex.cap_strong + ex.cap_weak) * (int64_t)sizeof(int32_t) > kMaxPaddedPools)
        ex.compact_only = true;
}

static void build_lists_direct(Plan& pl, hipStream_t s, long long* totals, const int64_t* pbox)
{
    Tree& t = *pl.tree;
    TreeSchedule& sc = *t.sched;
    const PlanExtra& ex = *pl.ex;
    k_totals_init<<<1, 64, 0, s>>>(totals, t.err.p);
    for (auto [l0, l1] : traversal_passes(sc.max_levels)) {
        TravCtx c;
        c.boxes = ex.d_level_boxes.p + ex.level_boxes_off[l0];
        c.n = (int)(ex.level_boxes_off[l1 + 1] - ex.level_boxes_off[l0]);
        if (c.n == 0) continue;
        c.l0 = l0;
        c.cs = ex.cap_strong;
        c.cw = ex.cap_weak;
        c.prob = sc.d_box_prob.p; c.level = sc.d_box_level.p; c.pbox = pbox;
        c.geom = t.geom.p; c.theta = pl.theta;
        c.first = sc.nprob == 1 && sc.pbox[0] == 0 && l0 == l1 ? level_base(l0) : -1;
        c.child0 = ex.child0.p; c.box_count = sc.d_box_count.p; c.nsrc = pl.nsrc.p;
        if (l0 == l1 && l0 >= 1) {
            // one level: sibling groups (the level's box list is four-aligned)
            const int groups = c.n / 4;
            k_traverse_sib<2><<<(unsigned)((groups + 3) / 4), 256, 0, s>>>(c, pl.s_beg.p, pl.s_cnt.p, pl.w_beg.p,
                                                                          pl.w_cnt.p, pl.s_ids.p, pl.w_ids.p,
                                                                          (int64_t)pl.s_ids.n, (int64_t)pl.w_ids.n,
                                                                          totals);
        } else {
            k_traverse<2><<<(unsigned)((c.n + 3) / 4), 256, 0, s>>>(c, pl.s_beg.p, pl.s_cnt.p, pl.w_beg.p,
                                                                    pl.w_cnt.p, pl.s_ids.p, pl.w_ids.p,
                                                                    (int64_t)pl.s_ids.n, (int64_t)pl.w_ids.n,
                                                                    totals);
        }
        check_launch("one-pass lists");
    }
}

// list sizes of all boxes (totals[0], totals[1]) by block sums
__global__ void __launch_bounds__(1024)
k_sum_counts(int64_t n, const int32_t* s_cnt, const int32_t* w_cnt, long long* totals)
{
    __shared__ long long sh[2][16];
    const int64_t i = blockIdx.x * (int64_t)1024 + threadIdx.x;
    long long a = 0, b = 0;
    if (i < n) { a = s_cnt[i]; b = w_cnt[i]; }
    block_sum2(a, b, sh);
    if (threadIdx.x == 0) {
        atomicAdd((unsigned long long*)&totals[0], (unsigned long long)a);
        atomicAdd((unsigned long long*)&totals[1], (unsigned long long)b);
    }
}

void list_totals_device(Plan& pl, hipStream_t s)
{
    if (pl.totals_known) return;
    TreeSchedule& sc = *pl.tree->sched;
    DBuf<long long> totals;
    totals.alloc(4, s);
    k_totals_init<<<1, 64, 0, s>>>(totals.p, pl.tree->err.p);
    k_sum_counts<<<(unsigned)((sc.nbox + 1023) / 1024), 1024, 0, s>>>(sc.nbox, pl.s_cnt.p, pl.w_cnt.p, totals.p);
    const int nl = (int)sc.nleaf;
    k_count_p2p<<<(nl + 3) / 4, 256, 0, s>>>(pl.ex->leaves.p, nl, sc.d_box_count.p, pl.s_beg.p, pl.s_cnt.p,
                                                 pl.s_ids.p, totals.p, (int64_t)pl.s_ids.n);
    check_launch("list totals");
    long long h[4];
    FMM_HIP(hipMemcpyAsync(h, totals.p, sizeof(h), hipMemcpyDeviceToHost, s));
    FMM_HIP(hipStreamSynchronize(s));
    pl.n_strong = h[0];
    pl.n_weak = h[1];
    pl.n_p2p_pairs = h[3];
    pl.totals_known = true;
}

// Enqueue the list build without waiting: the one-pass build when the
// capacities allow it.  build_lists_finish reads its flags (one
// synchronisation) and runs the compact or level-wise build if needed.
// The kernels go to `ls`; the plan's buffers are allocated on `as` (the
// stream that later uses and releases them, joined to `ls` by events).
void build_lists_begin(Plan& pl, hipStream_t ls, hipStream_t as)
{
    Tree& t = *pl.tree;
    TreeSchedule& sc = *t.sched;
    int64_t nb = sc.nbox;
    hipStream_t s = ls;
    pl.s_beg.alloc(nb, as); pl.s_cnt.alloc(nb, as); pl.w_beg.alloc(nb, as); pl.w_cnt.alloc(nb, as);
    pl.lt_totals.alloc(4, as);
    pl.list_stream = s;
    PlanExtra& ex = *pl.ex;
    if (ex.cap_strong == 0) { ex.cap_strong = kCapStrong; ex.cap_weak = kCapWeak; }
    pl.lists_direct = nb * std::max(ex.cap_strong, ex.cap_weak) < INT32_MAX && !ex.levelwise_only &&
                      !ex.compact_only;
    if (pl.lists_direct) {
        pl.s_ids.alloc(nb * ex.cap_strong, as);
        pl.w_ids.alloc(nb * ex.cap_weak, as);
        pl.nsrc.alloc(nb, as);
        build_lists_direct(pl, s, pl.lt_totals.p, sc.d_pbox.p);
        if (!pl.ev_lists_k) FMM_HIP(hipEventCreateWithFlags(&pl.ev_lists_k, hipEventDisableTiming));
        FMM_HIP(hipEventRecord(pl.ev_lists_k, s));
        // the flags go to a pinned word now, so that reading them later does
        // not wait for work enqueued after the lists
        pl.flag_slot = flag_slot_acquire();
        if (pl.flag_slot >= 0) {
            if (!pl.ev_lists) FMM_HIP(hipEventCreateWithFlags(&pl.ev_lists, hipEventDisableTiming));
            FMM_HIP(hipMemcpyAsync((void*)flag_slot_ptr(pl.flag_slot), pl.lt_totals.p + 2, sizeof(long long),
                                   hipMemcpyDeviceToHost, s));
            FMM_HIP(hipEventRecord(pl.ev_lists, s));
        }
    }
    pl.lists_pending = true;
}

void release_list_flag(Plan& pl)
{
    if (pl.flag_slot >= 0) {
        (void)hipEventSynchronize(pl.ev_lists);   // the copy into the word has landed
        flag_slot_release(pl.flag_slot);
        pl.flag_slot = -1;
    }
    if (pl.ev_lists) { (void)hipEventDestroy(pl.ev_lists); pl.ev_lists = nullptr; }
}

void build_lists_finish(Plan& pl)
{
    if (!pl.lists_pending) return;
    pl.lists_pending = false;
    hipStream_t s = pl.list_stream;
    Tree& t = *pl.tree;
    TreeSchedule& sc = *t.sched;
    int64_t nb = sc.nbox;
    long long* totals_p = pl.lt_totals.p;
    const int64_t* pbox_p = sc.d_pbox.p;
    PlanExtra& ex = *pl.ex;
    bool grow = false;
    if (pl.lists_direct) {
        long long flag = 0;
        if (pl.flag_slot >= 0) {
            FMM_HIP(hipEventSynchronize(pl.ev_lists));
            flag = *flag_slot_ptr(pl.flag_slot);
            release_list_flag(pl);
        } else {
            FMM_HIP(hipMemcpyAsync(&flag, totals_p + 2, sizeof(flag), hipMemcpyDeviceToHost, s));
            FMM_HIP(hipStreamSynchronize(s));
        }
        pl.list_flag = flag;
        // an evaluation enqueued ahead of these flags skipped its list work
        // (flag set); nothing below may touch the lists or the flag word
        // before that evaluation has drained
        if (flag != 0 && pl.ev_spec) FMM_HIP(hipStreamWaitEvent(s, pl.ev_spec, 0));
        check_tree_flag(flag);
        if ((flag & 3) == 0) {
            pl.totals_known = false;    // list sizes and pair counts are summed on request
            pl.split_p2p = (flag & 4) != 0;
            pl.split_m2l = (flag & 8) != 0;
            return;
        }
        grow = (flag & 2) == 0;         // capacities too small, no frontier overflow
        if (flag & 2) ex.levelwise_only = true;
    }
    DBuf<long long> snap; snap.alloc(2, s);
    DBuf<long long> bsum; bsum.alloc(2 * ((nb + 1023) / 1024), s);
    // pool sizes: a per-box guess, or the totals of the last build of this
    // layout grown by a quarter when larger, so that a layout whose lists
    // outgrow the guess (clustered points) is built once, not twice
    int64_t cap_s = std::max<int64_t>({pl.n_strong, 24 * nb + 1024, ex.pool_strong});
    int64_t cap_w = std::max<int64_t>({pl.n_weak, 64 * nb + 1024, ex.pool_weak});
    bool single = ex.levelwise_only;
    for (int attempt = 0; attempt < 4; ++attempt) {
        pl.s_ids.alloc(cap_s, s);
        pl.w_ids.alloc(cap_w, s);
        build_lists_traversal(pl, s, cap_s, cap_w, totals_p, pbox_p, bsum.p, snap.p, single);
        long long h[4];
        FMM_HIP(hipMemcpyAsync(h, totals_p, sizeof(h), hipMemcpyDeviceToHost, s));
        FMM_HIP(hipStreamSynchronize(s));
        check_tree_flag(h[2]);
        if ((h[2] & 2) && !single) {        // a frontier overflowed: one level per pass
            single = true;
            ex.levelwise_only = true;
            continue;
        }
        pl.n_strong = h[0];
        pl.n_weak = h[1];
        pl.totals_known = false;            // the pair count is summed on request
        ex.pool_strong = h[0] + h[0] / 4 + 1024;
        ex.pool_weak = h[1] + h[1] / 4 + 1024;
        if (!(h[2] & 3)) {
            if (grow) grow_capacities(pl, s);
            pl.split_p2p = pl.split_m2l = true;   // decided by the chunk counts
            return;
        }
        cap_s = ex.pool_strong;
        cap_w = ex.pool_weak;
    }
    throw Error(FMM_EDEVICE, "connectivity lists did not fit after growing the pools");
}

void build_lists_device(Plan& pl, hipStream_t s)
{
    build_lists_begin(pl, s, s);
    build_lists_finish(pl);
}

}  // namespace fmm
