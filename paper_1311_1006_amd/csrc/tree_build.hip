// tree_build.hip -- balanced median-split tree (Sec. 2.2) on gfx950.
//
// Every box is split in four by two successive binary splits.  A binary
// split cuts the longer side of the tight bounding box of the points being
// split (x when equal) and sends the floor(n/2) points smallest in
// (coordinate, input index) to the first half.  Because every split halves a
// count exactly, the size and position of every segment depend on N only;
// the host precomputes them and the device only decides membership.
//
// Device pipeline for one build (all problems of a batch at once):
//   init        copy positions into SoA buffers, bounding box of each root,
//               finiteness check;
//   per global stage s (segments larger than one workgroup's LDS):
//     hist1     256-bucket histogram of the split coordinate per segment
//               (buckets are equal-width in value over a range that holds
//               the segment, hence monotone in the coordinate): at stage 0
//               a kernel of its own over the root's bounding box; at later
//               stages the parent stage's partition has already counted its
//               children on both axes over the parent's bounding box;
//     hist2     if the bucket holding the median rank has too many points,
//               a second 2048-bucket histogram inside that bucket;
//     collect   each tile counts its points below the median's bucket and
//               appends the points of that bucket to a candidate list (an
//               exact single-workgroup radix select is the fallback for
//               pathological ties);
//     partition every tile takes the exact median (coordinate, index) from
//               the sorted candidates and its output offset, then does a
//               stable two-way partition into the next buffer, with the
//               bounding boxes of both halves (atomic min/max on
//               order-preserving integer images of the doubles) and the
//               children's histograms for the next stage;
//   lds split   each remaining segment (<= 4096 points) is finished by one
//               workgroup: the points are sorted once by (x, index) and once
//               by (y, index); every later split keeps both lists sorted by
//               a stable partition of the list of the other axis;
//   geometry    box centre (bbox midpoint) and radius (half diagonal),
//               computed with explicitly rounded operations so that they are
//               bit-identical to a plain IEEE evaluation, and the scaling
//               radius (r, or the nearest ancestor's r when r = 0).
// The point order inside a segment after a stable partition is a function of
// the input order only, and the final order inside a leaf is sorted by
// (x, index), so the whole build is deterministic.
#include <algorithm>
#include <cstring>

#include "fmm_internal.h"
#include "kernels_common.h"

// Box geometry, split axes and the theta-criterion must round every product
// and sum on its own (no fused multiply-add), like a plain IEEE evaluation.
#pragma clang fp contract(off)

namespace fmm {

// ------------------------------------------------------------------ schedule

static void seg_range(int64_t off, int64_t n, int s, int64_t j, int64_t* start, int64_t* cnt)
{
    int64_t st = off, c = n;
    for (int t = s - 1; t >= 0; --t) {
        int64_t h = c / 2;
        if ((j >> t) & 1) { st += h; c -= h; } else c = h;
    }
    *start = st; *cnt = c;
}

TreeSchedule* make_schedule(const std::vector<int64_t>& off, const std::vector<int>& L)
{
    auto* sc = new TreeSchedule();
    int nprob = (int)L.size();
    sc->nprob = nprob;
    sc->off = off;
    sc->L = L;
    sc->n = off[nprob];
    sc->pbox.resize(nprob);
    int64_t nb = 0, nl = 0;
    std::vector<int> g(nprob), S(nprob);
    std::vector<char> lds(nprob);
    int nstage = 0;
    for (int b = 0; b < nprob; ++b) {
        sc->pbox[b] = nb;
        nb += nbox_levels(L[b]);
        nl += int64_t(1) << (2 * (L[b] - 1));
        sc->max_levels = std::max(sc->max_levels, L[b]);
        int64_t n = off[b + 1] - off[b];
        S[b] = 2 * (L[b] - 1);
        int gb = 0;
        while (gb < S[b] && ((n + (int64_t(1) << gb) - 1) >> gb) > kLdsCap) ++gb;
        g[b] = gb;
        lds[b] = ((n + (int64_t(1) << gb) - 1) >> gb) <= kLdsCap;
        nstage = std::max(nstage, gb);
    }
    sc->nbox = nb;
    sc->nleaf = nl;
    sc->nstage = nstage;
    // key segments of stage s: problems with s <= g_b
    sc->nkeys.assign(nstage + 1, 0);
    sc->keys_off.assign(nstage + 2, 0);
    std::vector<std::vector<int64_t>> kbase(nstage + 1, std::vector<int64_t>(nprob, -1));
    for (int s = 0; s <= nstage; ++s) {
        int64_t c = 0;
        for (int b = 0; b < nprob; ++b)
            if (s <= g[b]) { kbase[s][b] = c; c += int64_t(1) << s; }
        sc->nkeys[s] = (int)c;
        sc->keys_off[s + 1] = sc->keys_off[s] + c;
    }
    sc->total_keys = sc->keys_off[nstage + 1];
    sc->segs.assign(sc->total_keys, SegInfo{});
    sc->tile_off.assign(nstage + 1, 0);
    sc->ntile.assign(nstage, 0);
    for (int s = 0; s <= nstage; ++s) {
        for (int b = 0; b < nprob; ++b) {
            if (s > g[b]) continue;
            int64_t n = off[b + 1] - off[b];
            for (int64_t j = 0; j < (int64_t(1) << s); ++j) {
                int64_t st, cnt;
                seg_range(off[b], n, s, j, &st, &cnt);
                int64_t gi = sc->keys_off[s] + kbase[s][b] + j;
                SegInfo& si = sc->segs[gi];
                si.start = (int32_t)st;
                si.count = (int32_t)cnt;
                si.box = (s % 2 == 0) ? (int32_t)(sc->pbox[b] + level_base(s / 2) + j) : -1;
                si.child = -1;
                si.tile0 = 0;
                si.ntile = 0;
                if (s < g[b]) {
                    si.child = (int32_t)(sc->keys_off[s + 1] + kbase[s + 1][b] + 2 * j);
                    si.tile0 = (int32_t)sc->tiles.size();
                    int32_t nt = (int32_t)((cnt + kTile - 1) / kTile);
                    si.ntile = nt;
                    for (int32_t t = 0; t < nt; ++t) {
                        TileInfo ti;
                        ti.seg = (int32_t)gi;
                        ti.start = (int32_t)(st + int64_t(t) * kTile);
                        ti.count = (int32_t)std::min<int64_t>(kTile, cnt - int64_t(t) * kTile);
                        ti.rank = t;
                        ti.seg_start = si.start;
                        ti.seg_count = si.count;
                        ti.tile0 = si.tile0;
                        ti.child = si.child;
                        ti.range = s == 0 ? (int32_t)gi : (int32_t)(sc->keys_off[s - 1] + kbase[s - 1][b] + (j >> 1));
                        ti.flags = (s + 1 < g[b]) ? 1 : 0;
                        sc->tiles.push_back(ti);
                    }
                }
            }
        }
        if (s < nstage) {
            sc->tile_off[s + 1] = (int64_t)sc->tiles.size();
            sc->ntile[s] = (int)(sc->tile_off[s + 1] - sc->tile_off[s]);
        }
    }
    sc->total_tile = (int64_t)sc->tiles.size();
    // init tiles: every problem's root (stage-0 key segment b' = kbase[0][b])
    sc->copy_tiles.clear();
    // geometry jobs from global-stage keys, lds work, copy tiles
    sc->geom_stage_off.assign(nstage + 2, 0);
    for (int s = 0; s <= nstage; ++s) {
        sc->geom_stage_off[s] = (int64_t)sc->geom.size();
        if (s % 2) continue;
        for (int b = 0; b < nprob; ++b) {
            bool from_keys = (s < g[b]) || (!lds[b] && s == g[b]);
            if (!from_keys) continue;
            for (int64_t j = 0; j < (int64_t(1) << s); ++j) {
                GeomJob gj;
                gj.box = (int32_t)(sc->pbox[b] + level_base(s / 2) + j);
                gj.seg = (int32_t)(sc->keys_off[s] + kbase[s][b] + j);
                sc->geom.push_back(gj);
            }
        }
    }
    sc->geom_stage_off[nstage + 1] = (int64_t)sc->geom.size();
    for (int b = 0; b < nprob; ++b) {
        int64_t n = off[b + 1] - off[b];
        if (lds[b]) {
            for (int64_t j = 0; j < (int64_t(1) << g[b]); ++j) {
                int64_t st, cnt;
                seg_range(off[b], n, g[b], j, &st, &cnt);
                LdsWork w;
                w.start = (int32_t)st; w.count = (int32_t)cnt;
                w.stages = S[b] - g[b]; w.stage0 = g[b]; w.j0 = (int32_t)j;
                w.boxbase = (int32_t)sc->pbox[b];
                w.pad0 = w.pad1 = 0;
                sc->lds.push_back(w);
            }
        } else {
            for (int64_t st = off[b]; st < off[b + 1]; st += kTile) {
                TileInfo ti;
                ti.seg = g[b] % 2;      // ping-pong buffer holding the final stage
                ti.start = (int32_t)st;
                ti.count = (int32_t)std::min<int64_t>(kTile, off[b + 1] - st);
                ti.rank = 0;
                ti.seg_start = ti.seg_count = ti.tile0 = ti.child = ti.range = ti.flags = 0;
                sc->copy_tiles.push_back(ti);
            }
        }
    }
    // per-box ranges, parents, levels, problems
    sc->box_start.assign(nb, 0); sc->box_count.assign(nb, 0);
    sc->box_parent.assign(nb, -1); sc->box_level.assign(nb, 0); sc->box_prob.assign(nb, 0);
    for (int b = 0; b < nprob; ++b) {
        int64_t n = off[b + 1] - off[b];
        for (int l = 0; l < L[b]; ++l) {
            for (int64_t j = 0; j < (int64_t(1) << (2 * l)); ++j) {
                int64_t st, cnt;
                seg_range(off[b], n, 2 * l, j, &st, &cnt);
                int64_t id = sc->pbox[b] + level_base(l) + j;
                sc->box_start[id] = (int32_t)st;
                sc->box_count[id] = (int32_t)cnt;
                sc->box_parent[id] = l ? (int32_t)(sc->pbox[b] + level_base(l - 1) + (j >> 2)) : -1;
                sc->box_level[id] = (int8_t)l;
                sc->box_prob[id] = b;
            }
        }
    }
    return sc;
}

template <class T>
static void upload(DBuf<T>& d, const std::vector<T>& h, hipStream_t s)
{
    d.alloc(std::max<size_t>(h.size(), 1), s);
    if (!h.empty())
        FMM_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

void upload_schedule(TreeSchedule& sc, hipStream_t s)
{
    upload(sc.d_segs, sc.segs, s);
    upload(sc.d_tiles, sc.tiles, s);
    upload(sc.d_copy, sc.copy_tiles, s);
    upload(sc.d_lds, sc.lds, s);
    upload(sc.d_geom, sc.geom, s);
    upload(sc.d_box_start, sc.box_start, s);
    upload(sc.d_box_count, sc.box_count, s);
    upload(sc.d_box_parent, sc.box_parent, s);
    upload(sc.d_box_level, sc.box_level, s);
    upload(sc.d_box_prob, sc.box_prob, s);
    upload(sc.d_off, sc.off, s);
    upload(sc.d_pbox, sc.pbox, s);
    // the host vectors must stay alive until the copies ran
    FMM_HIP(hipStreamSynchronize(s));
}

// ------------------------------------------------------------ device helpers

// order-preserving unsigned image of a double (+0 and -0 map to the same key)
__device__ __forceinline__ uint64_t okey(double x)
{
    x = x + 0.0;
    uint64_t u = (uint64_t)__double_as_longlong(x);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double okey_inv(uint64_t k)
{
    uint64_t u = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)u);
}

// geometry of a box from its bounding box, every operation rounded alone
__device__ __forceinline__ void box_geometry(double x0, double x1, double y0, double y1,
                                             double* bb, double* gm)
{
    bb[0] = x0; bb[1] = x1; bb[2] = y0; bb[3] = y1;
    gm[0] = (0.5 * (x0 + x1));
    gm[1] = (0.5 * (y0 + y1));
    double dx = (x1 - x0), dy = (y1 - y0);
    gm[2] = 0.5 * __dsqrt_rn((dx * dx) + (dy * dy));
}

// Every segment's bounding box is kept as kKeyCopies copies of four order
// keys (xmin, xmax, ymin, ymax) so that the workgroups updating it with
// atomics spread over several addresses; readers combine the copies.
constexpr int kKeyCopies = 32;
constexpr int kKeyWords = 4 * kKeyCopies;

__device__ __forceinline__ void read_keys(const uint64_t* k, double* bb)
{
    uint64_t a = k[0], b = k[1], c = k[2], d = k[3];
#pragma unroll
    for (int i = 1; i < kKeyCopies; ++i) {
        a = min(a, k[4 * i]); b = max(b, k[4 * i + 1]); c = min(c, k[4 * i + 2]); d = max(d, k[4 * i + 3]);
    }
    bb[0] = okey_inv(a); bb[1] = okey_inv(b); bb[2] = okey_inv(c); bb[3] = okey_inv(d);
}

// read_keys for a whole workgroup: lane c of wave 0 reads copy c and the
// wave combines them; every thread receives the result (one barrier)
static_assert(kKeyCopies == 32, "one key copy per lane of a half wavefront");
__device__ __forceinline__ void block_read_keys(const uint64_t* k, double* bb)
{
    // the copies as doubles (an untouched copy decodes to NaN, which the
    // minimum and maximum ignore, as the integer order placed it last)
    __shared__ double sk[4];
    if (threadIdx.x < 64) {
        const int c = threadIdx.x & (kKeyCopies - 1);
        const double a = half_wave_min(okey_inv(k[4 * c])), b = half_wave_max(okey_inv(k[4 * c + 1]));
        const double d = half_wave_min(okey_inv(k[4 * c + 2])), e = half_wave_max(okey_inv(k[4 * c + 3]));
        if (threadIdx.x == 0) { sk[0] = a; sk[1] = b; sk[2] = d; sk[3] = e; }
    }
    __syncthreads();
    bb[0] = sk[0]; bb[1] = sk[1]; bb[2] = sk[2]; bb[3] = sk[3];
}

// Two levels of bucket selection: the first histogram of a segment has
// kBuckets1 buckets over its extent, the second kBuckets2 buckets inside the
// first-level bucket that holds the median (when that bucket is large).
constexpr int kBuckets1 = 256;
constexpr int kBuckets2 = kBuckets;
// Every first-level histogram is kept as kHistCopies copies, updated by
// workgroups of different block index, so that the atomics of the many
// tiles of a large segment spread over several addresses; readers add them.
// Layout: ((segment * 2 + axis) * kHistCopies + copy) * kBuckets1 + bucket.
constexpr int kHistCopies = 8;
static_assert(kBuckets1 == kTileThreads, "one first-level bucket per thread");

template <class W>
__device__ __forceinline__ W* hist1_at(W* h, int64_t seg, int axis, int copy)
{
    return h + ((seg * 2 + axis) * kHistCopies + copy) * kBuckets1;
}

struct Bucketer {
    double lo, scale;
    int axis;
};

// first-level buckets of one axis over the bounding box bb (x0 x1 y0 y1)
__device__ __forceinline__ Bucketer axis_bucketer(const double* bb, int axis)
{
    Bucketer b;
    b.axis = axis;
    b.lo = axis ? bb[2] : bb[0];
    const double ext = axis ? (bb[3] - bb[2]) : (bb[1] - bb[0]);
    const double sc = ext > 0.0 ? (double)kBuckets1 / ext : 0.0;
    b.scale = (sc < 1e300) ? sc : 0.0;
    return b;
}

// read_keys of two segments for a whole workgroup (one barrier)
__device__ __forceinline__ void block_read_keys2(const uint64_t* k0, const uint64_t* k1, double* b0, double* b1)
{
    __shared__ double sk[8];
    if (threadIdx.x < 64) {
        const uint64_t* k = threadIdx.x < 32 ? k0 : k1;   // one segment per half wavefront
        const int c = threadIdx.x & (kKeyCopies - 1);
        const double a = half_wave_min(okey_inv(k[4 * c])), b = half_wave_max(okey_inv(k[4 * c + 1]));
        const double d = half_wave_min(okey_inv(k[4 * c + 2])), e = half_wave_max(okey_inv(k[4 * c + 3]));
        if ((threadIdx.x & 31) == 0) {
            const int o = threadIdx.x >> 3;   // 0 or 4
            sk[o] = a; sk[o + 1] = b; sk[o + 2] = d; sk[o + 3] = e;
        }
    }
    __syncthreads();
    for (int i = 0; i < 4; ++i) { b0[i] = sk[i]; b1[i] = sk[4 + i]; }
}

// The bucketer of a segment, computed by the whole workgroup (every thread
// of the block calls it, once per kernel): the split axis from the
// segment's own bounding box (the longer side), the bucket range from the
// bounding box of segment `range` along that axis (the parent, whose
// partition histograms the segment before its own box is complete).
__device__ __forceinline__ Bucketer make_bucketer(const uint64_t* keys, const uint64_t* range_keys,
                                                  double* own_bb = nullptr)
{
    double bb[4], rb[4];
    block_read_keys2(keys, range_keys, bb, rb);
    if (own_bb)
        for (int i = 0; i < 4; ++i) own_bb[i] = bb[i];
    const double w = (bb[1] - bb[0]), h = (bb[3] - bb[2]);
    return axis_bucketer(rb, (w >= h) ? 0 : 1);
}

__device__ __forceinline__ int bucket_of(const Bucketer& b, double c)
{
    double v = ((c - b.lo) * b.scale);
    int k = (int)fmin(fmax(v, 0.0), (double)(kBuckets1 - 1));
    return k;
}

__device__ __forceinline__ bool key_less(double c, int32_t i, double sc, int32_t si)
{
    return (c < sc) || (c == sc && i < si);
}

// block-wide exclusive scan of one value per thread (256 threads); returns
// the exclusive prefix, *total receives the block sum
template <int NT>
__device__ __forceinline__ int block_excl_scan(int v, int* sh, int* total)
{
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int x = wave_incl_scan(v);
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        int s = sh[w];
        if (w < wid) base += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

// ------------------------------------------------------------------ kernels

// start of a build: the counter words zeroed; the bounding-box keys (every
// copy: kxmin kxmax kymin kymax) set to the empty box; the tree's error word
// cleared
__global__ void k_fill_start(uint32_t* words, int64_t nwords, uint64_t* k, int64_t nkeywords, uint32_t* err)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *err = 0u;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nwords; i += stride) words[i] = 0u;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nkeywords; i += stride)
        k[i] = (i & 1) ? 0ull : ~0ull;
}

__device__ __forceinline__ void block_minmax_atomic(double x0, double x1, double y0, double y1,
                                                    uint64_t* keys, bool any)
{
    __shared__ double red[4][kTileThreads / 64];
    // over the wavefront as doubles (a thread without a point contributes
    // +-infinity), turned into order keys once per workgroup
    double a = wave_min(any ? x0 : INFINITY), b = wave_max(any ? x1 : -INFINITY);
    double c = wave_min(any ? y0 : INFINITY), d = wave_max(any ? y1 : -INFINITY);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { red[0][w] = a; red[1][w] = b; red[2][w] = c; red[3][w] = d; }
    __syncthreads();
    if (threadIdx.x == 0) {
        keys += 4 * (blockIdx.x & (kKeyCopies - 1));
        for (int i = 1; i < kTileThreads / 64; ++i) {
            a = fmin(a, red[0][i]); b = fmax(b, red[1][i]);
            c = fmin(c, red[2][i]); d = fmax(d, red[3][i]);
        }
        if (isfinite(a)) {
            atomicMin((unsigned long long*)&keys[0], (unsigned long long)okey(a));
            atomicMax((unsigned long long*)&keys[1], (unsigned long long)okey(b));
            atomicMin((unsigned long long*)&keys[2], (unsigned long long)okey(c));
            atomicMax((unsigned long long*)&keys[3], (unsigned long long)okey(d));
        }
    }
    __syncthreads();
}

// positions into SoA buffers, input order; root bounding boxes; finiteness
__global__ void __launch_bounds__(kTileThreads)
k_init(const double* __restrict__ z, const int64_t* __restrict__ poff, int nprob,
       double* X, double* Y, int32_t* I, uint64_t* keys0, uint32_t* err)
{
    constexpr int R = kTile / kTileThreads;
    int b = blockIdx.y;
    int64_t s0 = poff[b], s1 = poff[b + 1];
    int64_t t0 = s0 + (int64_t)blockIdx.x * kTile;
    if (t0 >= s1) return;   // uniform per block
    const int cnt = (int)min(s1 - t0, (int64_t)kTile);
    // every load of the tile issued before the first use
    double2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = r * kTileThreads + threadIdx.x;
        v[r] = reinterpret_cast<const double2*>(z)[t0 + (i < cnt ? i : 0)];
    }
    double x0 = 1e308, x1 = -1e308, y0 = 1e308, y1 = -1e308;
    bool any = false, bad = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = r * kTileThreads + threadIdx.x;
        if (i < cnt) {
            // a non-finite position is flagged and built as (0, 0): the tree
            // stays a valid permutation, whatever runs before the flag is read
            if (!(isfinite(v[r].x) && isfinite(v[r].y))) {
                bad = true;
                v[r] = make_double2(0.0, 0.0);
            }
            X[t0 + i] = v[r].x; Y[t0 + i] = v[r].y; I[t0 + i] = (int32_t)(t0 + i);
            x0 = fmin(x0, v[r].x); x1 = fmax(x1, v[r].x); y0 = fmin(y0, v[r].y); y1 = fmax(y1, v[r].y);
            any = true;
        }
    }
    if (bad) atomicOr(err, 1u);
    // any is false only for threads without points; min/max skip them
    block_minmax_atomic(x0, x1, y0, y1, keys0 + kKeyWords * b, any);
}

// the split coordinate of the tile's points (element r * kTileThreads + tid)
// into registers, every load issued before the first use
template <int R>
__device__ __forceinline__ void load_tile(const double* __restrict__ C, const TileInfo& t, double (&v)[R])
{
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = r * kTileThreads + threadIdx.x;
        v[r] = C[t.start + (i < t.count ? i : 0)];
    }
}

__global__ void __launch_bounds__(kTileThreads)
k_hist1(const TileInfo* __restrict__ tiles, const double* __restrict__ X,
        const double* __restrict__ Y, const uint64_t* __restrict__ keys, uint32_t* hist1)
{
    constexpr int R = kTile / kTileThreads;
    __shared__ uint32_t h[kBuckets1];
    TileInfo t = tiles[blockIdx.x];
    Bucketer bk = make_bucketer(keys + kKeyWords * (int64_t)t.seg, keys + kKeyWords * (int64_t)t.range);
    double v[R];
    load_tile(bk.axis ? Y : X, t, v);
    for (int i = threadIdx.x; i < kBuckets1; i += kTileThreads) h[i] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (r * kTileThreads + (int)threadIdx.x < t.count) atomicAdd(&h[bucket_of(bk, v[r])], 1u);
    __syncthreads();
    uint32_t* g = hist1_at(hist1, t.seg, bk.axis, blockIdx.x & (kHistCopies - 1));
    for (int i = threadIdx.x; i < kBuckets1; i += kTileThreads)
        if (h[i]) atomicAdd(&g[i], h[i]);
}

// find the bucket holding rank k among NB buckets: returns bucket, writes the
// rank inside it and the bucket's count.  hist in global memory, 256 threads.
// (find_bucket_loc: thread i holds the counts loc of buckets PER i .. PER i + PER - 1)
template <int PER>
__device__ int find_bucket_loc(const int (&loc)[PER], int k, int* rank_in, int* cnt_in, int* sh)
{
    int s = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) s += loc[i];
    int tot;
    int base = block_excl_scan<kTileThreads>(s, sh, &tot);
    // the thread whose range holds rank k writes the answer
    __shared__ int ans[3];
    int c = base;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        if (loc[i] > 0 && c <= k && k < c + loc[i]) {
            ans[0] = threadIdx.x * PER + i; ans[1] = k - c; ans[2] = loc[i];
        }
        c += loc[i];
    }
    __syncthreads();
    int b = ans[0];
    *rank_in = ans[1];
    *cnt_in = ans[2];
    __syncthreads();
    return b;
}
template <int NB>
__device__ int find_bucket(const uint32_t* hist, int k, int* rank_in, int* cnt_in, int* sh)
{
    static_assert(NB % kTileThreads == 0, "whole buckets per thread");
    constexpr int PER = NB / kTileThreads;
    int loc[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) loc[i] = (int)hist[threadIdx.x * PER + i];
    return find_bucket_loc<PER>(loc, k, rank_in, cnt_in, sh);
}

// a median bucket with more points than this is refined by a second histogram
// (a second pass over the segment's coordinates costs less than ranking a
// longer candidate list in every partition tile)
constexpr int kSubThreshold = 16;

struct SubBucketer {
    double lo, scale;
};
__device__ __forceinline__ SubBucketer make_sub(const Bucketer& bk, int b1)
{
    SubBucketer s;
    s.lo = bk.lo + (double)b1 / bk.scale;
    s.scale = (bk.scale * (double)kBuckets2);
    return s;
}
__device__ __forceinline__ int sub_of(const SubBucketer& s, double c)
{
    double v = ((c - s.lo) * s.scale);
    return (int)fmin(fmax(v, 0.0), (double)(kBuckets2 - 1));
}

// the first-level bucket of a segment's median (its rank inside the bucket
// and the bucket's population) and the segment's bucketer, found by hist2
// and read by collect (which then needs no bounding box of its own)
struct Level1 {
    int32_t b1, r1, c1, axis;
    double lo, scale;
    double bb[4];     // the segment's bounding box, for its partition
};

__global__ void __launch_bounds__(kTileThreads)
k_hist2(const TileInfo* __restrict__ tiles, const SegInfo* __restrict__ segs,
        const double* __restrict__ X, const double* __restrict__ Y,
        const uint64_t* __restrict__ keys, const uint32_t* __restrict__ hist1, uint32_t* hist2, Level1* lvl1)
{
    __shared__ uint32_t h[kBuckets2];
    __shared__ int sh[kTileThreads / 64];
    TileInfo t = tiles[blockIdx.x];
    // this thread's first-level bucket on both axes (the copies added),
    // loaded while the bounding boxes are read
    int hx = 0, hy = 0;
#pragma unroll
    for (int c = 0; c < kHistCopies; ++c) {
        hx += (int)hist1_at(hist1, t.seg, 0, c)[threadIdx.x];
        hy += (int)hist1_at(hist1, t.seg, 1, c)[threadIdx.x];
    }
    double bb[4];
    Bucketer bk = make_bucketer(keys + kKeyWords * (int64_t)t.seg, keys + kKeyWords * (int64_t)t.range, bb);
    int r1, c1;
    const int loc[1] = {bk.axis ? hy : hx};
    int b1 = find_bucket_loc<1>(loc, t.seg_count / 2, &r1, &c1, sh);
    if (t.rank == 0 && threadIdx.x == 0) {
        Level1 v;
        v.b1 = b1; v.r1 = r1; v.c1 = c1; v.axis = bk.axis;
        v.lo = bk.lo; v.scale = bk.scale;
        for (int i = 0; i < 4; ++i) v.bb[i] = bb[i];
        lvl1[t.seg] = v;
    }
    if (c1 <= kSubThreshold) return;   // uniform per block
    if (bk.scale == 0.0) return;  // all points in one bucket: the exact fallback handles it
    SubBucketer sb = make_sub(bk, b1);
    constexpr int R = kTile / kTileThreads;
    double v[R];
    load_tile(bk.axis ? Y : X, t, v);
    for (int i = threadIdx.x; i < kBuckets2; i += kTileThreads) h[i] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (r * kTileThreads + (int)threadIdx.x < t.count && bucket_of(bk, v[r]) == b1)
            atomicAdd(&h[sub_of(sb, v[r])], 1u);
    __syncthreads();
    uint32_t* g = hist2 + (int64_t)t.seg * kBuckets2;
    for (int i = threadIdx.x; i < kBuckets2; i += kTileThreads)
        if (h[i]) atomicAdd(&g[i], h[i]);
}

struct Cand {
    double c;
    int32_t idx;
    int32_t tile;
};
struct Splitter {
    double c;
    int32_t idx;
    int32_t pad;
};
// the median's class of a segment as collect found it, for the partition
struct ClassInfo {
    int32_t rank;     // rank of the median within the class
    int32_t count;    // points in the class (the candidates, when <= kCandCap)
    int32_t axis;     // split axis: 0 x, 1 y
    int32_t pad;
};

// candidate class of a point: -1 below, 0 inside, 1 above
struct ClassRule {
    Bucketer bk;
    SubBucketer sb;
    int b1, b2;     // b2 < 0: one level
};
__device__ __forceinline__ int class_of(const ClassRule& r, double c)
{
    int b = bucket_of(r.bk, c);
    if (b != r.b1) return b < r.b1 ? -1 : 1;
    if (r.b2 < 0) return 0;
    int s = sub_of(r.sb, c);
    return s == r.b2 ? 0 : (s < r.b2 ? -1 : 1);
}

// exact selection of the k-th smallest (coordinate, index) of a segment by a
// most-significant-digit radix select over the 96-bit key, by one workgroup.
__device__ void exact_select(const double* C, const int32_t* I, int start, int count, int k,
                             Splitter* out)
{
    __shared__ uint32_t h[256];
    __shared__ int sh[kTileThreads / 64];
    __shared__ uint64_t pre_hi;
    __shared__ uint32_t pre_lo;
    __shared__ int rk;
    if (threadIdx.x == 0) { pre_hi = 0; pre_lo = 0; rk = k; }
    __syncthreads();
    for (int d = 0; d < 12; ++d) {
        for (int i = threadIdx.x; i < 256; i += kTileThreads) h[i] = 0;
        __syncthreads();
        uint64_t ph = pre_hi;
        uint32_t pl = pre_lo;
        for (int i = threadIdx.x; i < count; i += kTileThreads) {
            uint64_t kh = okey(C[start + i]);
            uint32_t kl = (uint32_t)I[start + i];
            bool match;
            int digit;
            if (d < 8) {
                int sh_ = 8 * (8 - d);   // bits above the current digit
                match = (sh_ >= 64) ? true : ((kh >> sh_) == (ph >> sh_));
                digit = (int)((kh >> (8 * (7 - d))) & 0xff);
            } else {
                int dd = d - 8;
                int sh_ = 8 * (4 - dd);
                match = (kh == ph) && ((sh_ >= 32) ? true : ((kl >> sh_) == (pl >> sh_)));
                digit = (int)((kl >> (8 * (3 - dd))) & 0xff);
            }
            if (match) atomicAdd(&h[digit], 1u);
        }
        __syncthreads();
        int v = (int)h[threadIdx.x];
        int tot;
        int base = block_excl_scan<kTileThreads>(v, sh, &tot);
        int r = rk;
        __syncthreads();
        if (v > 0 && base <= r && r < base + v) {
            if (d < 8) pre_hi |= (uint64_t)threadIdx.x << (8 * (7 - d));
            else pre_lo |= (uint32_t)threadIdx.x << (8 * (3 - (d - 8)));
            rk = r - base;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out->c = okey_inv(pre_hi); out->idx = (int32_t)pre_lo; out->pad = 0; }
    __syncthreads();
}

// the candidate class (one or two histogram levels) of a segment's median,
// from the first-level bucket and the bucketer that hist2 recorded
__device__ __forceinline__ ClassRule median_class(const Level1* lvl1, const uint32_t* hist2, int seg, int* rank,
                                                  int* ccount, int* sh)
{
    ClassRule rule;
    const Level1 L1 = lvl1[seg];
    rule.bk.axis = L1.axis;
    rule.bk.lo = L1.lo;
    rule.bk.scale = L1.scale;
    const int r1 = L1.r1, c1 = L1.c1;
    rule.b1 = L1.b1;
    rule.b2 = -1;
    *rank = r1;
    *ccount = c1;
    if (c1 > kSubThreshold && rule.bk.scale != 0.0) {
        rule.sb = make_sub(rule.bk, rule.b1);
        int r2, c2;
        rule.b2 = find_bucket<kBuckets2>(hist2 + (int64_t)seg * kBuckets2, r1, &r2, &c2, sh);
        *rank = r2;
        *ccount = c2;
    }
    return rule;
}

// Segments whose median class holds more than kCandCap points (heavy ties):
// one workgroup finds the exact median (coordinate, index) of the segment
// by a radix select, and the output offset of every tile's lower half.
__device__ void pick_exact(int seg, const SegInfo& sg, const TileInfo* __restrict__ all_tiles,
                           const double* __restrict__ C, const int32_t* __restrict__ I, uint32_t* tile_below,
                           uint32_t* lo_base, Splitter* split, int* sh)
{
    __shared__ Splitter sp;
    const int k = sg.count / 2;
    exact_select(C, I, sg.start, sg.count, k, &sp);
    for (int tt = 0; tt < sg.ntile; ++tt) {
        TileInfo ti = all_tiles[sg.tile0 + tt];
        int cnt = 0;
        for (int i = threadIdx.x; i < ti.count; i += kTileThreads)
            cnt += key_less(C[ti.start + i], I[ti.start + i], sp.c, sp.idx);
        int tot2;
        block_excl_scan<kTileThreads>(cnt, sh, &tot2);
        if (threadIdx.x == 0) tile_below[sg.tile0 + tt] = (uint32_t)tot2;
    }
    __syncthreads();
    // exclusive scan of the per-tile lower counts into output offsets
    int run = 0;
    for (int c0 = 0; c0 < sg.ntile; c0 += kTileThreads) {
        int i = c0 + threadIdx.x;
        int v = (i < sg.ntile) ? (int)tile_below[sg.tile0 + i] : 0;
        int tot3;
        int ex = block_excl_scan<kTileThreads>(v, sh, &tot3);
        if (i < sg.ntile) lo_base[sg.tile0 + i] = (uint32_t)(run + ex);
        run += tot3;
    }
    if (threadIdx.x == 0) split[seg] = sp;
}

// every tile: count of points below the median's class, and the points of
// that class appended to the segment's candidate list.  When the class
// overflowed, the last tile of the segment to finish (per-segment counter
// seg_done) runs the exact selection for the whole segment; the partition
// tiles of other segments find the median themselves.
__global__ void __launch_bounds__(kTileThreads)
k_collect(const TileInfo* __restrict__ tiles, const TileInfo* __restrict__ all_tiles, const SegInfo* __restrict__ segs,
          const double* __restrict__ X, const double* __restrict__ Y, const int32_t* __restrict__ I,
          const Level1* __restrict__ lvl1, const uint32_t* __restrict__ hist2, Cand* cand, uint32_t* cand_cnt,
          uint32_t* tile_below, uint32_t* seg_done, ClassInfo* cinfo, uint32_t* lo_base, Splitter* split)
{
    __shared__ int sh[kTileThreads / 64];
    TileInfo t = tiles[blockIdx.x];
    constexpr int R = kTile / kTileThreads;
    int rank, ccount;
    ClassRule rule = median_class(lvl1, hist2, t.seg, &rank, &ccount, sh);
    const bool overflow = ccount > kCandCap;
    if (t.rank == 0 && threadIdx.x == 0) {
        ClassInfo ci;
        ci.rank = rank; ci.count = ccount; ci.axis = rule.bk.axis; ci.pad = 0;
        cinfo[t.seg] = ci;
    }
    double v[R];
    load_tile(rule.bk.axis ? Y : X, t, v);
    int below = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = r * kTileThreads + threadIdx.x;
        if (i >= t.count) continue;
        int cl = class_of(rule, v[r]);
        below += (cl < 0);
        if (cl == 0 && !overflow) {
            uint32_t pos = atomicAdd(&cand_cnt[t.seg], 1u);
            if (pos < (uint32_t)kCandCap) {
                Cand cd; cd.c = v[r]; cd.idx = I[t.start + i]; cd.tile = t.rank;
                cand[(int64_t)t.seg * kCandCap + pos] = cd;
            }
        }
    }
    int tot;
    block_excl_scan<kTileThreads>(below, sh, &tot);
    if (threadIdx.x == 0) tile_below[t.tile0 + t.rank] = (uint32_t)tot;
    if (overflow) {   // uniform per block
        __shared__ bool last;
        __threadfence();   // this tile's count is visible before the tile is counted done
        __syncthreads();
        if (threadIdx.x == 0) last = atomicAdd(&seg_done[t.seg], 1u) + 1u == (uint32_t)segs[t.seg].ntile;
        __syncthreads();
        if (last) {   // every tile of the segment has written its count: overwrite them all
            __threadfence();
            pick_exact(t.seg, segs[t.seg], all_tiles, rule.bk.axis ? Y : X, I, tile_below, lo_base, split, sh);
        }
    }
}

// bounding boxes of both halves of a tile into the next stage's keys (one
// barrier for the two)
__device__ __forceinline__ void block_minmax2_atomic(const double (&l)[4], const double (&u)[4], bool anyl,
                                                     bool anyu, uint64_t* keys_lo, uint64_t* keys_hi)
{
    __shared__ double red[8][kTileThreads / 64];
    // minima and maxima over the wavefront as doubles (a lane without a
    // point contributes +-infinity), turned into order keys once per
    // workgroup
    double k[8];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double inf = (q & 1) ? -INFINITY : INFINITY;
        k[q] = anyl ? l[q] : inf;
        k[4 + q] = anyu ? u[q] : inf;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) k[q] = (q & 1) ? wave_max(k[q]) : wave_min(k[q]);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < 8; ++q) red[q][w] = k[q];
    __syncthreads();
    // thread q < 8 combines value q over the waves and updates one key
    if (threadIdx.x < 8) {
        const int q = threadIdx.x;
        double v = red[q][0];
        for (int i = 1; i < kTileThreads / 64; ++i) v = (q & 1) ? fmax(v, red[q][i]) : fmin(v, red[q][i]);
        uint64_t* kk = (q < 4 ? keys_lo : keys_hi) + 4 * (blockIdx.x & (kKeyCopies - 1)) + (q & 3);
        const bool empty = !isfinite(v);
        const uint64_t a = empty ? 0ull : okey(v);
        if (!empty) {
            if (q & 1) atomicMax((unsigned long long*)kk, (unsigned long long)a);
            else atomicMin((unsigned long long*)kk, (unsigned long long)a);
        }
    }
}

// The median (coordinate, index) of a segment from its candidate list (the
// points of the median's class), and the lower points of the tiles before
// tile `rank_t`: below-class counts of those tiles plus their candidates
// ranked below the median.  Every tile of the segment computes the same
// median.  Up to one candidate per thread, a candidate's rank is its count
// of smaller candidates; longer lists are sorted (bitonic, in LDS).
__device__ void tile_median(const Cand* __restrict__ cs, int n, int rank, const uint32_t* __restrict__ below,
                            int rank_t, Splitter* sp, int* lob, int* sh)
{
    __shared__ uint64_t skey[kCandCap];
    __shared__ uint32_t sidx[kCandCap];
    __shared__ uint32_t stile[kCandCap];
    __shared__ Splitter ssp;
    int P = n;
    if (n > kTileThreads) {
        P = 1;
        while (P < n) P <<= 1;
    }
    for (int i = threadIdx.x; i < P; i += kTileThreads) {
        if (i < n) {
            const Cand cd = cs[i];
            skey[i] = okey(cd.c);
            sidx[i] = (uint32_t)cd.idx;
            stile[i] = (uint32_t)cd.tile;
        } else {
            skey[i] = ~0ull; sidx[i] = 0xffffffffu; stile[i] = 0xffffffffu;
        }
    }
    int v = 0;
    for (int i = threadIdx.x; i < rank_t; i += kTileThreads) v += (int)below[i];
    __syncthreads();
    if (n <= kTileThreads) {
        const int i = threadIdx.x;
        if (i < n) {
            const uint64_t ki = skey[i];
            const uint32_t ii = sidx[i];
            int ri = 0;
            for (int j = 0; j < n; ++j) ri += (skey[j] < ki) | ((skey[j] == ki) & (sidx[j] < ii));
            if (ri == rank) { ssp.c = okey_inv(ki); ssp.idx = (int32_t)ii; ssp.pad = 0; }
            v += (ri < rank) & ((int)stile[i] < rank_t);
        }
    } else {
        for (int kk = 2; kk <= P; kk <<= 1)
            for (int j = kk >> 1; j > 0; j >>= 1) {
                for (int i = threadIdx.x; i < P / 2; i += kTileThreads) {
                    const int lo = ((i & ~(j - 1)) << 1) | (i & (j - 1));
                    const int hi = lo + j;
                    const bool asc = (lo & kk) == 0;
                    const bool less_hl = (skey[hi] < skey[lo]) || (skey[hi] == skey[lo] && sidx[hi] < sidx[lo]);
                    if (less_hl == asc) {
                        const uint64_t a = skey[lo]; skey[lo] = skey[hi]; skey[hi] = a;
                        const uint32_t b = sidx[lo]; sidx[lo] = sidx[hi]; sidx[hi] = b;
                        const uint32_t c = stile[lo]; stile[lo] = stile[hi]; stile[hi] = c;
                    }
                }
                __syncthreads();
            }
        if (threadIdx.x == 0) { ssp.c = okey_inv(skey[rank]); ssp.idx = (int32_t)sidx[rank]; ssp.pad = 0; }
        for (int i = threadIdx.x; i < rank; i += kTileThreads) v += ((int)stile[i] < rank_t);
    }
    int tot;
    block_excl_scan<kTileThreads>(v, sh, &tot);   // its barriers also publish ssp
    *lob = tot;
    *sp = ssp;
}

// Stable two-way partition of one tile.  Element i = r * kTileThreads + tid
// is lower if (coordinate, index) < splitter; its rank among the lower
// (upper) elements of the tile comes from per-wave ballots of every row,
// combined with one barrier.  The splitter and the tile's output offset come
// from tile_median, or from the exact selection (pick_exact, run by the last
// collect tile) for a segment whose class overflowed.
__global__ void __launch_bounds__(kTileThreads)
k_partition(const TileInfo* __restrict__ tiles, const SegInfo* __restrict__ segs,
            const double* __restrict__ X, const double* __restrict__ Y, const int32_t* __restrict__ I,
            double* X2, double* Y2, int32_t* I2, uint64_t* keys_next, const ClassInfo* __restrict__ cinfo,
            const Cand* __restrict__ cand, const uint32_t* __restrict__ tile_below,
            const Splitter* __restrict__ split, const uint32_t* __restrict__ lo_base, uint32_t* hist1,
            const Level1* __restrict__ lvl1)
{
    constexpr int R = kTile / kTileThreads;
    constexpr int NW = kTileThreads / 64;
    __shared__ int wcnt[R][NW];
    __shared__ int sh[NW];
    __shared__ uint32_t chist[4 * kBuckets1];   // the children's first-level histograms, (child, axis)
    const TileInfo t = tiles[blockIdx.x];
    const bool hist_children = (t.flags & 1) != 0;   // uniform per block
    const int k = t.seg_count / 2;
    const int toff = t.start - t.seg_start;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    // the tile's points first: their loads overlap the median search
    double x[R], y[R];
    int32_t id[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = r * kTileThreads + threadIdx.x;
        const int ii = t.start + (i < t.count ? i : 0);
        x[r] = X[ii]; y[r] = Y[ii]; id[r] = I[ii];
    }
    // a child split by a later global stage is histogrammed here, on both
    // axes over this segment's bounding box (its split axis is not known yet)
    Bucketer cb[2];
    if (hist_children) {
        double bb[4];   // this segment's bounding box, as hist2 read it
        for (int i = 0; i < 4; ++i) bb[i] = lvl1[t.seg].bb[i];
        cb[0] = axis_bucketer(bb, 0);
        cb[1] = axis_bucketer(bb, 1);
        for (int i = threadIdx.x; i < 4 * kBuckets1; i += kTileThreads) chist[i] = 0u;
    }
    const ClassInfo ci = cinfo[t.seg];
    Splitter sp;
    int lob;
    if (ci.count > kCandCap) {
        sp = split[t.seg];
        lob = (int)lo_base[t.tile0 + t.rank];
    } else {
        tile_median(cand + (int64_t)t.seg * kCandCap, ci.count, ci.rank, tile_below + t.tile0, t.rank, &sp, &lob, sh);
    }
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int inwave[R];
    bool lower[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = r * kTileThreads + threadIdx.x;
        lower[r] = i < t.count && key_less(ci.axis ? y[r] : x[r], id[r], sp.c, sp.idx);
        const unsigned long long m = __ballot(lower[r]);
        inwave[r] = __popcll(m & lt);
        if (lane == 0) wcnt[r][wid] = __popcll(m);
    }
    __syncthreads();
    double l[4] = {1e308, -1e308, 1e308, -1e308}, u[4] = {1e308, -1e308, 1e308, -1e308};
    bool anyl = false, anyu = false;
    int before = 0;   // lower elements of the tile in earlier rows
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int rowtot = 0, prev = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int c = wcnt[r][w];
            prev += (w < wid) ? c : 0;
            rowtot += c;
        }
        const int i = r * kTileThreads + threadIdx.x;
        if (i < t.count) {
            const int lb = before + prev + inwave[r];   // lower elements before i in the tile
            int dst;
            if (lower[r]) {
                dst = t.seg_start + lob + lb;
                l[0] = fmin(l[0], x[r]); l[1] = fmax(l[1], x[r]); l[2] = fmin(l[2], y[r]); l[3] = fmax(l[3], y[r]);
                anyl = true;
            } else {
                dst = t.seg_start + k + (toff - lob) + (i - lb);
                u[0] = fmin(u[0], x[r]); u[1] = fmax(u[1], x[r]); u[2] = fmin(u[2], y[r]); u[3] = fmax(u[3], y[r]);
                anyu = true;
            }
            if (dst >= t.seg_start && dst < t.seg_start + t.seg_count) { X2[dst] = x[r]; Y2[dst] = y[r]; I2[dst] = id[r]; }
            if (hist_children) {
                const int c = lower[r] ? 0 : 2;   // (child, axis) slot of axis 0
                atomicAdd(&chist[c * kBuckets1 + bucket_of(cb[0], x[r])], 1u);
                atomicAdd(&chist[(c + 1) * kBuckets1 + bucket_of(cb[1], y[r])], 1u);
            }
        }
        before += rowtot;
    }
    // its barrier also completes the histogram updates above
    block_minmax2_atomic(l, u, anyl, anyu, keys_next + kKeyWords * (int64_t)t.child,
                         keys_next + kKeyWords * ((int64_t)t.child + 1));
    if (hist_children) {   // slot c * 2 + axis: child t.child + c, one bucket per thread
        const int copy = blockIdx.x & (kHistCopies - 1);
#pragma unroll
        for (int sl = 0; sl < 4; ++sl) {
            const uint32_t v = chist[sl * kBuckets1 + threadIdx.x];
            if (v) atomicAdd(&hist1_at(hist1, (int64_t)t.child + (sl >> 1), sl & 1, copy)[threadIdx.x], v);
        }
    }
}

// geometry of boxes whose bounding box came from a global stage
__global__ void k_geom_keys(const GeomJob* __restrict__ jobs, int64_t n, const uint64_t* __restrict__ keys,
                            double* bbox, double* geom)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    GeomJob j = jobs[i];
    double kb[4], bb[4], gm[3];
    read_keys(keys + kKeyWords * (int64_t)j.seg, kb);
    box_geometry(kb[0], kb[1], kb[2], kb[3], bb, gm);
    for (int q = 0; q < 4; ++q) bbox[4 * (int64_t)j.box + q] = bb[q];
    for (int q = 0; q < 3; ++q) geom[4 * (int64_t)j.box + q] = gm[q];
}

__global__ void k_copy_final(const TileInfo* __restrict__ tiles, const double* XA, const double* YA,
                             const int32_t* IA, const double* XB, const double* YB, const int32_t* IB,
                             double* X, double* Y, int32_t* I)
{
    TileInfo t = tiles[blockIdx.x];
    const double* xs = t.seg ? XB : XA;
    const double* ys = t.seg ? YB : YA;
    const int32_t* is = t.seg ? IB : IA;
    for (int i = threadIdx.x; i < t.count; i += blockDim.x) {
        X[t.start + i] = xs[t.start + i]; Y[t.start + i] = ys[t.start + i]; I[t.start + i] = is[t.start + i];
    }
}

// ------------------------------------------------- in-LDS completion kernel
// Sorted lists LX (by x, index) and LY (by y, index) of local point ids; a
// split along an axis keeps that axis' list as is (its first floor(n/2)
// entries are the lower half) and stably partitions the other list.  Both
// lists hold every sub-segment at the same positions, so a thread owns
// positions [kPer*tid, kPer*tid + kPer) of both and keeps the sub-segment of
// each of them (start, count, box) in registers.  posX/posY invert the
// lists: an element is in the lower half of its sub-segment iff its
// position in the split axis' list is below start + count/2.
constexpr int kLdsThreads = 1024;
constexpr int kLdsWaves = kLdsThreads / 64;
constexpr int kPer = kLdsCap / kLdsThreads;     // positions (and buckets) per thread

struct LdsSort {
    uint64_t key[kLdsCap];
    uint16_t id[kLdsCap];
};
struct LdsPos {
    uint16_t posX[kLdsCap];
    uint16_t posY[kLdsCap];
};
struct LdsBucket {
    uint32_t cnt[kLdsCap];      // bucket populations, then bucket ends
    uint64_t key[kLdsCap];      // order keys in bucket order
    uint16_t id[kLdsCap];       // local ids in bucket order (any order inside a bucket)
};
union LdsUnion {
    LdsSort s;
    LdsPos q;
    LdsBucket b;
};

__device__ void lds_sort(LdsSort& S, const uint32_t* idxs, int n)
{
    int P = 1;
    while (P < n) P <<= 1;
    for (int kk = 2; kk <= P; kk <<= 1)
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P / 2; i += kLdsThreads) {
                int lo = ((i & ~(j - 1)) << 1) | (i & (j - 1));
                int hi = lo + j;
                bool asc = (lo & kk) == 0;
                uint64_t a = S.key[lo], b = S.key[hi];
                uint16_t ia = S.id[lo], ib = S.id[hi];
                bool less_hl;
                if (ib == 0xffff) less_hl = false;          // padding sorts last
                else if (ia == 0xffff) less_hl = true;
                else less_hl = (b < a) || (b == a && idxs[ib] < idxs[ia]);
                if (less_hl == asc) {
                    S.key[lo] = b; S.key[hi] = a;
                    uint16_t c = S.id[lo]; S.id[lo] = S.id[hi]; S.id[hi] = c;
                }
            }
            __syncthreads();
        }
}

// Local ids 0..n-1 of the segment ordered by (coordinate, input index) into
// out.  Bucket sort: kLdsCap equal-width buckets between the segment's
// minimum and maximum coordinate (a monotone map), an exclusive scan of the
// populations, a scatter, and the place of every element inside its bucket
// from the count of the bucket's elements that precede it.  When a bucket
// holds more than kBucketMax points (ties, tight clusters) the bitonic sort
// runs instead.
constexpr int kBucketMax = 16;

__device__ void lds_order(LdsUnion& U, const double* __restrict__ c, const uint32_t* idxs, int n, uint16_t* out,
                          int* sh, double* red)
{
    constexpr int NB = kLdsCap;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    // range of the coordinate
    double lo = 1e308, hi = -1e308;
    double cv[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int i = tid + u * kLdsThreads;
        cv[u] = i < n ? c[i] : 0.0;
        if (i < n) { lo = fmin(lo, cv[u]); hi = fmax(hi, cv[u]); }
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    if (lane == 0) { red[wid] = lo; red[kLdsWaves + wid] = hi; }
    for (int b = tid; b < NB; b += kLdsThreads) U.b.cnt[b] = 0;
    __syncthreads();
    lo = red[0]; hi = red[kLdsWaves];
    for (int w = 1; w < kLdsWaves; ++w) { lo = fmin(lo, red[w]); hi = fmax(hi, red[kLdsWaves + w]); }
    const double ext = hi - lo;
    double scale = ext > 0.0 ? (double)NB / ext : 0.0;
    scale = scale < 1e300 ? scale : 0.0;
    int bk[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int i = tid + u * kLdsThreads;
        bk[u] = (int)fmin(fmax((cv[u] - lo) * scale, 0.0), (double)(NB - 1));
        if (i < n) atomicAdd(&U.b.cnt[bk[u]], 1u);
    }
    __syncthreads();
    // exclusive scan of the populations (thread t owns buckets kPer t .. kPer t + kPer - 1) and
    // the largest population
    uint32_t q[kPer];
    int loc = 0, mx = 0;
#pragma unroll
    for (int v = 0; v < kPer; ++v) {
        q[v] = U.b.cnt[kPer * tid + v];
        loc += (int)q[v];
        mx = max(mx, (int)q[v]);
    }
    mx = wave_max_i32(mx);
    int tot;
    int run = block_excl_scan<kLdsThreads>(loc, sh, &tot);
    if (lane == 0) sh[kLdsWaves + wid] = mx;
#pragma unroll
    for (int v = 0; v < kPer; ++v) {
        U.b.cnt[kPer * tid + v] = (uint32_t)run;
        run += (int)q[v];
    }
    __syncthreads();
    mx = 0;
    for (int w = 0; w < kLdsWaves; ++w) mx = max(mx, sh[kLdsWaves + w]);
    __syncthreads();
    if (mx > kBucketMax) {
        // bitonic fallback (uniform branch)
        int P = 1;
        while (P < n) P <<= 1;
        for (int i = tid; i < P; i += kLdsThreads) {
            if (i < n) { U.s.key[i] = okey(c[i]); U.s.id[i] = (uint16_t)i; }
            else { U.s.key[i] = ~0ull; U.s.id[i] = 0xffff; }
        }
        __syncthreads();
        lds_sort(U.s, idxs, n);
        for (int i = tid; i < n; i += kLdsThreads) out[i] = U.s.id[i];
        __syncthreads();
        return;
    }
    // scatter into bucket order; cnt becomes the end of every bucket
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int i = tid + u * kLdsThreads;
        if (i < n) {
            const uint32_t pos = atomicAdd(&U.b.cnt[bk[u]], 1u);
            U.b.key[pos] = okey(cv[u]);
            U.b.id[pos] = (uint16_t)i;
        }
    }
    __syncthreads();
    // the place of every element inside its bucket (at most kBucketMax
    // elements): the count of the bucket's elements smaller in (key, input
    // index); the reads of the bucket are independent, so they are issued
    // together
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int i = tid + u * kLdsThreads;
        if (i < n) {
            const int b = bk[u];
            const int e = (int)U.b.cnt[b], s0 = b == 0 ? 0 : (int)U.b.cnt[b - 1];
            const uint64_t km = okey(cv[u]);
            const uint32_t xm = idxs[i];
            // the first kRankFirst keys of the bucket are read unconditionally
            // (indices clamped into the bucket, which holds this element);
            // the input index only for an exact tie; larger buckets go on
            constexpr int kRankFirst = 8;
            uint64_t kk[kRankFirst];
#pragma unroll
            for (int t = 0; t < kRankFirst; ++t) kk[t] = U.b.key[min(s0 + t, e - 1)];
            int r = 0;
#pragma unroll
            for (int t = 0; t < kRankFirst; ++t) {
                if (s0 + t < e) {
                    r += kk[t] < km;
                    if (kk[t] == km) r += idxs[U.b.id[s0 + t]] < xm;
                }
            }
            for (int q = s0 + kRankFirst; q < e; ++q) {
                const uint64_t kq = U.b.key[q];
                r += (kq < km) | ((kq == km) & (idxs[U.b.id[q]] < xm));
            }
            out[s0 + r] = (uint16_t)i;
        }
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kLdsThreads)
k_lds_split(const LdsWork* __restrict__ work, const double* XA, const double* YA, const int32_t* IA,
            const double* XB, const double* YB, const int32_t* IB, double* Xo, double* Yo, int32_t* Io,
            double* bbox, double* geom)
{
    __shared__ LdsUnion U;
    __shared__ uint32_t idxs[kLdsCap];
    __shared__ uint16_t LX[kLdsCap], LY[kLdsCap];
    __shared__ int sh[2 * (kLdsThreads / 64)];
    __shared__ double red[2 * (kLdsThreads / 64)];
    __shared__ double xs[kLdsCap], ys[kLdsCap];   // coordinates by local id
    LdsWork w = work[blockIdx.x];
    const double* xg = ((w.stage0 & 1) ? XB : XA) + w.start;
    const double* yg = ((w.stage0 & 1) ? YB : YA) + w.start;
    const int32_t* is = ((w.stage0 & 1) ? IB : IA) + w.start;
    int n = w.count;
    {
        // every load of the segment in flight before the first LDS store
        uint32_t li[kPer];
        double lx[kPer], ly[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int i = threadIdx.x + u * kLdsThreads;
            const int ic = i < n ? i : 0;
            li[u] = (uint32_t)is[ic];
            lx[u] = xg[ic];
            ly[u] = yg[ic];
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int i = threadIdx.x + u * kLdsThreads;
            if (i < n) {
                idxs[i] = li[u];
                xs[i] = lx[u];
                ys[i] = ly[u];
            }
        }
    }
    __syncthreads();
    lds_order(U, xs, idxs, n, LX, sh, red);
    lds_order(U, ys, idxs, n, LY, sh, red);
    uint16_t* posX = U.q.posX;
    uint16_t* posY = U.q.posY;
    for (int i = threadIdx.x; i < n; i += kLdsThreads) {
        posX[LX[i]] = (uint16_t)i;
        posY[LY[i]] = (uint16_t)i;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int st[kPer], cn[kPer], sid[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) { st[u] = 0; cn[u] = n; sid[u] = 0; }
    for (int d = 0; d <= w.stages; ++d) {
        const int t = w.stage0 + d;
        // split axis of the sub-segment of every owned position, from the
        // ends of both lists; the head position (the sub-segment's first)
        // writes the box geometry at even stages
        int ax[kPer];
        bool valid[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int i = kPer * threadIdx.x + u;
            valid[u] = i < n;
            ax[u] = 0;
            if (!valid[u]) continue;
            if (u > 0 && valid[u - 1] && st[u] == st[u - 1]) { ax[u] = ax[u - 1]; continue; }
            const int e1 = st[u] + cn[u] - 1;
            const double x0 = xs[LX[st[u]]], x1 = xs[LX[e1]];
            const double y0 = ys[LY[st[u]]], y1 = ys[LY[e1]];
            ax[u] = ((x1 - x0) >= (y1 - y0)) ? 0 : 1;
            if (i == st[u] && (t & 1) == 0) {
                const int64_t box = (int64_t)w.boxbase + level_base(t / 2) + ((int64_t)w.j0 << d) + sid[u];
                double bb[4], gm[3];
                box_geometry(x0, x1, y0, y1, bb, gm);
                for (int c = 0; c < 4; ++c) bbox[4 * box + c] = bb[c];
                for (int c = 0; c < 3; ++c) geom[4 * box + c] = gm[c];
            }
        }
        if (d == w.stages) break;
        // element of the other list at every owned position and whether it
        // lies in the lower half along the split axis
        uint16_t e[kPer];
        int f[kPer], lb[kPer];
        bool tail[kPer];   // no head at or before this position within the thread
        int run = 0;
        bool seen = false;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int i = kPer * threadIdx.x + u;
            f[u] = 0;
            e[u] = 0;
            if (valid[u]) {
                e[u] = ax[u] ? LX[i] : LY[i];
                const int pa = ax[u] ? (int)posY[e[u]] : (int)posX[e[u]];
                f[u] = (pa - st[u]) < (cn[u] >> 1);
                if (i == st[u]) { run = 0; seen = true; }
            }
            tail[u] = !seen;
            lb[u] = run;
            run += f[u];
        }
        // segmented exclusive scan of the lower flags over the positions
        // (restarting at every sub-segment head): within the wavefront by
        // lane permutations, across wavefronts through one barrier
        int v = run, hf = seen ? 1 : 0, ev, eh;
        wave_seg_scan(hf, v, eh, ev);
        if (lane == 63) { sh[wid] = v; sh[kLdsWaves + wid] = hf; }
        __syncthreads();
        int carry = 0;
        for (int q = 0; q < wid; ++q) carry = sh[kLdsWaves + q] ? sh[q] : carry + sh[q];
        const int cin = eh ? ev : carry + ev;
        // scatter the other list's elements in place (every read of the
        // lists and positions of this stage came before the barrier) and
        // step every owned position into its child
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            if (!valid[u]) continue;
            const int i = kPer * threadIdx.x + u;
            const int before = lb[u] + (tail[u] ? cin : 0);   // lower elements in [st, i)
            const int kq = cn[u] >> 1, rel = i - st[u];
            const int dst = f[u] ? st[u] + before : st[u] + kq + (rel - before);
            if (ax[u]) { LX[dst] = e[u]; posX[e[u]] = (uint16_t)dst; }
            else { LY[dst] = e[u]; posY[e[u]] = (uint16_t)dst; }
            if (rel < kq) { cn[u] = kq; sid[u] = 2 * sid[u]; }
            else { st[u] += kq; cn[u] -= kq; sid[u] = 2 * sid[u] + 1; }
        }
        __syncthreads();
    }
    // final order: sorted by (x, index) inside every leaf
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int i = threadIdx.x + u * kLdsThreads;
        if (i < n) {
            const int id = LX[i];
            Xo[w.start + i] = xs[id]; Yo[w.start + i] = ys[id]; Io[w.start + i] = (int32_t)idxs[id];
        }
    }
}

// scaling radius: r, else the nearest ancestor's r, else 1
__global__ void k_scaling_radius(int64_t nbox, const int32_t* __restrict__ parent, double* geom)
{
    int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    int64_t a = b;
    double rs = 1.0;
    while (a >= 0) {
        double r = geom[4 * a + 2];
        if (r > 0.0) { rs = r; break; }
        a = parent[a];
    }
    geom[4 * b + 3] = rs;
}

__global__ void k_update_positions(const double* __restrict__ z, const int32_t* __restrict__ perm,
                                   int64_t n, double* X, double* Y)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 v = reinterpret_cast<const double2*>(z)[perm[i]];
    X[i] = v.x; Y[i] = v.y;
}

// ------------------------------------------------------------------- driver

static int grid_for(int64_t n, int bs) { return (int)std::min<int64_t>((n + bs - 1) / bs, 65535 * 4); }

static void build_tree_select(Tree& t, const double* z, hipStream_t s)
{
    TreeSchedule& sc = *t.sched;
    int64_t n = sc.n;
    // workspace
    DBuf<double> XA, YA, XB, YB;
    DBuf<int32_t> IA, IB;
    XA.alloc(n, s); YA.alloc(n, s); IA.alloc(n, s);
    if (sc.nstage > 0) { XB.alloc(n, s); YB.alloc(n, s); IB.alloc(n, s); }
    int64_t nkeys = sc.total_keys;
    DBuf<uint64_t> keys; keys.alloc(kKeyWords * nkeys, s);
    int64_t nseg_split = sc.nstage > 0 ? sc.keys_off[sc.nstage] : 0;   // segments of split stages
    DBuf<uint32_t> words;   // hist1 | hist2 | cand_cnt | tiles done per segment | tile_below | tile_extra | lo_base | err
    int64_t nt = sc.total_tile;
    int64_t o_h1 = 0, o_h2 = nseg_split * 2 * kHistCopies * kBuckets1, o_cc = o_h2 + nseg_split * kBuckets2;
    int64_t o_sd = o_cc + nseg_split, o_tb = o_sd + nseg_split;
    int64_t o_te = o_tb + nt, o_lb = o_te + nt, o_err = o_lb + nt, nwords = o_err + 1;
    words.alloc(nwords, s);
    DBuf<Cand> cand; cand.alloc(std::max<int64_t>(nseg_split, 1) * kCandCap, s);
    DBuf<Splitter> split; split.alloc(std::max<int64_t>(nseg_split, 1), s);
    DBuf<ClassInfo> cinfo; cinfo.alloc(std::max<int64_t>(nseg_split, 1), s);
    DBuf<Level1> lvl1; lvl1.alloc(std::max<int64_t>(nseg_split, 1), s);

    k_fill_start<<<grid_for(std::max<int64_t>(nwords, kKeyWords * nkeys), 256), 256, 0, s>>>(
        words.p, nwords, keys.p, kKeyWords * nkeys, t.err.p);
    check_launch("fill");
    uint32_t* W = words.p;
    // init: every problem's root segment is stage-0 key segment b
    int64_t maxn = 0;
    for (int b = 0; b < sc.nprob; ++b) maxn = std::max(maxn, sc.off[b + 1] - sc.off[b]);
    dim3 gi((unsigned)((maxn + kTile - 1) / kTile), (unsigned)sc.nprob);
    k_init<<<gi, kTileThreads, 0, s>>>(z, sc.d_off.p, sc.nprob, XA.p, YA.p, IA.p, keys.p, t.err.p);
    check_launch("init");
    double* Xb[2] = {XA.p, XB.p};
    double* Yb[2] = {YA.p, YB.p};
    int32_t* Ib[2] = {IA.p, IB.p};
    for (int st = 0; st < sc.nstage; ++st) {
        int ntl = sc.ntile[st];
        if (ntl == 0) continue;
        const TileInfo* tl = sc.d_tiles.p + sc.tile_off[st];
        int a = st & 1;
        // later stages' first-level histograms come from the previous partition
        if (st == 0) k_hist1<<<ntl, kTileThreads, 0, s>>>(tl, Xb[a], Yb[a], keys.p, W + o_h1);
        k_hist2<<<ntl, kTileThreads, 0, s>>>(tl, sc.d_segs.p, Xb[a], Yb[a], keys.p, W + o_h1, W + o_h2, lvl1.p);
        k_collect<<<ntl, kTileThreads, 0, s>>>(tl, sc.d_tiles.p, sc.d_segs.p, Xb[a], Yb[a], Ib[a], lvl1.p, W + o_h2,
                                              cand.p, W + o_cc, W + o_tb, W + o_sd, cinfo.p, W + o_lb, split.p);
        k_partition<<<ntl, kTileThreads, 0, s>>>(tl, sc.d_segs.p, Xb[a], Yb[a], Ib[a], Xb[a ^ 1], Yb[a ^ 1],
                                                Ib[a ^ 1], keys.p, cinfo.p, cand.p, W + o_tb, split.p, W + o_lb,
                                                W + o_h1, lvl1.p);
        check_launch("split stage");
    }
    if (!sc.lds.empty()) {
        k_lds_split<<<(unsigned)sc.lds.size(), kLdsThreads, 0, s>>>(sc.d_lds.p, XA.p, YA.p, IA.p, XB.p, YB.p,
                                                                    IB.p, t.x.p, t.y.p, t.perm.p, t.bbox.p,
                                                                    t.geom.p);
        check_launch("lds split");
    }
    if (!sc.copy_tiles.empty()) {
        k_copy_final<<<(unsigned)sc.copy_tiles.size(), 256, 0, s>>>(sc.d_copy.p, XA.p, YA.p, IA.p, XB.p, YB.p,
                                                                    IB.p, t.x.p, t.y.p, t.perm.p);
        check_launch("copy final");
    }
    if (!sc.geom.empty()) {
        int64_t ng = (int64_t)sc.geom.size();
        k_geom_keys<<<grid_for(ng, 256), 256, 0, s>>>(sc.d_geom.p, ng, keys.p, t.bbox.p, t.geom.p);
        check_launch("geom");
    }
    k_scaling_radius<<<grid_for(sc.nbox, 256), 256, 0, s>>>(sc.nbox, sc.d_box_parent.p, t.geom.p);
    check_launch("scaling radius");
    // non-finite positions: t.err, read at the next synchronising call on the tree
}

void build_tree_device(Tree& t, const double* z, hipStream_t s)
{
    TreeSchedule& sc = *t.sched;
    const int64_t n = sc.n;
    t.x.alloc(n, s); t.y.alloc(n, s); t.perm.alloc(n, s);
    t.bbox.alloc(4 * sc.nbox, s); t.geom.alloc(4 * sc.nbox, s);
    t.err.alloc(1, s);
    build_tree_select(t, z, s);
}

void update_positions_device(Tree& t, const double* z, hipStream_t s)
{
    int64_t n = t.sched->n;
    k_update_positions<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(z, t.perm.p, n, t.x.p, t.y.p);
    check_launch("update positions");
}

}  // namespace fmm
