// evaluate.hip -- the FMM evaluation sequence (Sec. 2.1, Fig. 2.2) and the
// host-side work lists of a plan.
//
//   gather  strengths to tree order (the P2P sources, with the tree's positions)
//   P2M     leaves of every problem (does the gather when the leaves hold
//           every point, which is the case for every tree this library builds)
//   M2M     level by level, deepest parents first
//   M2L     every box over its weak list (writes the box's local expansion)
//   L2L     level by level from level 2 down (adds the parent's expansion)
//   P2P     leaves over their strong lists (near field, tree order)
//   L2P     leaves: far field + near field, scattered to input order
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <type_traits>

#include "fmm_internal.h"
#include "kernels_common.h"
#include "plan_extra.h"

namespace fmm {

void launch_gather(int64_t n, const int32_t* perm, const double* m, double* mtree, hipStream_t s);
template <class T>
void launch_p2m(const int32_t*, int, const int32_t*, const int32_t*, int, const double*, const double*,
                const double*, const double*, int, void*, hipStream_t, const int32_t* = nullptr,
                const double* = nullptr, const GatherOut* = nullptr);
template <class T>
void launch_m2m(const int32_t*, int, const int32_t*, const double*, const double*, int, void*, hipStream_t);
template <class T>
void launch_l2l(const int32_t*, int, const int32_t*, const double*, const double*, int, void*, hipStream_t);
template <class T>
void launch_l2p(const int32_t*, int, const int32_t*, const int32_t*, int, const double*, const double*,
                const double*, void*, int, const double*, const int32_t*, double*, double*, double*, hipStream_t,
                const long long*, const int32_t*, const double*);
template <class T>
void launch_m2l(const int32_t*, int, const int2*, int, const int32_t*, const int32_t*, double*, bool,
                const int32_t*, const int32_t*, const int32_t*, const double*, const double*, int, const void*, void*,
                hipStream_t, int, const long long*);

bool subtree_ok(int L, int p);
template <class T>
void launch_up_subtree(int nprob, int L, const int32_t* bstart, const int32_t* bcount, const double* geom,
                       const double* X, const double* Y, const double* mt, int p, void* mp, const double* binom,
                       const GatherOut* go, hipStream_t s, hipEvent_t after_leaves = nullptr);
template <class T>
void launch_down_subtree(int nprob, int L, const int32_t* bstart, const int32_t* bcount, const double* geom,
                         const double* X, const double* Y, void* loc, int p, const double* nearf,
                         const int32_t* perm, double* phi, double* phi_near, double* phi_far, const long long* guard,
                         const double* binom, hipStream_t s);

struct P2PItemH {
    int32_t leaf, t0, tn, pad;
};

// P2P launch shape for a leaf of nt targets: SUB lane subgroups, TG targets
// per lane (TG <= 8 in FP64, <= 16 in FP32, and 2 TG <= 64/SUB); a work item
// covers at most TG*SUB targets.  `knob` (> 0) fixes SUB, `tknob` (> 0) TG
// (with SUB then the most subgroups that TG allows unless knob fixes it).
static void p2p_shape(int nt, int knob, int tknob, bool mixed, int* tg, int* sub)
{
    if (tknob > 0) {
        *tg = tknob;
        *sub = knob > 0 ? knob : (tknob <= 4 ? 4 : 2);
        return;
    }
    int tgmax = mixed ? 16 : 8;
    int s = knob > 0 ? knob : 4;   // measured best for 15..61 targets per leaf, both precisions
    int need = (nt + s - 1) / s;
    int t = 1;
    while (t < need && t < tgmax) t <<= 1;
    int lo = s == 4 ? 1 : (s == 2 ? 2 : 4);
    int hi = s == 4 ? 4 : tgmax;
    t = t < lo ? lo : (t > hi ? hi : t);
    *tg = t;
    *sub = s;
}

template <class T>
static void upload_vec(DBuf<T>& d, const std::vector<T>& h, hipStream_t s)
{
    d.alloc(std::max<size_t>(h.size(), 1), s);
    if (!h.empty())
        FMM_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

void prepare_plan_host(Plan& pl, PlanExtra& ex, hipStream_t s)
{
    TreeSchedule& sc = *pl.tree->sched;
    int ml = sc.max_levels;
    ex.level_boxes.assign(ml, {});
    ex.m2m_boxes.assign(ml, {});
    std::vector<int32_t> leaves, child0(sc.nbox, -1);
    for (int b = 0; b < sc.nprob; ++b) {
        for (int l = 0; l < sc.L[b]; ++l) {
            int64_t base = sc.pbox[b] + level_base(l);
            for (int64_t j = 0; j < (int64_t(1) << (2 * l)); ++j) {
                int32_t id = (int32_t)(base + j);
                ex.level_boxes[l].push_back(id);
                if (l + 1 < sc.L[b]) {
                    child0[id] = (int32_t)(sc.pbox[b] + level_base(l + 1) + 4 * j);
                    ex.m2m_boxes[l].push_back(id);
                } else {
                    leaves.push_back(id);
                    ex.leaf_max = std::max(ex.leaf_max, (int)sc.box_count[id]);
                }
            }
        }
    }
    {
        bool same = sc.nprob > 0;
        for (int b = 0; b < sc.nprob; ++b) same = same && sc.L[b] == sc.L[0];
        ex.leaf_l2l_in_l2p = same && sc.L[0] >= 2;
        ex.leaf_m2m_in_p2m = ex.leaf_l2l_in_l2p && ex.leaf_max <= 16;
        int64_t covered = 0;
        for (int32_t g : leaves) covered += sc.box_count[g];
        ex.gather_in_p2m = covered == sc.n;
    }
    std::vector<int32_t> all;
    ex.level_boxes_off.assign(ml + 1, 0);
    for (int l = 0; l < ml; ++l) {
        ex.level_boxes_off[l] = (int64_t)all.size();
        all.insert(all.end(), ex.level_boxes[l].begin(), ex.level_boxes[l].end());
    }
    ex.level_boxes_off[ml] = (int64_t)all.size();
    upload_vec(ex.d_level_boxes, all, s);
    upload_vec(ex.leaves, leaves, s);
    upload_vec(ex.child0, child0, s);
    std::vector<int32_t> m2m;
    ex.m2m_off.assign(ml + 1, 0);
    for (int l = 0; l < ml; ++l) {
        ex.m2m_off[l] = (int64_t)m2m.size();
        m2m.insert(m2m.end(), ex.m2m_boxes[l].begin(), ex.m2m_boxes[l].end());
    }
    ex.m2m_off[ml] = (int64_t)m2m.size();
    upload_vec(ex.d_m2m, m2m, s);
    // P2P work items grouped by launch shape
    const bool mixed = pl.precision == FMM_MIXED;
    std::map<std::pair<int, int>, std::vector<P2PItemH>> cls;
    for (int32_t g : leaves) {
        int nt = sc.box_count[g];
        int tg, sub;
        p2p_shape(nt, pl.tune.p2p_split, pl.tune.p2p_targets, mixed, &tg, &sub);
        int chunk = tg * sub;
        for (int t0 = 0; t0 < nt; t0 += chunk)
            cls[{tg, sub}].push_back(P2PItemH{g, t0, std::min(chunk, nt - t0), 0});
    }
    std::vector<P2PItemH> items;
    ex.p2p_class.clear();
    for (auto& kv : cls) {
        ex.p2p_class.push_back({kv.first.first, kv.first.second, (int64_t)items.size(), (int64_t)kv.second.size()});
        items.insert(items.end(), kv.second.begin(), kv.second.end());
    }
    {
        std::vector<char> raw(items.size() * sizeof(P2PItemH));
        if (!items.empty()) std::memcpy(raw.data(), items.data(), raw.size());
        upload_vec(ex.p2p_items, raw, s);
    }
    prepare_adjoint_items(pl, ex, leaves, s);
    // binomial table C(n, k), n < kBinomRows, k < kBinomStride (Pascal's rule)
    std::vector<double> bin(kBinomRows * kBinomStride, 0.0);
    for (int n = 0; n < kBinomRows; ++n) {
        bin[n * kBinomStride] = 1.0;
        for (int k = 1; k <= n && k < kBinomStride; ++k)
            bin[n * kBinomStride + k] = bin[(n - 1) * kBinomStride + k - 1] + (k < n ? bin[(n - 1) * kBinomStride + k] : 0.0);
    }
    upload_vec(ex.binom, bin, s);
    FMM_HIP(hipStreamSynchronize(s));
}

void alloc_eval_buffers(Plan& pl, hipStream_t s)
{
    TreeSchedule& sc = *pl.tree->sched;
    int64_t n = sc.n;
    bool mixed = pl.precision == FMM_MIXED;
    size_t cs = mixed ? sizeof(float) : sizeof(double);
    pl.mtree.alloc(2 * n, s);
    pl.near.alloc(2 * n, s);
    pl.mpole.alloc(2 * cs * sc.nbox * pl.p, s);
    pl.local.alloc(2 * cs * sc.nbox * pl.p, s);
}

// whether P2M also forms the M2M of the leaves' parents
static bool leaf_m2m(const Plan& pl, const PlanExtra& ex) { return ex.leaf_m2m_in_p2m && pl.p <= 32; }

// whether the far field runs by subtrees (subtree.hip): every problem of the
// same depth L >= 3, the leaves holding every point, p <= 32
static bool use_subtree(const Plan& pl, const PlanExtra& ex)
{
    const TreeSchedule& sc = *pl.tree->sched;
    return ex.leaf_l2l_in_l2p && ex.gather_in_p2m && subtree_ok(sc.L[0], pl.p) &&
           !(pl.tune.flags & FMM_FLAG_LEVELWISE);
}

// the whole upward pass by subtrees, with the gather
template <class T>
static void run_up_subtree(Plan& pl, const double* m, hipStream_t s, hipEvent_t after_leaves = nullptr)
{
    Tree& t = *pl.tree;
    TreeSchedule& sc = *t.sched;
    GatherOut go{t.perm.p, (const double2*)m, (double2*)pl.mtree.p};
    launch_up_subtree<T>(sc.nprob, sc.L[0], sc.d_box_start.p, sc.d_box_count.p, t.geom.p, t.x.p, t.y.p, pl.mtree.p,
                         pl.p, pl.mpole.p, pl.ex->binom.p, &go, s, after_leaves);
}

// gather (own kernel, or inside P2M) and P2M; m = strengths in input order
template <class T>
static void run_p2m(Plan& pl, PlanExtra& ex, const double* m, hipStream_t s)
{
    Tree& t = *pl.tree;
    TreeSchedule& sc = *t.sched;
    const bool mixed = std::is_same<T, float>::value;
    GatherOut go{t.perm.p, (const double2*)m, (double2*)pl.mtree.p};
    if (!ex.gather_in_p2m)
        launch_gather(sc.n, t.perm.p, m, pl.mtree.p, s);
    // with leaf_m2m_in_p2m the P2M kernel also forms the leaves' parents
    // (up to 32 terms: above that P2M runs in two blocks of terms)
    const bool fm = leaf_m2m(pl, ex);
    launch_p2m<T>(ex.leaves.p, (int)sc.nleaf, sc.d_box_start.p, sc.d_box_count.p, ex.leaf_max, t.geom.p, t.x.p, t.y.p,
                  pl.mtree.p, pl.p, pl.mpole.p, s, fm ? sc.d_box_parent.p : nullptr, ex.binom.p,
                  ex.gather_in_p2m ? &go : nullptr);
}

// M2M above what P2M formed
template <class T>
static void run_m2m(Plan& pl, PlanExtra& ex, void* mp, hipStream_t s)
{
    Tree& t = *pl.tree;
    TreeSchedule& sc = *t.sched;
    const bool fm = leaf_m2m(pl, ex);
    for (int l = sc.max_levels - (fm ? 3 : 2); l >= 1; --l) {
        int n = (int)(ex.m2m_off[l + 1] - ex.m2m_off[l]);
        launch_m2m<T>(ex.d_m2m.p + ex.m2m_off[l], n, ex.child0.p, t.geom.p, ex.binom.p, pl.p, mp, s);
    }
}

struct PhaseTimer;

template <class T>
static void run_far_down(Plan& pl, PlanExtra& ex, const void* mp, void* loc, hipStream_t s, PhaseTimer& tm,
                         const long long* guard, bool all_l2l = false);

struct PhaseTimer {
    static constexpr int kEvents = 6;
    bool on;
    hipStream_t s;
    hipEvent_t ev[kEvents];
    int k = 0;
    PhaseTimer(bool o, hipStream_t st) : on(o), s(st)
    {
        if (on)
            for (auto& e : ev) FMM_HIP(hipEventCreate(&e));
    }
    void mark()
    {
        if (on) FMM_HIP(hipEventRecord(ev[k++], s));
    }
    float between(int a, int b)
    {
        float ms = 0;
        FMM_HIP(hipEventElapsedTime(&ms, ev[a], ev[b]));
        return ms * 1000.0f;
    }
    ~PhaseTimer()
    {
        if (on)
            for (auto& e : ev) (void)hipEventDestroy(e);
    }
};

template <class T>
static void run_far_down(Plan& pl, PlanExtra& ex, const void* mp, void* loc, hipStream_t s, PhaseTimer& tm,
                         const long long* guard, bool all_l2l)
{
    Tree& t = *pl.tree;
    TreeSchedule& sc = *t.sched;
    const Plan::Balance& b = pl.bal_m2l;
    // parents at level l (non-leaf) hand their expansion to level l+1; the
    // hand-over into the leaves is done by L2P when every problem has the
    // same depth (all_l2l: every level here, the leaves' expansions whole)
    const int lend = sc.max_levels - (ex.leaf_l2l_in_l2p && !all_l2l ? 2 : 1);
    // The top levels' chain (M2L of levels < cut, then the L2L steps among
    // them) runs on a third stream beside the M2L of the deeper levels, which
    // takes nearly all the work: every L2L step adds to a child's expansion
    // after that child's M2L wrote it, and the children of those steps are
    // all above the cut.  Lists split into chunks, and phase timing, keep the
    // single launch.
    const int cut = std::min(sc.max_levels - 3, 6);
    if (use_subtree(pl, ex) && !all_l2l) {
        // M2L only: the L2L hand-over is part of the subtree L2P.  The top
        // levels' M2L (a small, latency-bound launch) runs on the third
        // stream beside the deeper levels'.
        if (!tm.on && b.xitems.p == nullptr && b.total == sc.nbox && cut >= 1) {
            if (!pl.ev_top0) {
                FMM_HIP(hipEventCreateWithFlags(&pl.ev_top0, hipEventDisableTiming));
                FMM_HIP(hipEventCreateWithFlags(&pl.ev_top1, hipEventDisableTiming));
            }
            hipStream_t ts = side_stream(t.device, kTopStream);
            const int na = (int)ex.level_boxes_off[cut];
            const int nb = (int)(ex.level_boxes_off[sc.max_levels] - na);
            FMM_HIP(hipEventRecord(pl.ev_top0, s));
            FMM_HIP(hipStreamWaitEvent(ts, pl.ev_top0, 0));
            launch_m2l<T>(ex.d_level_boxes.p, na, nullptr, na, nullptr, nullptr, nullptr, false, pl.w_beg.p,
                          pl.w_cnt.p, pl.w_ids.p, t.geom.p, ex.binom.p, pl.p, mp, loc, ts, pl.tune.m2l_batch, guard);
            FMM_HIP(hipEventRecord(pl.ev_top1, ts));
            launch_m2l<T>(ex.d_level_boxes.p + na, nb, nullptr, nb, nullptr, nullptr, nullptr, false, pl.w_beg.p,
                          pl.w_cnt.p, pl.w_ids.p, t.geom.p, ex.binom.p, pl.p, mp, loc, s, pl.tune.m2l_batch, guard);
            FMM_HIP(hipStreamWaitEvent(s, pl.ev_top1, 0));
        } else {
            launch_m2l<T>(nullptr, (int)sc.nbox, b.xitems.p, (int)b.total, b.icnt.p, b.ioff.p, b.partial.p,
                          b.total > sc.nbox, pl.w_beg.p, pl.w_cnt.p, pl.w_ids.p, t.geom.p, ex.binom.p, pl.p, mp, loc,
                          s, pl.tune.m2l_batch, guard);
        }
        tm.mark();
        return;
    }
    const int ltop = std::min(cut - 2, lend - 1);      // last parent level of the side chain
    int lstart = 1;
    if (!tm.on && b.xitems.p == nullptr && b.total == sc.nbox && ltop >= 1) {
        if (!pl.ev_top0) {
            FMM_HIP(hipEventCreateWithFlags(&pl.ev_top0, hipEventDisableTiming));
            FMM_HIP(hipEventCreateWithFlags(&pl.ev_top1, hipEventDisableTiming));
        }
        hipStream_t ts = side_stream(t.device, kTopStream);
        const int na = (int)ex.level_boxes_off[cut];   // boxes of levels 0 .. cut-1, all problems
        const int nb = (int)(ex.level_boxes_off[sc.max_levels] - na);
        FMM_HIP(hipEventRecord(pl.ev_top0, s));
        FMM_HIP(hipStreamWaitEvent(ts, pl.ev_top0, 0));
        launch_m2l<T>(ex.d_level_boxes.p, na, nullptr, na, nullptr, nullptr, nullptr, false, pl.w_beg.p, pl.w_cnt.p,
                      pl.w_ids.p, t.geom.p, ex.binom.p, pl.p, mp, loc, ts, pl.tune.m2l_batch, guard);
        for (int l = 1; l <= ltop; ++l) {
            int n = (int)(ex.m2m_off[l + 1] - ex.m2m_off[l]);
            launch_l2l<T>(ex.d_m2m.p + ex.m2m_off[l], n, ex.child0.p, t.geom.p, ex.binom.p, pl.p, loc, ts);
        }
        FMM_HIP(hipEventRecord(pl.ev_top1, ts));
        launch_m2l<T>(ex.d_level_boxes.p + na, nb, nullptr, nb, nullptr, nullptr, nullptr, false, pl.w_beg.p,
                      pl.w_cnt.p, pl.w_ids.p, t.geom.p, ex.binom.p, pl.p, mp, loc, s, pl.tune.m2l_batch, guard);
        FMM_HIP(hipStreamWaitEvent(s, pl.ev_top1, 0));
        lstart = ltop + 1;
    } else {
        launch_m2l<T>(nullptr, (int)sc.nbox, b.xitems.p, (int)b.total, b.icnt.p, b.ioff.p, b.partial.p,
                      b.total > sc.nbox, pl.w_beg.p, pl.w_cnt.p, pl.w_ids.p, t.geom.p, ex.binom.p, pl.p, mp, loc, s,
                      pl.tune.m2l_batch, guard);
    }
    tm.mark();
    for (int l = lstart; l < lend; ++l) {
        int n = (int)(ex.m2m_off[l + 1] - ex.m2m_off[l]);
        launch_l2l<T>(ex.d_m2m.p + ex.m2m_off[l], n, ex.child0.p, t.geom.p, ex.binom.p, pl.p, loc, s);
    }
}

void combine_chunks(const Plan::Balance& b, const void* items, int n, const int32_t* bstart, double* out,
                    hipStream_t s);

static void run_p2p(Plan& pl, PlanExtra& ex, hipStream_t s, const long long* guard, bool log_kernel = false)
{
    Tree& t = *pl.tree;
    TreeSchedule& sc = *t.sched;
    bool mixed = pl.precision == FMM_MIXED;
    const Plan::Balance& b = pl.bal;
    int nitems = 0;
    for (size_t c = 0; c < ex.p2p_class.size(); ++c) {
        const P2PClass& k = ex.p2p_class[c];
        nitems = std::max<int>(nitems, (int)(k.off + k.n));
        const int64_t x0 = b.cls[c], x1 = b.cls[c + 1];
        launch_p2p(mixed, k.tg, k.sub, ex.p2p_items.p, (int)x0, b.xitems.p ? b.xitems.p + x0 : nullptr,
                   (int)(x1 - x0), b.icnt.p, b.ioff.p,
                   b.partial.p, sc.d_box_start.p, sc.d_box_count.p, pl.s_beg.p, pl.s_cnt.p, pl.s_ids.p,
                   t.x.p, t.y.p, (const double2*)pl.mtree.p, pl.near.p, s, guard,
                   pl.tune.smooth_delta > 0.0 ? 1.0 / (pl.tune.smooth_delta * pl.tune.smooth_delta) : 0.0,
                   log_kernel, Targets{}, pl.tune.p2p_src_tile);
    }
    combine_chunks(b, ex.p2p_items.p, nitems, sc.d_box_start.p, pl.near.p, s);
}

// Side streams per device (the near field; the list build), shared by all
// plans and kept until the process ends (creating a stream per plan costs
// more than a whole step).  Plans that share one are ordered by their own
// events.
hipStream_t side_stream(int device, int which)
{
    static std::mutex mu;
    static std::map<std::pair<int, int>, hipStream_t> streams;
    std::lock_guard<std::mutex> lk(mu);
    auto it = streams.find({device, which});
    if (it != streams.end()) return it->second;
    hipStream_t st = nullptr;
    FMM_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    streams[{device, which}] = st;
    return st;
}

// The evaluation's side stream and events, made when the plan is made (the
// evaluations then create nothing)
void plan_events(Plan& pl)
{
    if (!pl.nstream) {
        pl.nstream = side_stream(pl.tree->device, kNearStream);
        FMM_HIP(hipEventCreateWithFlags(&pl.ev_fork, hipEventDisableTiming));
        FMM_HIP(hipEventCreateWithFlags(&pl.ev_join, hipEventDisableTiming));
    }
    if (!pl.ev_top0) {
        FMM_HIP(hipEventCreateWithFlags(&pl.ev_top0, hipEventDisableTiming));
        FMM_HIP(hipEventCreateWithFlags(&pl.ev_top1, hipEventDisableTiming));
    }
}

// The part of an evaluation that needs no lists: gather and the upward
// pass.  evaluate_device then continues from there on the same stream (the
// near field is forked there, after the plan's remaining kernels).
void evaluate_upward(Plan& pl, const double* m, hipStream_t s)
{
    Tree& t = *pl.tree;
    TreeSchedule& sc = *t.sched;
    PlanExtra& ex = *extra(pl);
    const bool mixed = pl.precision == FMM_MIXED;
    if (!pl.nstream) {
        pl.nstream = side_stream(t.device, kNearStream);
        FMM_HIP(hipEventCreateWithFlags(&pl.ev_fork, hipEventDisableTiming));
        FMM_HIP(hipEventCreateWithFlags(&pl.ev_join, hipEventDisableTiming));
    }
    if (use_subtree(pl, ex)) {
        if (mixed) run_up_subtree<float>(pl, m, s);
        else run_up_subtree<double>(pl, m, s);
    } else if (mixed) {
        run_p2m<float>(pl, ex, m, s);
        run_m2m<float>(pl, ex, pl.mpole.p, s);
    } else {
        run_p2m<double>(pl, ex, m, s);
        run_m2m<double>(pl, ex, pl.mpole.p, s);
    }
    pl.upward_done = true;
}

// The far field of every box and nothing at the sources: the upward pass
// (with the gather of the strengths) and the M2L / L2L sweep over every
// level, so that the multipole expansion and the complete local expansion of
// every box are in the plan's buffers (evaluation at points apart from the
// sources).
void far_field_all(Plan& pl, const double* m, hipStream_t s)
{
    PlanExtra& ex = *extra(pl);
    PhaseTimer tm(false, s);
    pl.upward_done = false;
    if (pl.precision == FMM_MIXED) {
        run_p2m<float>(pl, ex, m, s);
        run_m2m<float>(pl, ex, pl.mpole.p, s);
        run_far_down<float>(pl, ex, pl.mpole.p, pl.local.p, s, tm, nullptr, true);
    } else {
        run_p2m<double>(pl, ex, m, s);
        run_m2m<double>(pl, ex, pl.mpole.p, s);
        run_far_down<double>(pl, ex, pl.mpole.p, pl.local.p, s, tm, nullptr, true);
    }
    // the plan's buffers now hold the far field of m, not a forward evaluation
    pl.have_forward = false;
}

void launch_real_to_complex(int64_t n, const double* q, double* m, hipStream_t s);
template <class T>
void launch_log_constants(int nbox, const int32_t* w_beg, const int32_t* w_cnt, const int32_t* w_ids,
                          const double* geom, const void* mp, const void* loc, int p, const int32_t* level_boxes,
                          const std::vector<int64_t>& level_off, int nlevels, const int32_t* parent, double* c0,
                          hipStream_t s);
template <class T>
void launch_l2p_log(const int32_t* leaves, int nleaf, const int32_t* bstart, const int32_t* bcount,
                    const double* geom, const double* X, const double* Y, const void* loc, int p, const double* c0,
                    const double* near, const int32_t* perm, double* u, hipStream_t s);

// The logarithmic potential (see log.hip): the harmonic upward pass and far
// field of the strengths q as complex numbers, the near field with the
// logarithmic kernel (on the second stream, beside the far field, from the
// strengths in tree order P2M writes), the constant terms of the local expansions,
// and L2P of the integrated series after the join.
void evaluate_log_device(Plan& pl, const double* q, double* u, hipStream_t s, double* mlog, double* c0)
{
    Tree& t = *pl.tree;
    TreeSchedule& sc = *t.sched;
    PlanExtra& ex = *extra(pl);
    const bool mixed = pl.precision == FMM_MIXED;
    if (!pl.nstream) {
        pl.nstream = side_stream(t.device, kNearStream);
        FMM_HIP(hipEventCreateWithFlags(&pl.ev_fork, hipEventDisableTiming));
        FMM_HIP(hipEventCreateWithFlags(&pl.ev_join, hipEventDisableTiming));
    }
    if (!mlog) {
        pl.mlog.alloc(2 * sc.n, s);
        pl.c0.alloc(sc.nbox, s);
        mlog = pl.mlog.p;
        c0 = pl.c0.p;
    }
    launch_real_to_complex(sc.n, q, mlog, s);
    PhaseTimer tm(false, s);
    if (mixed) run_p2m<float>(pl, ex, mlog, s);
    else run_p2m<double>(pl, ex, mlog, s);
    FMM_HIP(hipEventRecord(pl.ev_fork, s));
    FMM_HIP(hipStreamWaitEvent(pl.nstream, pl.ev_fork, 0));
    run_p2p(pl, ex, pl.nstream, nullptr, true);
    FMM_HIP(hipEventRecord(pl.ev_join, pl.nstream));
    if (mixed) {
        run_m2m<float>(pl, ex, pl.mpole.p, s);
        run_far_down<float>(pl, ex, pl.mpole.p, pl.local.p, s, tm, nullptr, true);
    } else {
        run_m2m<double>(pl, ex, pl.mpole.p, s);
        run_far_down<double>(pl, ex, pl.mpole.p, pl.local.p, s, tm, nullptr, true);
    }
    auto constants = mixed ? launch_log_constants<float> : launch_log_constants<double>;
    constants((int)sc.nbox, pl.w_beg.p, pl.w_cnt.p, pl.w_ids.p, t.geom.p, pl.mpole.p, pl.local.p, pl.p,
              ex.d_level_boxes.p, ex.level_boxes_off, sc.max_levels, sc.d_box_parent.p, c0, s);
    FMM_HIP(hipStreamWaitEvent(s, pl.ev_join, 0));
    auto l2p = mixed ? launch_l2p_log<float> : launch_l2p_log<double>;
    l2p(ex.leaves.p, (int)sc.nleaf, sc.d_box_start.p, sc.d_box_count.p, t.geom.p, t.x.p, t.y.p, pl.local.p, pl.p,
        c0, pl.near.p, t.perm.p, u, s);
    // the harmonic state of the plan now holds these strengths: no adjoint of it
    pl.have_forward = false;
}

void evaluate_device(Plan& pl, const double* m, double* phi, double* phi_near, double* phi_far, hipStream_t s,
                     hipEvent_t lists_ev, const long long* guard)
{
    Tree& t = *pl.tree;
    TreeSchedule& sc = *t.sched;
    PlanExtra& ex = *extra(pl);
    bool mixed = pl.precision == FMM_MIXED;
    PhaseTimer tm((pl.tune.flags & FMM_FLAG_PHASE_TIMING) != 0, s);
    // The near field needs only the gathered sources: it runs on a second
    // stream beside the far-field chain (P2M .. L2L) and joins before L2P.
    // Phase timing keeps the phases one after another on `s`.
    const bool overlap = !tm.on;
    if (lists_ev && !overlap) throw Error(FMM_EINVAL, "an evaluation ahead of its lists needs the overlapped order");
    if (overlap && !pl.nstream) {
        pl.nstream = side_stream(t.device, kNearStream);
        FMM_HIP(hipEventCreateWithFlags(&pl.ev_fork, hipEventDisableTiming));
        FMM_HIP(hipEventCreateWithFlags(&pl.ev_join, hipEventDisableTiming));
    }
    tm.mark();
    const bool up = pl.upward_done && overlap;   // gather and upward pass enqueued by evaluate_upward
    pl.upward_done = false;
    const bool sub = use_subtree(pl, ex);
    // by subtrees, the near field forks as soon as the leaves' kernel (which
    // writes the strengths in tree order) is done, beside the upper levels' M2M
    const bool early_fork = overlap && !up && sub;
    if (!up) {
        if (sub) {
            hipEvent_t ev = early_fork ? pl.ev_fork : nullptr;
            if (mixed) run_up_subtree<float>(pl, m, s, ev);
            else run_up_subtree<double>(pl, m, s, ev);
        } else if (mixed) {
            run_p2m<float>(pl, ex, m, s);
        } else {
            run_p2m<double>(pl, ex, m, s);
        }
    }
    if (overlap) {
        // the near field starts after everything enqueued on `s` so far: the
        // gather (with P2M), and the list and work-chunk kernels of the plan
        // (which follow the upward pass when evaluate_upward ran first); or,
        // by subtrees, after the leaves' kernel (the event recorded there)
        if (!early_fork) FMM_HIP(hipEventRecord(pl.ev_fork, s));
        FMM_HIP(hipStreamWaitEvent(pl.nstream, pl.ev_fork, 0));
        if (lists_ev) FMM_HIP(hipStreamWaitEvent(pl.nstream, lists_ev, 0));
        run_p2p(pl, ex, pl.nstream, guard);
        FMM_HIP(hipEventRecord(pl.ev_join, pl.nstream));
    }
    if (!up && !sub) {
        if (mixed) run_m2m<float>(pl, ex, pl.mpole.p, s);
        else run_m2m<double>(pl, ex, pl.mpole.p, s);
    }
    tm.mark();
    if (lists_ev) FMM_HIP(hipStreamWaitEvent(s, lists_ev, 0));
    if (mixed) run_far_down<float>(pl, ex, pl.mpole.p, pl.local.p, s, tm, guard);
    else run_far_down<double>(pl, ex, pl.mpole.p, pl.local.p, s, tm, guard);
    tm.mark();
    if (overlap) FMM_HIP(hipStreamWaitEvent(s, pl.ev_join, 0));
    else run_p2p(pl, ex, s, nullptr);
    tm.mark();
    if (sub) {
        auto down = mixed ? launch_down_subtree<float> : launch_down_subtree<double>;
        down(sc.nprob, sc.L[0], sc.d_box_start.p, sc.d_box_count.p, t.geom.p, t.x.p, t.y.p, pl.local.p, pl.p,
             pl.near.p, t.perm.p, phi, phi_near, phi_far, guard, ex.binom.p, s);
    } else if (mixed)
        launch_l2p<float>(ex.leaves.p, (int)sc.nleaf, sc.d_box_start.p, sc.d_box_count.p, ex.leaf_max, t.geom.p, t.x.p, t.y.p,
                          pl.local.p, pl.p, pl.near.p, t.perm.p, phi, phi_near, phi_far, s, guard,
                          ex.leaf_l2l_in_l2p ? sc.d_box_parent.p : nullptr, ex.binom.p);
    else
        launch_l2p<double>(ex.leaves.p, (int)sc.nleaf, sc.d_box_start.p, sc.d_box_count.p, ex.leaf_max, t.geom.p, t.x.p, t.y.p,
                           pl.local.p, pl.p, pl.near.p, t.perm.p, phi, phi_near, phi_far, s, guard,
                          ex.leaf_l2l_in_l2p ? sc.d_box_parent.p : nullptr, ex.binom.p);
    tm.mark();
    if (tm.on) {
        FMM_HIP(hipEventSynchronize(tm.ev[5]));
        pl.t_up = tm.between(0, 1);
        pl.t_m2l = tm.between(1, 2);
        pl.t_l2l = tm.between(2, 3);
        pl.t_p2p = tm.between(3, 4);
        pl.t_down = tm.between(4, 5);
        pl.t_total = tm.between(0, 5);
    }
    pl.have_forward = true;
}

}  // namespace fmm
