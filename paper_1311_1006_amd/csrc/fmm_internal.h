// fmm_internal.h -- shared declarations of the HIP FMM library (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fmm.h"

namespace fmm {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define FMM_HIP(call)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            throw ::fmm::Error(e_ == hipErrorOutOfMemory ? FMM_ENOMEM : FMM_EDEVICE,      \
                               std::string(#call) + ": " + hipGetErrorString(e_));        \
    } while (0)

#define FMM_REQUIRE(cond, msg)                                                            \
    do {                                                                                  \
        if (!(cond)) throw ::fmm::Error(FMM_EINVAL, msg);                                 \
    } while (0)

inline void check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        throw Error(FMM_EDEVICE, std::string("launch ") + what + ": " + hipGetErrorString(e));
}

// ------------------------------------------------------------- constants
constexpr int kMaxLevels = 16;
constexpr int kMaxP = 64;          // expansion terms at most (Table 4.1 reaches p = 39)
// tree build
constexpr int kTile = 2048;        // points per workgroup tile in the global split stages
constexpr int kTileThreads = 256;
constexpr int kBuckets = 2048;     // histogram buckets per level of bucket selection
constexpr int kCandCap = 2048;     // candidates sorted in LDS by one workgroup
constexpr int kLdsCap = 4096;      // segments at most this large finish in one workgroup
constexpr int kChunkSrc = 2048;    // near-field sources per work chunk (longer lists are split)
constexpr int kItemTargets = 32;   // targets per near-field work item, at most

// Targets of the near-field kernels other than the leaves' own points
// (evaluation points apart from the sources): FP64 positions x[], y[],
// sorted by leaf, start[g] = the first target of leaf g.
// start == nullptr: the targets are the leaves' own points.
// whether the near-field kernel has a shape with tg targets per lane and
// `split` lane subgroups (split 0: some subgroup count does): 4 subgroups
// take 1..4 targets per lane, 2 take 2..16, 1 takes 4..16
inline bool p2p_shape_ok(int tg, int split)
{
    return split == 0 || (split == 4 && tg <= 4) || (split == 2 && tg >= 2) || (split == 1 && tg >= 4);
}

struct Targets {
    const double* x = nullptr;
    const double* y = nullptr;
    const int32_t* start = nullptr;
};

// The near field over the chunks of one launch class (p2p.hip): the sources
// are the points in tree order, positions X, Y and strengths M (FP64; the
// mixed kernels round the strengths to FP32 as they stage them).
void launch_p2p(bool mixed, int tg, int sub, const void* items, int item_base, const int2* xitems, int nx,
                const int32_t* icnt, const int32_t* ioff, double* partial, const int32_t* bstart,
                const int32_t* bcount, const int32_t* s_beg, const int32_t* s_cnt, const int32_t* s_ids,
                const double* X, const double* Y, const double2* M, double* out, hipStream_t s,
                const long long* guard, double id2, bool log_kernel, const Targets& tgt = Targets{},
                int src_tile = 0);
constexpr int kChunkPairs = 128;   // M2L weak pairs per work chunk (longer lists are split)

__host__ __device__ inline int64_t level_base(int l) { return ((int64_t(1) << (2 * l)) - 1) / 3; }
__host__ __device__ inline int64_t nbox_levels(int L) { return level_base(L); }

// ---------------------------------------------------------- device memory
void* dev_alloc(size_t bytes, hipStream_t s);
void dev_free(void* p, hipStream_t s);

template <class T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    hipStream_t s = nullptr;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void alloc(size_t count, hipStream_t st) {
        release();
        s = st;
        n = count;
        if (count) p = static_cast<T*>(dev_alloc(count * sizeof(T), st));
    }
    void release() {
        if (p) dev_free(p, s);
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
};

// ------------------------------------------------------------ tree layout
// Per-stage bookkeeping of the global split stages (one binary split per
// stage; level l's boxes are the segments of stage 2l).
struct SegInfo {      // one segment of one stage
    int32_t start;    // first point (global position)
    int32_t count;
    int32_t tile0;    // first tile (stage-local)
    int32_t ntile;
    int32_t child;    // stage-local index of the lower child in the next stage's arrays
    int32_t box;      // global box id if this stage is even (a level), else -1
    int32_t pad0, pad1;
};
struct TileInfo {
    int32_t seg;      // stage-local segment
    int32_t start;    // first point
    int32_t count;
    int32_t rank;     // tile index within its segment
    // the segment's fields the split kernels need, copied here so that a
    // tile's first load brings them (no second dependent load)
    int32_t seg_start, seg_count, tile0, child;
    int32_t range;    // segment whose bounding box sets the first-level histogram range
                      // (the parent; the segment itself at stage 0)
    int32_t flags;    // bit 0: the children are split by a global stage (this tile's
                      // partition histograms them)
};
struct LdsWork {      // one segment finished by the in-LDS split kernel
    int32_t start, count;
    int32_t stages;   // binary splits still to do
    int32_t stage0;   // stage of the segment
    int32_t j0;       // segment index at stage0 within its problem
    int32_t boxbase;  // global id of the problem's box 0 (root)
    int32_t pad0, pad1;
};
struct GeomJob {      // a box whose geometry comes from the bbox keys of a global stage
    int32_t box;
    int32_t seg;      // index into the stage's bbox key array (absolute, see keys_off)
};

struct PlanExtra;

struct TreeSchedule {
    // launch lists of plans on trees of this layout, by (precision, P2P knob)
    std::map<int, std::shared_ptr<PlanExtra>> plan_cache;
    int nprob = 0;
    int64_t n = 0;
    std::vector<int64_t> off;
    std::vector<int> L;
    std::vector<int64_t> pbox;      // first global box id per problem
    int64_t nbox = 0, nleaf = 0;
    int nstage = 0;                 // number of global stages
    std::vector<int> nseg, ntile;   // per global stage (active segments / tiles)
    std::vector<int64_t> seg_off, tile_off, keys_off;   // offsets into packed arrays
    std::vector<int> nkeys;         // bbox-key segments per stage (stage 0..nstage)
    int64_t total_seg = 0, total_tile = 0, total_keys = 0;
    std::vector<SegInfo> segs;
    std::vector<TileInfo> tiles;
    std::vector<int32_t> key_child_dummy;
    std::vector<LdsWork> lds;
    std::vector<GeomJob> geom;      // boxes whose geometry comes from global-stage keys
    std::vector<int64_t> geom_stage_off;  // geom jobs grouped by stage
    std::vector<TileInfo> copy_tiles;     // big-leaf problems: copy to final order
    std::vector<int32_t> box_start, box_count;
    std::vector<int32_t> box_parent;      // global id of the parent (-1 for roots)
    std::vector<int8_t> box_level;
    std::vector<int32_t> box_prob;
    int max_levels = 0;
    // device copies
    DBuf<SegInfo> d_segs;
    DBuf<TileInfo> d_tiles, d_copy;
    DBuf<LdsWork> d_lds;
    DBuf<GeomJob> d_geom;
    DBuf<int32_t> d_box_start, d_box_count, d_box_parent;
    DBuf<int32_t> d_box_prob;
    DBuf<int64_t> d_off;           // point offsets of the problems [nprob + 1]
    DBuf<int64_t> d_pbox;          // global id of every problem's root box [nprob]
    DBuf<int8_t> d_box_level;
};

struct Tree {
    int device = 0;
    hipStream_t stream = nullptr;
    TreeSchedule* sched = nullptr;   // shared with the schedule cache
    std::shared_ptr<TreeSchedule> sched_ref;
    // points in tree order
    DBuf<double> x, y;
    DBuf<int32_t> perm;       // tree position -> global input index
    DBuf<int32_t> iperm;      // global input index -> tree position
    // per box (global id)
    DBuf<double> bbox;        // [nbox][4] xmin xmax ymin ymax
    DBuf<double> geom;        // [nbox][4] cx cy r rs (rs = scaling radius)
    DBuf<uint32_t> err;       // nonzero when a position is not finite (set by the build)
    double t_build_us = 0;
};

// ------------------------------------------------------------------ plans

struct Plan {
    Tree* tree = nullptr;
    PlanExtra* ex = nullptr;     // launch lists, shared by plans of the same tree layout
    std::shared_ptr<PlanExtra> ex_ref;
    int p = 0, precision = 0;
    double theta = 0;
    fmm_tuning tune{};
    // connectivity, per global box: [begin, count) into the id pools
    DBuf<int32_t> s_beg, s_cnt, w_beg, w_cnt;
    DBuf<int32_t> s_ids, w_ids;    // global box ids
    int64_t n_strong = 0, n_weak = 0;
    int64_t n_p2p_pairs = 0;
    bool totals_known = false;     // n_strong, n_weak, n_p2p_pairs summed
    hipStream_t list_stream = nullptr;
    // list build enqueued by fmm_plan and finished by the first call that
    // needs the lists (see plan_finalize)
    bool lists_pending = false, lists_direct = false, finalized = false;
    int final_code = 0;            // an error of the deferred part, repeated by later calls
    std::string final_msg;
    DBuf<long long> lt_totals;     // list totals and flags of the pending build
    int flag_slot = -1;            // pinned host word receiving the one-pass flags
    hipEvent_t ev_lists = nullptr; // recorded after that copy
    hipEvent_t ev_lists_k = nullptr;     // recorded after the list kernels (before the copy)
    hipEvent_t ev_spec = nullptr;  // after an evaluation enqueued ahead of the flags
    long long list_flag = -1;      // the flags read by build_lists_finish (-1: not read)
    hipEvent_t ev_tree = nullptr;  // the tree's work on the caller's stream, before the lists
    hipEvent_t ev_plan_done = nullptr;   // the plan's last device work (list stream)
    bool upward_done = false;      // the evaluation's upward pass is already enqueued
    bool split_p2p = false, split_m2l = false;   // some list may need work chunks
    // evaluation buffers
    DBuf<double> mtree;            // [N][2] strengths in tree order (FP64); with the tree's
                                   // positions, the sources of the near field
    DBuf<double> near;             // [N][2] P2P result, tree order
    DBuf<double> mlog;             // [N][2] real strengths of the logarithmic kernel as complex numbers
    DBuf<double> c0;               // [nbox] constant term of the logarithmic local expansions
    // near-field work split into source chunks (see balance.hip)
    DBuf<int32_t> nsrc;            // [nbox] sources in the strong list of every leaf
    struct Balance {
        DBuf<int32_t> icnt, ioff;  // per item: chunks, exclusive prefix (+ total)
        DBuf<int2> xitems;         // (item, chunk) for every chunk, grouped by launch class
        DBuf<double> partial;      // per chunk of a split item: kItemTargets x values
        DBuf<int64_t> d_cls;       // expanded offsets of the classes (device)
        std::vector<int64_t> cls;  // the same on the host, nclass + 1 entries
        DBuf<int32_t> bsum;        // scan workspace
        DBuf<int64_t> d_base;      // class starts in the item array
        std::vector<int64_t> h_base;
        int64_t total = 0;
        int vals = 0;              // values per target in the partial sums
        int32_t h32 = 0;           // host copy of a device total
    } bal, bal_adj, bal_m2l;
    DBuf<char> mpole, local;       // [nbox][p] complex coefficients (T)
    // adjoint buffers
    DBuf<double> gtree;            // conj(G_phi) in tree order
    DBuf<double> near_d;           // derivative sums of the adjoint P2P
    DBuf<char> amp, aloc;          // adjoint coefficient arrays
    bool have_forward = false;
    const double* last_m = nullptr;
    // timing
    double t_plan_us = 0;
    double t_up = 0, t_m2l = 0, t_l2l = 0, t_down = 0, t_p2p = 0, t_total = 0;
    // graph
    hipGraphExec_t graph = nullptr;
    const double* graph_m = nullptr;
    double* graph_phi = nullptr;
    hipStream_t gstream = nullptr;         // capture / replay stream of graph mode
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipStream_t nstream = nullptr;         // near-field stream of the device (shared, not owned)
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_top0 = nullptr, ev_top1 = nullptr;   // the top levels' far field on a third stream
};

// ---------------------------------------------------------- launchers
void build_tree_device(Tree& t, const double* z, hipStream_t s);
void update_positions_device(Tree& t, const double* z, hipStream_t s);
void build_lists_device(Plan& pl, hipStream_t s);
void build_lists_begin(Plan& pl, hipStream_t ls, hipStream_t as);
void build_lists_finish(Plan& pl);
void release_list_flag(Plan& pl);
// pinned host words for flags read back without stalling the stream
int flag_slot_acquire();
volatile long long* flag_slot_ptr(int slot);
void flag_slot_release(int slot);
void evaluate_upward(Plan& pl, const double* m, hipStream_t s);
double rel_err2_device(const double* a, const double* ref, int64_t n, hipStream_t s);
constexpr int kNearStream = 0, kListStream = 1, kTopStream = 2;
hipStream_t side_stream(int device, int which);
void plan_join(Plan& pl, hipStream_t s);
void plan_events(Plan& pl);
void plan_finalize(Plan& pl);
void plan_balance(Plan& pl, hipStream_t s);
void list_totals_device(Plan& pl, hipStream_t s);
// lists_ev/guard: an evaluation enqueued before the list flags are read.
// Its list-reading kernels wait for lists_ev and do nothing when the flag
// word *guard is non-zero (the lists then need a rebuild or work chunks).
void evaluate_device(Plan& pl, const double* m, double* phi, double* phi_near, double* phi_far,
                     hipStream_t s, hipEvent_t lists_ev = nullptr, const long long* guard = nullptr);
void field_device(Plan& pl, const double* m, double* phi, double* dphi, hipStream_t s);
void evaluate_points_device(Plan& pl, const double* m, const double* y, int64_t M, double* phi, double* dphi,
                            hipStream_t s);
// fmm_evaluate_static: the evaluation with its working buffers in the fixed
// device array of static_eval.hip, and the bytes of that array it needs
void evaluate_static(Plan& pl, const double* m, double* phi, hipStream_t s);
size_t static_eval_bytes(Plan& pl);
// the logarithmic potential u (real, input order) of real strengths q; mlog
// (2 N doubles: q as complex numbers in input order) and c0 (one double per
// box: the constant terms) are the plan's own buffers when mlog is NULL
void evaluate_log_device(Plan& pl, const double* q, double* u, hipStream_t s, double* mlog = nullptr,
                         double* c0 = nullptr);
// the gather of an evaluation (the strengths into tree order: with the
// tree's positions, the near field's sources), done by the P2M kernel as it
// reads every point of its leaves
struct GatherOut {
    const int32_t* perm;     // tree position -> input index
    const double2* m;        // strengths, input order
    double2* mtree;          // strengths, tree order
};
void adjoint_device(Plan& pl, const double* m, const double* gphi, double* gm, double* gz,
                    hipStream_t s);

TreeSchedule* make_schedule(const std::vector<int64_t>& off, const std::vector<int>& L);
void upload_schedule(TreeSchedule& sc, hipStream_t s);

}  // namespace fmm
