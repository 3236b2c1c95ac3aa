// api.cpp -- the C ABI of include/fmm.h: argument validation, handle
// lifetimes, a stream-ordered caching device allocator and the cache of tree
// schedules (they depend only on the problem sizes and level counts).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>

#include "fmm_internal.h"
#include "plan_extra.h"

namespace fmm {

// -------------------------------------------------------------- allocator
// Blocks are never returned to the driver while the process lives (hipFree
// synchronises the device); a freed block is reused for a request of the
// same size class on the same stream only.  A block is freed in stream order
// on the stream it was allocated on (work of other streams on it has been
// joined into that stream), so a reuse there needs no wait at all; a request
// on another stream takes a fresh block instead of waiting for the old
// stream (which would stall the host behind unrelated work queued there).
namespace {
struct Block {
    void* p;
    size_t cls;
    hipStream_t s;
};
std::mutex g_mu;
std::multimap<std::pair<hipStream_t, size_t>, Block> g_free;
std::map<void*, size_t> g_cls;
int64_t g_live = 0;         // blocks handed out and not returned
int64_t g_fail_after = -1;  // allocations left before an injected failure (-1: none)

size_t size_class(size_t b)
{
    size_t c = 256;
    while (c < b) c <<= 1;
    return c;
}
}  // namespace

void* dev_alloc(size_t bytes, hipStream_t s)
{
    size_t c = size_class(bytes);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (g_fail_after == 0) {
            g_fail_after = -1;
            throw Error(FMM_ENOMEM, "device allocation of " + std::to_string(c) + " bytes failed (injected)");
        }
        if (g_fail_after > 0) --g_fail_after;
        auto it = g_free.find({s, c});
        if (it != g_free.end()) {
            Block b = it->second;
            g_free.erase(it);
            ++g_live;
            return b.p;
        }
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, c);
    if (e != hipSuccess) {
        // release cached blocks and retry once
        std::vector<void*> drop;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            for (auto& kv : g_free) drop.push_back(kv.second.p);
            g_free.clear();
        }
        (void)hipDeviceSynchronize();
        for (void* q : drop) {
            (void)hipFree(q);
            std::lock_guard<std::mutex> lk(g_mu);
            g_cls.erase(q);
        }
        (void)hipGetLastError();
        e = hipMalloc(&p, c);
        if (e != hipSuccess) throw Error(FMM_ENOMEM, "device allocation of " + std::to_string(c) + " bytes failed");
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_cls[p] = c;
    ++g_live;
    return p;
}

void dev_free(void* p, hipStream_t s)
{
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cls.find(p);
    if (it == g_cls.end()) return;
    g_free.insert({{s, it->second}, Block{p, it->second, s}});
    --g_live;
}

// ------------------------------------------------------ pinned flag words
namespace {
constexpr int kFlagSlots = 4096;
std::mutex g_flag_mu;
long long* g_flags = nullptr;       // pinned, allocated once
std::vector<int> g_flag_free;
}  // namespace

int flag_slot_acquire()
{
    std::lock_guard<std::mutex> lk(g_flag_mu);
    if (!g_flags) {
        void* p = nullptr;
        FMM_HIP(hipHostMalloc(&p, sizeof(long long) * kFlagSlots, hipHostMallocDefault));
        g_flags = static_cast<long long*>(p);
        for (int i = kFlagSlots - 1; i >= 0; --i) g_flag_free.push_back(i);
    }
    if (g_flag_free.empty()) return -1;
    const int s = g_flag_free.back();
    g_flag_free.pop_back();
    return s;
}

volatile long long* flag_slot_ptr(int slot) { return g_flags + slot; }

void flag_slot_release(int slot)
{
    if (slot < 0) return;
    std::lock_guard<std::mutex> lk(g_flag_mu);
    g_flag_free.push_back(slot);
}

// --------------------------------------------------------- schedule cache
namespace {
struct SchedKey {     // schedules hold device arrays: one per device
    int device;
    std::vector<int64_t> off;
    std::vector<int> L;
    bool operator<(const SchedKey& o) const
    {
        if (device != o.device) return device < o.device;
        return off != o.off ? off < o.off : L < o.L;
    }
};
}  // namespace

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

static int fail(const std::exception& e)
{
    if (auto* fe = dynamic_cast<const Error*>(&e)) {
        g_err = fe->what();
        return fe->code;
    }
    g_err = e.what();
    return FMM_EDEVICE;
}

template <class F>
static int guarded(F&& f)
{
    try {
        g_err.clear();
        f();
        return FMM_OK;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return FMM_ENOMEM;
    } catch (const std::exception& e) {
        return fail(e);
    }
}

static void check_device_state()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error(FMM_EDEVICE, std::string("earlier device error: ") + hipGetErrorString(e));
}

}  // namespace fmm

using namespace fmm;

struct fmm_tree_s {
    Tree t;
    std::vector<int64_t> off;
    std::vector<int> L;
};
struct fmm_plan_s {
    Plan pl;
    fmm_tree_s* tree;
};

extern "C" {

const char* fmm_last_error(void) { return g_err.c_str(); }

int fmm_debug_fail_alloc(int64_t after)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_fail_after = after < 0 ? -1 : after;
    return FMM_OK;
}

int fmm_debug_live_blocks(int64_t* live)
{
    if (!live) {
        g_err = "live is NULL";
        return FMM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    *live = g_live;
    return FMM_OK;
}

int fmm_p_from_tol(double tol, double theta)
{
    if (!(tol > 0.0 && tol < 1.0) || !(theta > 0.0 && theta < 1.0)) {
        g_err = "fmm_p_from_tol: need 0 < tol < 1 and 0 < theta < 1";
        return FMM_EINVAL;
    }
    // p ~ log TOL / log theta (Sec. 2.3); the constant 17 and the geometric
    // tail (1 - theta) reproduce Table 4.1
    return (int)std::ceil(std::log(17.0 * tol * (1.0 - theta)) / std::log(theta));
}

int fmm_choose_order(fmm_tree_t t, const double* m, double theta, double tol, int p_lo, int p_hi,
                     void* stream, int* p_out, double* err_out)
{
    return guarded([&] {
        FMM_REQUIRE(t && m && p_out, "NULL argument");
        *p_out = -1;
        FMM_REQUIRE(1 <= p_lo && p_lo <= p_hi && p_hi <= 48, "need 1 <= p_lo <= p_hi <= 48");
        FMM_REQUIRE(theta > 0.0 && theta < 1.0, "theta must be in (0, 1)");
        FMM_REQUIRE(tol > 0.0 && tol < 1.0, "tol must be in (0, 1)");
        check_device_state();
        hipStream_t s = (hipStream_t)stream;
        const int64_t n = t->t.sched->n;
        DBuf<double> ref, phi;
        ref.alloc(2 * (size_t)n, s);
        phi.alloc(2 * (size_t)n, s);
        // one evaluation through the public calls (a plan per order)
        auto run = [&](int p, int precision, double* out) {
            fmm_plan_t pl = nullptr;
            int rc = fmm_plan(t, p, theta, precision, nullptr, stream, &pl);
            if (rc != FMM_OK) throw Error(rc, g_err);
            rc = fmm_evaluate(pl, m, out, stream);
            const std::string msg = g_err;
            fmm_plan_destroy(pl);
            if (rc != FMM_OK) throw Error(rc, msg);
        };
        // the reference order: 32 terms for the usual range, else 16 more
        // than the highest order tried (at most 64)
        const int pref = p_hi <= 24 ? 32 : std::min(kMaxP, p_hi + 16);
        run(pref, FMM_FP64, ref.p);
        double e[2] = {0.0, 0.0};
        for (int p = p_lo; p <= p_hi; ++p) {
            run(p, FMM_FP64, phi.p);
            e[0] = rel_err2_device(phi.p, ref.p, n, s);
            run(p, FMM_MIXED, phi.p);
            e[1] = rel_err2_device(phi.p, ref.p, n, s);
            if (e[0] <= tol && e[1] <= tol) {
                *p_out = p;
                break;
            }
        }
        if (err_out) { err_out[0] = e[0]; err_out[1] = e[1]; }
    });
}

int fmm_build_tree(const double* z, const int64_t* offsets, int nprob, const int* n_levels, void* stream,
                   fmm_tree_t* out)
{
    return guarded([&] {
        FMM_REQUIRE(out, "out is NULL");
        *out = nullptr;
        FMM_REQUIRE(nprob >= 1, "nprob must be >= 1");
        FMM_REQUIRE(offsets && n_levels, "offsets / n_levels are NULL");
        FMM_REQUIRE(offsets[0] == 0, "offsets[0] must be 0");
        std::vector<int64_t> off(offsets, offsets + nprob + 1);
        std::vector<int> L(n_levels, n_levels + nprob);
        for (int b = 0; b < nprob; ++b) {
            int64_t nb = off[b + 1] - off[b];
            FMM_REQUIRE(nb >= 1, "every problem needs at least one point");
            FMM_REQUIRE(L[b] >= 1 && L[b] <= kMaxLevels, "n_levels out of range [1, 16]");
            FMM_REQUIRE((int64_t(1) << (2 * (L[b] - 1))) <= nb, "4^(n_levels-1) must not exceed the point count");
            FMM_REQUIRE(nb <= 100000000, "at most 1e8 points per problem");
        }
        FMM_REQUIRE(off[nprob] < (int64_t(1) << 31) - 1, "at most 2^31-2 points in total");
        FMM_REQUIRE(z != nullptr, "z is NULL");
        check_device_state();
        hipStream_t s = (hipStream_t)stream;
        int device = 0;
        FMM_HIP(hipGetDevice(&device));
        static std::mutex mu;
        static std::map<SchedKey, std::shared_ptr<TreeSchedule>> cache;
        std::shared_ptr<TreeSchedule> sched;
        {
            std::lock_guard<std::mutex> lk(mu);
            SchedKey k{device, off, L};
            auto it = cache.find(k);
            if (it != cache.end()) sched = it->second;
        }
        if (!sched) {
            sched.reset(make_schedule(off, L));
            upload_schedule(*sched, s);
            std::lock_guard<std::mutex> lk(mu);
            if (cache.size() > 16) cache.clear();
            cache[SchedKey{device, off, L}] = sched;
        }
        auto tr = std::make_unique<fmm_tree_s>();
        tr->off = off;
        tr->L = L;
        tr->t.stream = s;
        tr->t.device = device;   // the device of the tree, its plans and their side streams
        // the schedule is shared with the cache: keep a reference in the tree
        tr->t.sched = sched.get();
        tr->t.sched_ref = sched;
        build_tree_device(tr->t, z, s);
        *out = tr.release();
    });
}

int fmm_tree_update_positions(fmm_tree_t t, const double* z, void* stream)
{
    return guarded([&] {
        FMM_REQUIRE(t && z, "NULL argument");
        check_device_state();
        update_positions_device(t->t, z, (hipStream_t)stream);
    });
}

void fmm_tree_destroy(fmm_tree_t t) { delete t; }

int fmm_plan(fmm_tree_t t, int p, double theta, int precision, const fmm_tuning* tune, void* stream,
             fmm_plan_t* out)
{
    return guarded([&] {
        FMM_REQUIRE(out, "out is NULL");
        *out = nullptr;
        FMM_REQUIRE(t, "tree is NULL");
        FMM_REQUIRE(p >= 1 && p <= kMaxP, "p must be in [1, 64]");
        FMM_REQUIRE(theta > 0.0 && theta < 1.0, "theta must be in (0, 1)");
        FMM_REQUIRE(precision == FMM_FP64 || precision == FMM_MIXED, "unknown precision");
        fmm_tuning tn{};
        if (tune) tn = *tune;
        FMM_REQUIRE(tn.p2p_split == 0 || tn.p2p_split == 1 || tn.p2p_split == 2 || tn.p2p_split == 4,
                    "p2p_split must be 0, 1, 2 or 4");
        FMM_REQUIRE(tn.m2l_batch == 0 || tn.m2l_batch == 1 || tn.m2l_batch == 2 || tn.m2l_batch == 4 ||
                        tn.m2l_batch == 8 || tn.m2l_batch == 16,
                    "m2l_batch must be 0, 1, 2, 4, 8 or 16");
        FMM_REQUIRE(tn.smooth_delta >= 0.0 && std::isfinite(tn.smooth_delta), "smooth_delta must be >= 0 and finite");
        FMM_REQUIRE(tn.p2p_targets == 0 || tn.p2p_targets == 1 || tn.p2p_targets == 2 || tn.p2p_targets == 4 ||
                        tn.p2p_targets == 8 || tn.p2p_targets == 16,
                    "p2p_targets must be 0, 1, 2, 4, 8 or 16");
        FMM_REQUIRE(!(precision == FMM_FP64 && tn.p2p_targets > 8), "p2p_targets is at most 8 in FP64");
        FMM_REQUIRE(tn.p2p_targets == 0 || p2p_shape_ok(tn.p2p_targets, tn.p2p_split),
                    "no P2P shape for this p2p_targets and p2p_split");
        FMM_REQUIRE(tn.p2p_src_tile == 0 || tn.p2p_src_tile == 64 || tn.p2p_src_tile == 128 || tn.p2p_src_tile == 256,
                    "p2p_src_tile must be 0, 64, 128 or 256");
        check_device_state();
        hipStream_t s = (hipStream_t)stream;
        // a plan that fails half-way is released by fmm_plan_destroy, which
        // waits for list work already enqueued before its buffers are reused
        std::unique_ptr<fmm_plan_s, void (*)(fmm_plan_s*)> pp(new fmm_plan_s, fmm_plan_destroy);
        pp->tree = t;
        Plan& pl = pp->pl;
        pl.tree = &t->t;
        pl.p = p;
        pl.theta = theta;
        pl.precision = precision;
        pl.tune = tn;
        {
            TreeSchedule& sc = *t->t.sched;
            int key = (precision * 64 + tn.p2p_split) * 32 + tn.p2p_targets;   // the launch classes
            auto it = sc.plan_cache.find(key);
            if (it != sc.plan_cache.end()) {
                pl.ex_ref = it->second;
            } else {
                pl.ex_ref = std::make_shared<PlanExtra>();
                pl.ex = pl.ex_ref.get();
                prepare_plan_host(pl, *pl.ex, s);
                sc.plan_cache[key] = pl.ex_ref;
            }
            pl.ex = pl.ex_ref.get();
        }
        // the lists are enqueued on the device's list stream after the tree's
        // work on `s`, so they run beside what the caller enqueues next (the
        // upward pass); their flags are read by the first call that needs
        // them (plan_finalize), so the host returns meanwhile
        alloc_eval_buffers(pl, s);
        plan_events(pl);
        hipStream_t ls = side_stream(pl.tree->device, kListStream);
        FMM_HIP(hipEventCreateWithFlags(&pl.ev_tree, hipEventDisableTiming));
        FMM_HIP(hipEventRecord(pl.ev_tree, s));
        FMM_HIP(hipStreamWaitEvent(ls, pl.ev_tree, 0));
        build_lists_begin(pl, ls, s);
        *out = pp.release();
    });
}

}  // extern "C"

namespace fmm {
// Finish a plan's list build (flags, fallbacks) and its work balancing, once.
// An error of this deferred part is kept and repeated by every later call.
void plan_finalize(Plan& P)
{
    if (P.finalized) return;
    if (P.final_code) throw Error(P.final_code, P.final_msg);
    try {
        build_lists_finish(P);
        plan_balance(P, P.list_stream);
    } catch (const Error& e) {
        P.final_code = e.code;
        P.final_msg = e.what();
        throw;
    }
    P.lt_totals.release();
    // the plan's last device work on the list stream: consumers wait for it
    if (!P.ev_plan_done) FMM_HIP(hipEventCreateWithFlags(&P.ev_plan_done, hipEventDisableTiming));
    FMM_HIP(hipEventRecord(P.ev_plan_done, P.list_stream));
    P.finalized = true;
}

// order `s` after the plan's list and work-chunk kernels
void plan_join(Plan& P, hipStream_t s)
{
    if (P.ev_plan_done) FMM_HIP(hipStreamWaitEvent(s, P.ev_plan_done, 0));
}
}  // namespace fmm

extern "C" {

void fmm_plan_destroy(fmm_plan_t pl)
{
    if (!pl) return;
    Plan& P = pl->pl;
    if (P.graph) (void)hipGraphExecDestroy(P.graph);
    if (P.gstream) {
        (void)hipStreamSynchronize(P.gstream);
        (void)hipStreamDestroy(P.gstream);
        (void)hipEventDestroy(P.ev_in);
        (void)hipEventDestroy(P.ev_out);
    }
    // the near-field stream is shared; work on it is joined into the
    // evaluation stream, so the plan's buffers are released in stream order
    if (P.ev_fork) (void)hipEventDestroy(P.ev_fork);
    if (P.ev_join) (void)hipEventDestroy(P.ev_join);
    if (P.ev_top0) (void)hipEventDestroy(P.ev_top0);
    if (P.ev_top1) (void)hipEventDestroy(P.ev_top1);
    release_list_flag(P);
    // list work still in flight (a plan never used, or one whose creation
    // failed after its list kernels were enqueued) finishes before its
    // buffers go back to the pool
    if (P.list_stream && !P.finalized) (void)hipStreamSynchronize(P.list_stream);
    if (P.ev_tree) (void)hipEventDestroy(P.ev_tree);
    if (P.ev_lists_k) (void)hipEventDestroy(P.ev_lists_k);
    if (P.ev_spec) (void)hipEventDestroy(P.ev_spec);
    if (P.ev_plan_done) (void)hipEventDestroy(P.ev_plan_done);
    delete pl;
}

int fmm_evaluate(fmm_plan_t pl, const double* m, double* phi, void* stream)
{
    return guarded([&] {
        FMM_REQUIRE(pl && m && phi, "NULL argument");
        check_device_state();
        hipStream_t s = (hipStream_t)stream;
        Plan& P = pl->pl;
        const bool pending = !P.finalized && !P.final_code && !(P.tune.flags & (FMM_FLAG_GRAPH | FMM_FLAG_PHASE_TIMING));
        if (pending && P.lists_pending && P.lists_direct && P.flag_slot >= 0) {
            // The one-pass lists are still in flight.  The whole evaluation
            // is enqueued now for the usual outcome (no flag: every list fit
            // and none needs work chunks); its list-reading kernels wait for
            // the lists and read the device flag word first, doing nothing
            // when it is set.  The host reads the same flags meanwhile; only
            // when one is set does it enqueue the evaluation again, after
            // the rebuild or the work chunks.
            P.split_p2p = P.split_m2l = false;
            plan_balance(P, s);                 // unsplit tables: host only
            evaluate_device(P, m, phi, nullptr, nullptr, s, P.ev_lists_k, P.lt_totals.p + 2);
            if (!P.ev_spec) FMM_HIP(hipEventCreateWithFlags(&P.ev_spec, hipEventDisableTiming));
            FMM_HIP(hipEventRecord(P.ev_spec, s));
            plan_finalize(P);
            if (P.list_flag == 0) {
                P.last_m = m;
                return;
            }
        } else if (pending) {
            // lists built by several passes: the upward pass (which needs no
            // lists) goes first, so the device works while the flags arrive
            evaluate_upward(P, m, s);
        }
        plan_finalize(P);
        if (P.tune.flags & FMM_FLAG_GRAPH) {
            // capture and replay on a plan-owned stream (the legacy null stream
            // cannot be captured), ordered after the caller's stream by events
            if (!P.gstream) {
                FMM_HIP(hipStreamCreateWithFlags(&P.gstream, hipStreamNonBlocking));
                FMM_HIP(hipEventCreateWithFlags(&P.ev_in, hipEventDisableTiming));
                FMM_HIP(hipEventCreateWithFlags(&P.ev_out, hipEventDisableTiming));
            }
            FMM_HIP(hipEventRecord(P.ev_in, s));
            FMM_HIP(hipStreamWaitEvent(P.gstream, P.ev_in, 0));
            plan_join(P, P.gstream);
            if (!P.graph || P.graph_m != m || P.graph_phi != phi) {
                if (P.graph) { FMM_HIP(hipGraphExecDestroy(P.graph)); P.graph = nullptr; }
                hipGraph_t g = nullptr;
                FMM_HIP(hipStreamBeginCapture(P.gstream, hipStreamCaptureModeThreadLocal));
                int saved = P.tune.flags;
                P.tune.flags &= ~FMM_FLAG_PHASE_TIMING;
                try {
                    evaluate_device(P, m, phi, nullptr, nullptr, P.gstream);
                } catch (...) {
                    P.tune.flags = saved;
                    hipGraph_t dead = nullptr;
                    (void)hipStreamEndCapture(P.gstream, &dead);
                    if (dead) (void)hipGraphDestroy(dead);
                    throw;
                }
                P.tune.flags = saved;
                FMM_HIP(hipStreamEndCapture(P.gstream, &g));
                hipError_t e = hipGraphInstantiate(&P.graph, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) throw Error(FMM_EDEVICE, "hipGraphInstantiate failed");
                P.graph_m = m;
                P.graph_phi = phi;
            }
            FMM_HIP(hipGraphLaunch(P.graph, P.gstream));
            FMM_HIP(hipEventRecord(P.ev_out, P.gstream));
            FMM_HIP(hipStreamWaitEvent(s, P.ev_out, 0));
            P.have_forward = true;
        } else {
            plan_join(P, s);
            evaluate_device(P, m, phi, nullptr, nullptr, s);
        }
        P.last_m = m;
    });
}

int fmm_evaluate_static(fmm_plan_t pl, const double* m, double* phi, void* stream)
{
    return guarded([&] {
        FMM_REQUIRE(pl && m && phi, "NULL argument");
        check_device_state();
        hipStream_t s = (hipStream_t)stream;
        plan_join(pl->pl, s);
        evaluate_static(pl->pl, m, phi, s);
    });
}

int fmm_evaluate_parts(fmm_plan_t pl, const double* m, double* phi_near, double* phi_far, void* stream)
{
    return guarded([&] {
        FMM_REQUIRE(pl && m, "NULL argument");
        check_device_state();
        plan_finalize(pl->pl);
        plan_join(pl->pl, (hipStream_t)stream);
        evaluate_device(pl->pl, m, nullptr, phi_near, phi_far, (hipStream_t)stream);
        pl->pl.last_m = m;
    });
}

int fmm_evaluate_points(fmm_plan_t pl, const double* m, const double* y, int64_t M, double* phi_y, double* dphi_y,
                        void* stream)
{
    return guarded([&] {
        FMM_REQUIRE(pl && m, "NULL argument");
        FMM_REQUIRE(M >= 0, "M must be >= 0");
        FMM_REQUIRE(M == 0 || (y && phi_y), "NULL points or output");
        FMM_REQUIRE(pl->pl.tune.smooth_delta == 0.0, "a smoothed near field is evaluated by fmm_evaluate only");
        check_device_state();
        plan_finalize(pl->pl);
        plan_join(pl->pl, (hipStream_t)stream);
        evaluate_points_device(pl->pl, m, y, M, phi_y, dphi_y, (hipStream_t)stream);
    });
}

int fmm_evaluate_field(fmm_plan_t pl, const double* m, double* phi, double* dphi, void* stream)
{
    return guarded([&] {
        FMM_REQUIRE(pl && m && phi && dphi, "NULL argument");
        FMM_REQUIRE(pl->pl.tune.smooth_delta == 0.0, "a smoothed near field is evaluated by fmm_evaluate only");
        check_device_state();
        hipStream_t s = (hipStream_t)stream;
        Plan& P = pl->pl;
        plan_finalize(P);
        plan_join(P, s);
        field_device(P, m, phi, dphi, s);
        P.last_m = m;
    });
}

int fmm_evaluate_log(fmm_plan_t pl, const double* q, double* u, void* stream)
{
    return guarded([&] {
        FMM_REQUIRE(pl && q && u, "NULL argument");
        FMM_REQUIRE(pl->pl.tune.smooth_delta == 0.0, "a smoothed near field has no logarithmic form");
        check_device_state();
        hipStream_t s = (hipStream_t)stream;
        Plan& P = pl->pl;
        plan_finalize(P);
        plan_join(P, s);
        evaluate_log_device(P, q, u, s);
    });
}

int fmm_evaluate_adjoint(fmm_plan_t pl, const double* m, const double* g_phi, double* g_m, double* g_z,
                         void* stream)
{
    return guarded([&] {
        FMM_REQUIRE(pl && m && g_phi, "NULL argument");
        if (!pl->pl.have_forward) throw Error(FMM_ESTATE, "fmm_evaluate_adjoint needs a preceding fmm_evaluate");
        FMM_REQUIRE(pl->pl.tune.smooth_delta == 0.0, "a smoothed near field is evaluated by fmm_evaluate only");
        check_device_state();
        plan_finalize(pl->pl);
        plan_join(pl->pl, (hipStream_t)stream);
        adjoint_device(pl->pl, m, g_phi, g_m, g_z, (hipStream_t)stream);
    });
}

int fmm_plan_stats(fmm_plan_t pl, fmm_stats* st)
{
    return guarded([&] {
        FMM_REQUIRE(pl && st, "NULL argument");
        Plan& P = pl->pl;
        TreeSchedule& sc = *P.tree->sched;
        plan_finalize(P);
        list_totals_device(P, P.list_stream);
        std::memset(st, 0, sizeof(*st));
        st->n_points = sc.n;
        st->n_boxes = sc.nbox;
        st->n_leaves = sc.nleaf;
        st->n_p2p_pairs = P.n_p2p_pairs;
        st->n_m2l_pairs = P.n_weak;
        st->n_strong_entries = P.n_strong;
        st->p = P.p;
        st->precision = P.precision;
        st->max_levels = sc.max_levels;
        st->nprob = sc.nprob;
        st->theta = P.theta;
        st->t_upward_us = P.t_up;
        st->t_m2l_us = P.t_m2l;
        st->t_l2l_us = P.t_l2l;
        st->t_p2p_us = P.t_p2p;
        st->t_downward_us = P.t_down;
        st->t_total_us = P.t_total;
        st->t_tree_us = P.tree->t_build_us;
        st->t_plan_us = P.t_plan_us;
        st->static_bytes = (int64_t)static_eval_bytes(P);
    });
}

int fmm_tree_layout(fmm_tree_t t, int prob, int* n_levels, int64_t* n_points, int64_t* n_boxes)
{
    return guarded([&] {
        FMM_REQUIRE(t, "NULL tree");
        FMM_REQUIRE(prob >= 0 && prob < (int)t->L.size(), "problem index out of range");
        if (n_levels) *n_levels = t->L[prob];
        if (n_points) *n_points = t->off[prob + 1] - t->off[prob];
        if (n_boxes) *n_boxes = nbox_levels(t->L[prob]);
    });
}

int fmm_tree_download(fmm_tree_t t, int prob, int64_t* perm, int64_t* range, double* geom, void* stream)
{
    return guarded([&] {
        FMM_REQUIRE(t, "NULL tree");
        FMM_REQUIRE(prob >= 0 && prob < (int)t->L.size(), "problem index out of range");
        hipStream_t s = (hipStream_t)stream;
        TreeSchedule& sc = *t->t.sched;
        int64_t o = t->off[prob], n = t->off[prob + 1] - o;
        int64_t nb = nbox_levels(t->L[prob]), b0 = sc.pbox[prob];
        std::vector<int32_t> pm(n);
        std::vector<double> bb(4 * nb), gm(4 * nb);
        FMM_HIP(hipMemcpyAsync(pm.data(), t->t.perm.p + o, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
        FMM_HIP(hipMemcpyAsync(bb.data(), t->t.bbox.p + 4 * b0, sizeof(double) * 4 * nb, hipMemcpyDeviceToHost, s));
        FMM_HIP(hipMemcpyAsync(gm.data(), t->t.geom.p + 4 * b0, sizeof(double) * 4 * nb, hipMemcpyDeviceToHost, s));
        uint32_t err = 0;
        FMM_HIP(hipMemcpyAsync(&err, t->t.err.p, sizeof(err), hipMemcpyDeviceToHost, s));
        FMM_HIP(hipStreamSynchronize(s));
        if (err) throw Error(FMM_EINVAL, "non-finite position");
        if (perm)
            for (int64_t i = 0; i < n; ++i) perm[i] = pm[i] - o;
        if (range)
            for (int64_t b = 0; b < nb; ++b) {
                range[2 * b] = sc.box_start[b0 + b] - o;
                range[2 * b + 1] = sc.box_count[b0 + b];
            }
        if (geom)
            for (int64_t b = 0; b < nb; ++b) {
                for (int c = 0; c < 4; ++c) geom[7 * b + c] = bb[4 * b + c];
                for (int c = 0; c < 3; ++c) geom[7 * b + 4 + c] = gm[4 * b + c];
            }
    });
}

static void list_host(fmm_plan_t pl, int prob, int level, int kind, std::vector<int32_t>& beg,
                      std::vector<int32_t>& cnt, std::vector<int32_t>& ids, hipStream_t s)
{
    Plan& P = pl->pl;
    TreeSchedule& sc = *P.tree->sched;
    FMM_REQUIRE(prob >= 0 && prob < sc.nprob, "problem index out of range");
    FMM_REQUIRE(level >= 0 && level < sc.L[prob], "level out of range");
    FMM_REQUIRE(kind == 0 || kind == 1, "kind must be 0 (strong) or 1 (weak)");
    int64_t nb = int64_t(1) << (2 * level);
    int64_t b0 = sc.pbox[prob] + level_base(level);
    plan_join(P, s);   // after the list kernels on the list stream
    beg.resize(nb);
    cnt.resize(nb);
    const int32_t* db = kind ? P.w_beg.p : P.s_beg.p;
    const int32_t* dc = kind ? P.w_cnt.p : P.s_cnt.p;
    FMM_HIP(hipMemcpyAsync(beg.data(), db + b0, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, s));
    FMM_HIP(hipMemcpyAsync(cnt.data(), dc + b0, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, s));
    FMM_HIP(hipStreamSynchronize(s));
    int64_t tot = 0;
    for (int64_t b = 0; b < nb; ++b) tot += cnt[b];
    ids.clear();
    ids.reserve(tot);
    const int32_t* di = kind ? P.w_ids.p : P.s_ids.p;
    // the lists of one level's boxes lie in one run of the pool, in box order
    // (packed, or at fixed per-box capacities)
    if (tot) {
        int64_t first = beg[0], last = 0;
        for (int64_t b = 0; b < nb; ++b) last = std::max<int64_t>(last, (int64_t)beg[b] + cnt[b]);
        std::vector<int32_t> run(last - first);
        FMM_HIP(hipMemcpyAsync(run.data(), di + first, sizeof(int32_t) * (last - first), hipMemcpyDeviceToHost, s));
        FMM_HIP(hipStreamSynchronize(s));
        for (int64_t b = 0; b < nb; ++b)
            for (int e = 0; e < cnt[b]; ++e) ids.push_back(run[beg[b] - first + e]);
    }
}

int fmm_plan_list_size(fmm_plan_t pl, int prob, int level, int kind, int64_t* n_entries)
{
    return guarded([&] {
        FMM_REQUIRE(pl && n_entries, "NULL argument");
        plan_finalize(pl->pl);
        std::vector<int32_t> b, c, ids;
        list_host(pl, prob, level, kind, b, c, ids, nullptr);
        *n_entries = (int64_t)ids.size();
    });
}

int fmm_plan_download_list(fmm_plan_t pl, int prob, int level, int kind, int64_t* off, int64_t* ids,
                           void* stream)
{
    return guarded([&] {
        FMM_REQUIRE(pl, "NULL plan");
        plan_finalize(pl->pl);
        std::vector<int32_t> b, c, id;
        list_host(pl, prob, level, kind, b, c, id, (hipStream_t)stream);
        TreeSchedule& sc = *pl->pl.tree->sched;
        int64_t base = sc.pbox[prob] + level_base(level);
        int64_t acc = 0;
        for (size_t i = 0; i < c.size(); ++i) {
            if (off) off[i] = acc;
            acc += c[i];
        }
        if (off) off[c.size()] = acc;
        if (ids)
            for (size_t i = 0; i < id.size(); ++i) ids[i] = id[i] - base;
    });
}

}  // extern "C"
