// tuner.cpp -- online autotuner after Sec. 4.2 (Algorithm 4, "AT3b": directed
// walk with varying step size and cost estimation), over the integer knobs
// N_levels, P2P source split and M2L batch.
//
// What is kept from the paper:
//   * a move is tried, then accepted or rejected on the timings that follow;
//   * noise: a configuration is judged by the minimum time over a short
//     window of iterations (the problem is assumed to drift slowly);
//   * a rejected move reverses the walking direction of its knob;
//   * cost capping for N_levels: a rejected N_levels move adds its extra time
//     to upcost/downcost (each direction has its own budget), basetime sums
//     the iterations whose move was not rejected, and the next move in that
//     direction is scheduled
//       uptime     = (upcost + cost) / cap - basetime
//       upinterval = uptime * i / basetime
//     (run time still needed before another misstep of the same cost keeps
//     the accumulated tuning cost below cap * run time, converted into
//     iterations with the mean iteration time basetime / i);
//   * both directions due at once: the one that became due first moves.
// The theta step of AT2/AT3b is not used: theta is fixed by the accuracy
// target here, and the third knob pair (P2P split, M2L batch) takes the role
// of the second walking parameter, with the AT2 direction reversal.
#include <algorithm>
#include <cmath>
#include <limits>
#include <memory>
#include <string>
#include <vector>

#include "../../include/fmm.h"

namespace {

const int kSplits[] = {1, 2, 4};
const int kBatches[] = {4, 8, 16};

template <size_t N>
int index_of(const int (&v)[N], int x)
{
    for (size_t i = 0; i < N; ++i)
        if (v[i] == x) return (int)i;
    return -1;
}

enum Move { kNone = 0, kUp, kDown, kSplit, kBatch };

}  // namespace

struct fmm_tuner_s {
    fmm_tuner_config cfg;
    fmm_tuner_params cur, prev;
    Move pending = kNone;
    int64_t i = 0;                 // iterations observed
    double basetime = 0.0;         // accumulated time of iterations whose move was not rejected
    double runtime = 0.0;          // all iterations
    double upcost = 0.0, downcost = 0.0, knobcost = 0.0;
    double next_up = 0.0, next_down = 0.0, next_knob = 0.0;
    int split_dir = 1, batch_dir = 1, knob_turn = 0;
    std::vector<double> win;
    double ref = std::numeric_limits<double>::infinity();   // judged time of the accepted config
    double cost_total = 0.0;
};

static thread_local std::string g_tuner_err;

extern "C" {

int fmm_tuner_create(const fmm_tuner_config* cfg, fmm_tuner_t* out)
{
    if (!cfg || !out) return FMM_EINVAL;
    *out = nullptr;
    const fmm_tuner_config& c = *cfg;
    if (c.min_levels < 1 || c.max_levels < c.min_levels || c.init.n_levels < c.min_levels ||
        c.init.n_levels > c.max_levels || !(c.cap > 0.0) || c.window < 1 || c.knob_interval < 1)
        return FMM_EINVAL;
    if (index_of(kSplits, c.init.p2p_split) < 0 || index_of(kBatches, c.init.m2l_batch) < 0) return FMM_EINVAL;
    auto t = std::make_unique<fmm_tuner_s>();
    t->cfg = c;
    t->cur = t->prev = c.init;
    // first N_levels moves once the first window has been judged
    t->next_up = t->next_down = c.window;
    t->next_knob = c.window + c.knob_interval;
    *out = t.release();
    return FMM_OK;
}

int fmm_tuner_next(fmm_tuner_t tu, fmm_tuner_params* out)
{
    if (!tu || !out) return FMM_EINVAL;
    *out = tu->cur;
    return FMM_OK;
}

static void schedule_after_reject(fmm_tuner_s& t, double cost, bool up)
{
    double& acc = up ? t.upcost : t.downcost;
    acc += cost;
    double base = std::max(t.basetime, 1e-30);
    double uptime = (acc + cost) / t.cfg.cap - base;
    double interval = uptime * (double)t.i / base;
    interval = std::max(interval, (double)t.cfg.window);
    (up ? t.next_up : t.next_down) = (double)t.i + interval;
}

int fmm_tuner_observe(fmm_tuner_t tu, double seconds)
{
    if (!tu || !(seconds >= 0.0)) return FMM_EINVAL;
    fmm_tuner_s& t = *tu;
    ++t.i;
    t.runtime += seconds;
    t.win.push_back(seconds);
    if ((int)t.win.size() < t.cfg.window) return FMM_OK;
    double m = *std::min_element(t.win.begin(), t.win.end());
    double spent = 0.0;
    for (double w : t.win) spent += w;
    t.win.clear();
    if (t.pending != kNone) {
        if (m > t.ref) {
            // reject: the extra time of this window is the cost of the misstep
            double cost = (m - t.ref) * t.cfg.window;
            t.cost_total += std::max(0.0, spent - t.ref * t.cfg.window);
            if (t.pending == kUp) schedule_after_reject(t, cost, true);
            else if (t.pending == kDown) schedule_after_reject(t, cost, false);
            else if (t.pending == kSplit) t.split_dir = -t.split_dir;
            else t.batch_dir = -t.batch_dir;
            t.cur = t.prev;
        } else {
            t.ref = m;
            t.basetime += spent;
        }
        t.pending = kNone;
        return FMM_OK;
    }
    t.basetime += spent;
    t.ref = m;   // steady state: follow the drifting time of the current configuration
    // choose the next move
    const double i = (double)t.i;
    bool up_ok = t.cur.n_levels + 1 <= t.cfg.max_levels && i >= t.next_up;
    bool down_ok = t.cur.n_levels - 1 >= t.cfg.min_levels && i >= t.next_down;
    if (up_ok && down_ok) {
        if (t.next_up <= t.next_down) down_ok = false; else up_ok = false;
    }
    t.prev = t.cur;
    if (up_ok) {
        t.cur.n_levels += 1;
        t.pending = kUp;
        t.next_up = i + t.cfg.window;      // rescheduled by the outcome
    } else if (down_ok) {
        t.cur.n_levels -= 1;
        t.pending = kDown;
        t.next_down = i + t.cfg.window;
    } else if (i >= t.next_knob) {
        t.next_knob = i + t.cfg.knob_interval;
        for (int tries = 0; tries < 2 && t.pending == kNone; ++tries) {
            if ((t.knob_turn++ & 1) == 0) {
                int k = index_of(kSplits, t.cur.p2p_split) + t.split_dir;
                if (k >= 0 && k < 3) { t.cur.p2p_split = kSplits[k]; t.pending = kSplit; }
                else t.split_dir = -t.split_dir;
            } else {
                int k = index_of(kBatches, t.cur.m2l_batch) + t.batch_dir;
                if (k >= 0 && k < 3) { t.cur.m2l_batch = kBatches[k]; t.pending = kBatch; }
                else t.batch_dir = -t.batch_dir;
            }
        }
    }
    return FMM_OK;
}

int fmm_tuner_best(fmm_tuner_t tu, fmm_tuner_params* best, double* cost_s, double* run_s)
{
    if (!tu) return FMM_EINVAL;
    if (best) *best = tu->pending == kNone ? tu->cur : tu->prev;
    if (cost_s) *cost_s = tu->cost_total;
    if (run_s) *run_s = tu->runtime;
    return FMM_OK;
}

void fmm_tuner_destroy(fmm_tuner_t tu) { delete tu; }

}  // extern "C"
