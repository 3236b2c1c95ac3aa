// tuner.cpp -- online autotuner after Sec. 4.2 (Algorithms 1, 2 and 4: AT1
// random walk, AT2 directed walk with Fibonacci step cycles, AT3b directed
// walk with cost estimation) over N_levels and theta, plus the P2P source
// split and the M2L batch as launch-shape knobs of the AT3b walk.
//
// What is kept from the paper:
//   * a move is tried, then accepted or rejected on the timings that follow;
//   * noise: a configuration is judged by the minimum time over a short
//     window of iterations (the problem is assumed to drift slowly);
//   * when several moves are due, N_levels moves first, then theta;
//   * AT2/AT3b: a rejected move reverses the walking direction of its
//     parameter; a rejected theta move also takes the next step length of a
//     cycle through the Fibonacci numbers, whose length grows by one each
//     time the cycle wraps, so that a walk held at an apparent optimum
//     probes ever farther on both sides;
//   * AT3b cost capping for N_levels: a rejected N_levels move adds its extra
//     time to upcost/downcost (each direction has its own budget), basetime
//     sums the iterations whose move was not rejected, and the next move in
//     that direction is scheduled
//       uptime     = (upcost + cost) / cap - basetime
//       upinterval = uptime * i / basetime
//     (run time still needed before another misstep of the same cost keeps
//     the accumulated tuning cost below cap * run time, converted into
//     iterations with the mean iteration time basetime / i);
//     both directions due at once: the one that became due first moves;
//   * AT1: moves at regular intervals in a random direction (SplitMix64).
// theta lives on the grid theta_min + k * theta_unit; with a tolerance the
// expansion order follows theta by the rule of Table 4.1, so that theta is a
// pure performance knob (Sec. 2.3).
#include <algorithm>
#include <cmath>
#include <iterator>
#include <limits>
#include <memory>
#include <string>
#include <vector>

#include "../../include/fmm.h"

namespace {

const int kSplits[] = {1, 2, 4};
const int kBatches[] = {1, 2, 4, 8, 16};

template <size_t N>
int index_of(const int (&v)[N], int x)
{
    for (size_t i = 0; i < N; ++i)
        if (v[i] == x) return (int)i;
    return -1;
}

enum Move { kNone = 0, kUp, kDown, kTheta, kSplit, kBatch };

// SplitMix64 (Steele, Lea and Flood, 2014): one 64-bit output per call
uint64_t splitmix64(uint64_t& s)
{
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// fib(1) = fib(2) = 1, fib(n) = fib(n-1) + fib(n-2)
int64_t fib(int n)
{
    int64_t a = 1, b = 1;
    for (int k = 2; k < n; ++k) {
        const int64_t c = a + b;
        a = b;
        b = c;
    }
    return n <= 2 ? 1 : b;
}

}  // namespace

struct fmm_tuner_s {
    fmm_tuner_config cfg;
    fmm_tuner_params cur, prev;
    Move pending = kNone;
    int64_t i = 0;                 // iterations observed
    double basetime = 0.0;         // accumulated time of iterations whose move was not rejected
    double runtime = 0.0;          // all iterations
    double upcost = 0.0, downcost = 0.0;
    double next_up = 0.0, next_down = 0.0, next_knob = 0.0, next_level = 0.0, next_theta = 0.0;
    int split_dir = 1, batch_dir = 1, knob_turn = 0;
    int nl_dir = 1;                // AT2 N_levels direction
    // theta on its grid: theta = theta_min + theta_k * theta_unit, 0 <= theta_k <= theta_kmax
    int theta_k = 0, theta_kmax = 0, prev_theta_k = 0;
    int theta_dir = 1, fibcount = 1, fiblength = 2;
    int64_t theta_step = 1;
    uint64_t rng = 0;
    std::vector<double> win;
    double ref = std::numeric_limits<double>::infinity();   // judged time of the accepted config
    double cost_total = 0.0;

    bool tunes_theta() const { return cfg.theta_interval > 0; }
    void set_theta_k(int k)
    {
        theta_k = k;
        cur.theta = cfg.theta_min + (double)k * cfg.theta_unit;
        if (cfg.tol > 0.0) cur.p = fmm_p_from_tol(cfg.tol, cur.theta);
    }
    bool randbit() { return (splitmix64(rng) >> 63) != 0; }
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
    if (c.algorithm != FMM_TUNER_AT3B && c.algorithm != FMM_TUNER_AT2 && c.algorithm != FMM_TUNER_AT1)
        return FMM_EINVAL;
    if (c.algorithm != FMM_TUNER_AT3B && c.level_interval < 1) return FMM_EINVAL;
    if (c.theta_interval < 0 || !(c.tol >= 0.0 && c.tol < 1.0) || c.init.p < 0) return FMM_EINVAL;
    auto t = std::make_unique<fmm_tuner_s>();
    t->cfg = c;
    t->cur = c.init;
    t->rng = c.seed;
    if (t->tunes_theta()) {
        if (!(c.theta_unit > 0.0) || !(c.theta_min > 0.0) || !(c.theta_max < 1.0) || !(c.theta_min <= c.theta_max) ||
            !(c.init.theta >= c.theta_min && c.init.theta <= c.theta_max) || c.fib_length < 2)
            return FMM_EINVAL;
        t->theta_kmax = (int)std::floor((c.theta_max - c.theta_min) / c.theta_unit + 1e-9);
        const int k0 = (int)std::lround((c.init.theta - c.theta_min) / c.theta_unit);
        t->fiblength = c.fib_length;
        t->set_theta_k(std::min(std::max(k0, 0), t->theta_kmax));
    } else if (c.tol > 0.0) {
        if (!(c.init.theta > 0.0 && c.init.theta < 1.0)) return FMM_EINVAL;
        t->cur.p = fmm_p_from_tol(c.tol, c.init.theta);
    }
    t->prev = t->cur;
    t->prev_theta_k = t->theta_k;
    // first moves once the first window has been judged
    t->next_up = t->next_down = t->next_level = t->next_theta = c.window;
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

// a rejected theta move (AT2, AT3b): next step of the Fibonacci cycle, the
// cycle one longer when it wraps, the direction reversed
static void theta_rejected(fmm_tuner_s& t)
{
    if (t.fibcount < t.fiblength) {
        t.theta_step = fib(t.fibcount++);
    } else {
        t.fibcount = 1;
        t.theta_step = fib(1);
        // a step wider than the grid only reaches its ends: stop growing there
        if (fib(t.fiblength) <= (int64_t)t.theta_kmax) ++t.fiblength;
    }
    t.theta_dir = -t.theta_dir;
}

static bool level_move(fmm_tuner_s& t, int dir, double i)
{
    const int L = t.cur.n_levels + dir;
    if (L < t.cfg.min_levels || L > t.cfg.max_levels) return false;
    t.cur.n_levels = L;
    t.pending = dir > 0 ? kUp : kDown;
    (void)i;
    return true;
}

static bool try_levels(fmm_tuner_s& t, double i)
{
    if (t.cfg.algorithm == FMM_TUNER_AT3B) {
        bool up_ok = t.cur.n_levels + 1 <= t.cfg.max_levels && i >= t.next_up;
        bool down_ok = t.cur.n_levels - 1 >= t.cfg.min_levels && i >= t.next_down;
        if (up_ok && down_ok) {
            if (t.next_up <= t.next_down) down_ok = false; else up_ok = false;
        }
        if (up_ok) {
            t.next_up = i + t.cfg.window;      // rescheduled by the outcome
            return level_move(t, 1, i);
        }
        if (down_ok) {
            t.next_down = i + t.cfg.window;
            return level_move(t, -1, i);
        }
        return false;
    }
    if (i < t.next_level) return false;
    t.next_level = i + t.cfg.level_interval;
    if (t.cfg.algorithm == FMM_TUNER_AT2) {
        if (level_move(t, t.nl_dir, i)) return true;
        t.nl_dir = -t.nl_dir;                  // at the end of the range: walk back
        return level_move(t, t.nl_dir, i);
    }
    const int dir = t.randbit() ? 1 : -1;      // AT1
    return level_move(t, dir, i) || level_move(t, -dir, i);
}

static bool try_theta(fmm_tuner_s& t, double i)
{
    if (!t.tunes_theta() || i < t.next_theta) return false;
    t.next_theta = i + t.cfg.theta_interval;
    int k;
    if (t.cfg.algorithm == FMM_TUNER_AT1) {
        const int dir = t.randbit() ? 1 : -1;
        k = t.theta_k + dir;
        if (k < 0 || k > t.theta_kmax) k = t.theta_k - dir;
    } else {
        int64_t kk = (int64_t)t.theta_k + t.theta_dir * t.theta_step;
        if (kk < 0 || kk > t.theta_kmax) {
            t.theta_dir = -t.theta_dir;        // at the end of the grid: walk back
            kk = (int64_t)t.theta_k + t.theta_dir * t.theta_step;
        }
        k = (int)std::min<int64_t>(std::max<int64_t>(kk, 0), t.theta_kmax);
    }
    if (k < 0 || k > t.theta_kmax || k == t.theta_k) return false;
    t.set_theta_k(k);
    t.pending = kTheta;
    return true;
}

static bool try_knobs(fmm_tuner_s& t, double i)
{
    if (t.cfg.algorithm != FMM_TUNER_AT3B || i < t.next_knob) return false;
    t.next_knob = i + t.cfg.knob_interval;
    for (int tries = 0; tries < 2 && t.pending == kNone; ++tries) {
        if ((t.knob_turn++ & 1) == 0) {
            int k = index_of(kSplits, t.cur.p2p_split) + t.split_dir;
            if (k >= 0 && k < (int)std::size(kSplits)) { t.cur.p2p_split = kSplits[k]; t.pending = kSplit; }
            else t.split_dir = -t.split_dir;
        } else {
            int k = index_of(kBatches, t.cur.m2l_batch) + t.batch_dir;
            if (k >= 0 && k < (int)std::size(kBatches)) { t.cur.m2l_batch = kBatches[k]; t.pending = kBatch; }
            else t.batch_dir = -t.batch_dir;
        }
    }
    return t.pending != kNone;
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
            const bool at3b = t.cfg.algorithm == FMM_TUNER_AT3B, at2 = t.cfg.algorithm == FMM_TUNER_AT2;
            if (t.pending == kUp || t.pending == kDown) {
                if (at3b) schedule_after_reject(t, cost, t.pending == kUp);
                else if (at2) t.nl_dir = -t.nl_dir;
            } else if (t.pending == kTheta) {
                if (!(t.cfg.algorithm == FMM_TUNER_AT1)) theta_rejected(t);
            } else if (t.pending == kSplit) {
                t.split_dir = -t.split_dir;
            } else {
                t.batch_dir = -t.batch_dir;
            }
            t.cur = t.prev;
            t.theta_k = t.prev_theta_k;
        } else {
            t.ref = m;
            t.basetime += spent;
        }
        t.pending = kNone;
        return FMM_OK;
    }
    t.basetime += spent;
    t.ref = m;   // steady state: follow the drifting time of the current configuration
    // the next move: N_levels, else theta, else a launch-shape knob
    const double i = (double)t.i;
    t.prev = t.cur;
    t.prev_theta_k = t.theta_k;
    if (!try_levels(t, i) && !try_theta(t, i)) try_knobs(t, i);
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
