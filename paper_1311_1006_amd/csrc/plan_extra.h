// plan_extra.h -- per-plan launch lists (host + device), internal.
#pragma once
#include <map>

#include "fmm_internal.h"

namespace fmm {

struct P2PClass {
    int tg, sub;        // targets per lane, lane subgroups
    int64_t off, n;     // range in the item array
};

struct PlanExtra {
    std::vector<std::vector<int32_t>> level_boxes;  // global ids per level (all problems)
    std::vector<int64_t> level_boxes_off;
    DBuf<int32_t> d_level_boxes;                    // concatenated per level
    DBuf<int32_t> leaves;                           // global ids of all leaves
    int leaf_max = 0;                               // largest leaf population
    bool leaf_l2l_in_l2p = false;                   // every problem has the same N_levels >= 2: the
                                                    // L2L into the leaves runs inside L2P
    bool leaf_m2m_in_p2m = false;                   // ... and no leaf holds more than 16 points: the
                                                    // M2M of the leaves' parents runs inside P2M
    bool gather_in_p2m = false;                     // the leaves hold every point: P2M does the gather
    int cap_strong = 0, cap_weak = 0;               // per-box list capacities of the one-pass build
    bool levelwise_only = false;                    // a frontier overflowed on this layout
    int64_t pool_strong = 0, pool_weak = 0;        // id pool sizes for the next compact build
    bool compact_only = false;                      // fixed capacities would need too much memory
    DBuf<double> binom;                             // binomial table C(n, k), n, k < 64
    std::vector<std::vector<int32_t>> m2m_boxes;   // non-leaf boxes per level
    std::vector<int64_t> m2m_off;
    DBuf<int32_t> d_m2m, child0;
    DBuf<char> p2p_items;
    std::vector<P2PClass> p2p_class;
    DBuf<char> adj_items;                           // adjoint P2P work items
    std::vector<P2PClass> adj_class;
};

inline PlanExtra* extra(Plan& pl) { return pl.ex; }

void prepare_plan_host(Plan& pl, PlanExtra& ex, hipStream_t s);
void alloc_eval_buffers(Plan& pl, hipStream_t s);
void prepare_adjoint_items(Plan& pl, PlanExtra& ex, const std::vector<int32_t>& leaves, hipStream_t s);

}  // namespace fmm
