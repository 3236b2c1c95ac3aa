// plan_extra.h -- per-plan launch lists (host + device), internal.
#pragma once
#include "fmm_internal.h"

namespace fmm {

struct P2PClass {
    int ns, r;          // source splits, targets per lane
    int64_t off, n;     // range in the item array
};

struct PlanExtra {
    std::vector<std::vector<int32_t>> m2m_boxes;   // non-leaf boxes per level
    std::vector<int64_t> m2m_off;
    DBuf<int32_t> d_m2m, child0, all_boxes;
    DBuf<char> p2p_items;
    std::vector<P2PClass> p2p_class;
};

inline PlanExtra* extra(Plan& pl) { return pl.ex; }

void prepare_plan_host(Plan& pl, PlanExtra& ex, hipStream_t s);
void alloc_eval_buffers(Plan& pl, hipStream_t s);

}  // namespace fmm
