// host_stubs.cpp -- stand-ins for the library's device-side functions, so
// that the host part of the C ABI (argument validation, error reporting,
// handle bookkeeping, the autotuner) builds and runs under the sanitizers
// on a machine without a GPU.  Every stand-in reports a device error.
#include "../../paper_1311_1006_amd/csrc/fmm_internal.h"
#include "../../paper_1311_1006_amd/csrc/plan_extra.h"

namespace fmm {
[[noreturn]] static void no_device() { throw Error(FMM_EDEVICE, "no device in the host-only sanitizer build"); }
void plan_events(Plan&) { no_device(); }
hipStream_t side_stream(int, int) { no_device(); }
void field_device(Plan&, const double*, double*, double*, hipStream_t) { no_device(); }
void evaluate_points_device(Plan&, const double*, const double*, int64_t, double*, double*, hipStream_t) { no_device(); }
void plan_balance(Plan&, hipStream_t) { no_device(); }
TreeSchedule* make_schedule(const std::vector<int64_t>&, const std::vector<int>&) { no_device(); }
void adjoint_device(Plan&, const double*, const double*, double*, double*, hipStream_t) { no_device(); }
void evaluate_device(Plan&, const double*, double*, double*, double*, hipStream_t, hipEvent_t, const long long*)
{
    no_device();
}
void evaluate_upward(Plan&, const double*, hipStream_t) { no_device(); }
void evaluate_static(Plan&, const double*, double*, hipStream_t) { no_device(); }
size_t static_eval_bytes(Plan&) { no_device(); }
double rel_err2_device(const double*, const double*, int64_t, hipStream_t) { no_device(); }
void upload_schedule(TreeSchedule&, hipStream_t) { no_device(); }
void build_lists_begin(Plan&, hipStream_t, hipStream_t) { no_device(); }
void build_tree_device(Tree&, const double*, hipStream_t) { no_device(); }
void prepare_plan_host(Plan&, PlanExtra&, hipStream_t) { no_device(); }
void release_list_flag(Plan&) {}
void alloc_eval_buffers(Plan&, hipStream_t) { no_device(); }
void build_lists_finish(Plan&) { no_device(); }
void list_totals_device(Plan&, hipStream_t) { no_device(); }
void evaluate_log_device(Plan&, const double*, double*, hipStream_t, double*, double*) { no_device(); }
void update_positions_device(Tree&, const double*, hipStream_t) { no_device(); }
}  // namespace fmm
