// adjoint.hip -- placeholder until the transposed chain lands.
#include "fmm_internal.h"

namespace fmm {
void adjoint_device(Plan&, const double*, const double*, double*, double*, hipStream_t)
{
    throw Error(FMM_ESTATE, "fmm_evaluate_adjoint is not available in this build");
}
}  // namespace fmm
