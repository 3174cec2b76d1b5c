// LDS-staged passes (placeholder until the staged kernels land).
#include "qsim_internal.h"

namespace qsim {
struct StagedPlan {
    int dummy;
};
int staged_build(int, int, const std::vector<qsim_gate> &, int, StagedPlan **out, qsim_plan_info *)
{
    *out = nullptr;
    return set_error(QSIM_EUNSUPPORTED, "staged plans are not built yet");
}
int staged_execute(StagedPlan *, qsim_state *) { return set_error(QSIM_EUNSUPPORTED, "staged plans are not built yet"); }
int staged_execute_timed(StagedPlan *, qsim_state *, double *, int32_t *, int32_t *)
{
    return set_error(QSIM_EUNSUPPORTED, "staged plans are not built yet");
}
void staged_free(StagedPlan *p) { delete p; }
}  // namespace qsim
