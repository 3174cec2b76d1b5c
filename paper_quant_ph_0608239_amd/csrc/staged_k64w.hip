// Wave-split staged pass kernels for complex64 states (instantiated here, launched from staged.hip).
#include "qsim_internal.h"
#include "staged_kernels.h"

namespace qsim {
namespace staged {

int launch_wave_c64(int log_e, int log_t, const PassLaunch &a)
{
    switch (log_e * 16 + log_t) {
    case 5 * 16 + 7: launch_wave<float, 5, 7, 4>(a); break;
    case 5 * 16 + 8: launch_wave<float, 5, 8, 4>(a); break;
    default: return set_error(QSIM_EINVAL, "staged: no wave-split kernel for this block shape");
    }
    return QSIM_OK;
}

}  // namespace staged
}  // namespace qsim
