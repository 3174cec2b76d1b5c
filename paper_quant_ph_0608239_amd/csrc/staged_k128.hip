// Full- and half-buffer staged pass kernels for complex128 states (instantiated here, launched from staged.hip).
#include "qsim_internal.h"
#include "staged_kernels.h"

namespace qsim {
namespace staged {

int launch_pass_c128(int form, int log_e, int log_t, const PassLaunch &a)
{
    const int v = log_e * 16 + log_t;
    if (form == QSIM_STAGED_HALF) {
        switch (v) {
        case 4 * 16 + 6: launch_half<double, 4, 6, 3>(a); break;
        case 4 * 16 + 7: launch_half<double, 4, 7, 3>(a); break;
        case 4 * 16 + 8: launch_half<double, 4, 8, 3>(a); break;
        default: return set_error(QSIM_EINVAL, "staged: no half-buffer kernel for this block shape");
        }
        return QSIM_OK;
    }
    switch (v) {
    case 3 * 16 + 7: launch_full<double, 3, 7, 4>(a); break;
    case 3 * 16 + 8: launch_full<double, 3, 8, 4>(a); break;
    case 3 * 16 + 9: launch_full<double, 3, 9, 3>(a); break;
    case 4 * 16 + 6: launch_full<double, 4, 6, 2>(a); break;
    case 4 * 16 + 7: launch_full<double, 4, 7, 2>(a); break;
    case 4 * 16 + 8: launch_full<double, 4, 8, 2>(a); break;
    case 4 * 16 + 9: launch_full<double, 4, 9, 2>(a); break;  // 13 resident qubits, one workgroup per CU
    default: return set_error(QSIM_EINVAL, "staged: no kernel for this block shape");
    }
    return QSIM_OK;
}

}  // namespace staged
}  // namespace qsim
