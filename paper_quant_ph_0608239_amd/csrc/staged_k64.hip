// Full- and half-buffer staged pass kernels for complex64 states (instantiated here, launched from staged.hip).
#include "qsim_internal.h"
#include "staged_kernels.h"

namespace qsim {
namespace staged {

int launch_pass_c64(int form, int log_e, int log_t, const PassLaunch &a)
{
    const int v = log_e * 16 + log_t;
    if (form == QSIM_STAGED_HALF) {
        switch (v) {
        case 5 * 16 + 6: launch_half<float, 5, 6, 3>(a); break;
        case 5 * 16 + 7: launch_half<float, 5, 7, 3>(a); break;
        case 5 * 16 + 8: launch_half<float, 5, 8, 3>(a); break;
        default: return set_error(QSIM_EINVAL, "staged: no half-buffer kernel for this block shape");
        }
        return QSIM_OK;
    }
    switch (v) {
    case 4 * 16 + 7: launch_full<float, 4, 7, 3>(a); break;
    case 4 * 16 + 8: launch_full<float, 4, 8, 3>(a); break;
    case 4 * 16 + 9: launch_full<float, 4, 9, 2>(a); break;
    case 4 * 16 + 10: launch_full<float, 4, 10, 4>(a); break;  // 14 resident qubits, 1024 threads
    case 5 * 16 + 6: launch_full<float, 5, 6, 1>(a); break;
    case 5 * 16 + 7: launch_full<float, 5, 7, 1>(a); break;
    case 5 * 16 + 8: launch_full<float, 5, 8, 1>(a); break;
    case 5 * 16 + 9: launch_full<float, 5, 9, 1>(a); break;    // 14 resident qubits, one workgroup per CU
    default: return set_error(QSIM_EINVAL, "staged: no kernel for this block shape");
    }
    return QSIM_OK;
}

}  // namespace staged
}  // namespace qsim
