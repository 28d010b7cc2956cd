// Instantiates the float64 adjoint (parameter-gradient) kernels of mt_kernels.h
// for the nine-parameter Tersoff form, one per coordination class.
#include <hip/hip_ext.h>

#include "mt_kernels.h"

namespace mt {

hipError_t launch_adj64f(int mc, dim3 g, dim3 b, size_t lds, hipStream_t st, const BArgs<double>& A,
                         hipEvent_t e0, hipEvent_t e1) {
    switch (mc) {
        case 4: hipExtLaunchKernelGGL((k_adjoint<double, 4, true>), g, b, lds, st, e0, e1, 0, A); break;
        case 12: hipExtLaunchKernelGGL((k_adjoint<double, 12, true>), g, b, lds, st, e0, e1, 0, A); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mt
