// Instantiates the float64 fitness kernels of mt_kernels.h for the
// nine-parameter Tersoff form, one per coordination class.
#include <hip/hip_ext.h>

#include "mt_kernels.h"

namespace mt {

hipError_t launch_fit64f(int mc, dim3 g, dim3 b, size_t lds, hipStream_t st, const BArgs<double>& A,
                        hipEvent_t e0, hipEvent_t e1) {
    if (A.resid) return launch_fitr64(mc, 1, g, b, lds, st, A, e0, e1);
    switch (mc) {
        case 4: hipExtLaunchKernelGGL((k_batched<double, MODE_FIT, 4, true>), g, b, lds, st, e0, e1, 0, A); break;
        case 16: hipExtLaunchKernelGGL((k_batched<double, MODE_FIT, 16, true>), g, b, lds, st, e0, e1, 0, A); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mt
