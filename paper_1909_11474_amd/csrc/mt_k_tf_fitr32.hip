// Instantiates the float fitness kernels that also write the force residuals
// (the gradient's fitness call) for the Tersoff form of mt_kernels.h.
#include <hip/hip_ext.h>

#include "mt_kernels.h"

namespace mt {

hipError_t launch_fitr32f(int mc, dim3 g, dim3 b, size_t lds, hipStream_t st, const BArgs<float>& A,
                          hipEvent_t e0, hipEvent_t e1) {
    switch (mc) {
        case 4: hipExtLaunchKernelGGL((k_batched<float, MODE_FIT, 4, true, true>), g, b, lds, st, e0, e1, 0, A); break;
        case 16: hipExtLaunchKernelGGL((k_batched<float, MODE_FIT, 16, true, true>), g, b, lds, st, e0, e1, 0, A); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mt
