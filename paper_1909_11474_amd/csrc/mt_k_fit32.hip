// Instantiates the float32 fitness kernels of mt_kernels.h, one per coordination class.
#include <hip/hip_ext.h>

#include "mt_kernels.h"

namespace mt {

// The M <= 4 class instance, in its own unit (mt_k_fit32_m4.hip) so that it
// can be compiled with its own code-generation flags.
hipError_t launch_fit32_m4(dim3 g, dim3 b, size_t lds, hipStream_t st, const BArgs<float>& A,
                           hipEvent_t e0, hipEvent_t e1);

hipError_t launch_fit32(int mc, dim3 g, dim3 b, size_t lds, hipStream_t st, const BArgs<float>& A,
                      hipEvent_t e0, hipEvent_t e1) {
    if (A.resid) return launch_fitr32(mc, 0, g, b, lds, st, A, e0, e1);
    switch (mc) {
        case 4: return launch_fit32_m4(g, b, lds, st, A, e0, e1);
        case 6: hipExtLaunchKernelGGL((k_batched<float, MODE_FIT, 6>), g, b, lds, st, e0, e1, 0, A); break;
        case 8: hipExtLaunchKernelGGL((k_batched<float, MODE_FIT, 8>), g, b, lds, st, e0, e1, 0, A); break;
        case 12: hipExtLaunchKernelGGL((k_batched<float, MODE_FIT, 12>), g, b, lds, st, e0, e1, 0, A); break;
        case 16: hipExtLaunchKernelGGL((k_batched<float, MODE_FIT, 16>), g, b, lds, st, e0, e1, 0, A); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mt
