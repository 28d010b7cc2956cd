// Instantiates the float32 fitness kernel of mt_kernels.h for the M <= 4
// coordination class (the other classes are in mt_k_fit32.hip).
#include <hip/hip_ext.h>

#include "mt_kernels.h"

namespace mt {

hipError_t launch_fit32_m4(dim3 g, dim3 b, size_t lds, hipStream_t st, const BArgs<float>& A,
                           hipEvent_t e0, hipEvent_t e1) {
    hipExtLaunchKernelGGL((k_batched<float, MODE_FIT, 4>), g, b, lds, st, e0, e1, 0, A);
    return hipGetLastError();
}

}  // namespace mt
