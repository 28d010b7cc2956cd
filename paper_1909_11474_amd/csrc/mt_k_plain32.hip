// Instantiates the float32 plain-schedule kernels of mt_kernels.h (one launch per
// candidate and structure), one per coordination class of the batched families.
#include "mt_kernels.h"

namespace mt {

hipError_t launch_plain32(int mode, bool full, int mc, dim3 b, size_t lds, hipStream_t st,
                          const BArgs<float>& A) {
    if (full) return launch_plain32f(mode, mc, b, lds, st, A);
    const dim3 g(1);
    if (mode == MODE_FIT) {
        switch (mc) {
            case 4: hipLaunchKernelGGL((k_plain<float, MODE_FIT, 4>), g, b, lds, st, A); break;
            case 6: hipLaunchKernelGGL((k_plain<float, MODE_FIT, 6>), g, b, lds, st, A); break;
            case 8: hipLaunchKernelGGL((k_plain<float, MODE_FIT, 8>), g, b, lds, st, A); break;
            case 12: hipLaunchKernelGGL((k_plain<float, MODE_FIT, 12>), g, b, lds, st, A); break;
            case 16: hipLaunchKernelGGL((k_plain<float, MODE_FIT, 16>), g, b, lds, st, A); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (mc) {
            case 4: hipLaunchKernelGGL((k_plain<float, MODE_EVAL, 4>), g, b, lds, st, A); break;
            case 8: hipLaunchKernelGGL((k_plain<float, MODE_EVAL, 8>), g, b, lds, st, A); break;
            case 16: hipLaunchKernelGGL((k_plain<float, MODE_EVAL, 16>), g, b, lds, st, A); break;
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

}  // namespace mt
