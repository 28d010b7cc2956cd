// Instantiates the float64 plain-schedule kernels of mt_kernels.h (one launch per
// candidate and structure), one per coordination class of the batched families.
#include "mt_kernels.h"

namespace mt {

hipError_t launch_plain64(int mode, bool full, int mc, dim3 b, size_t lds, hipStream_t st,
                          const BArgs<double>& A) {
    if (full) return launch_plain64f(mode, mc, b, lds, st, A);
    const dim3 g(1);
    if (mode == MODE_FIT) {
        switch (mc) {
            case 4: hipLaunchKernelGGL((k_plain<double, MODE_FIT, 4>), g, b, lds, st, A); break;
            case 16: hipLaunchKernelGGL((k_plain<double, MODE_FIT, 16>), g, b, lds, st, A); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (mc) {
            case 4: hipLaunchKernelGGL((k_plain<double, MODE_EVAL, 4>), g, b, lds, st, A); break;
            case 16: hipLaunchKernelGGL((k_plain<double, MODE_EVAL, 16>), g, b, lds, st, A); break;
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

}  // namespace mt
