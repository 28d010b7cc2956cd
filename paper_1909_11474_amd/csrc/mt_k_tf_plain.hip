// Instantiates the plain-schedule kernels of mt_kernels.h (one launch per
// candidate and structure) for the nine-parameter Tersoff form.
#include "mt_kernels.h"

namespace mt {

template <typename S>
static hipError_t launch_plain_tf(int mode, int mc, dim3 b, size_t lds, hipStream_t st,
                                  const BArgs<S>& A) {
    const dim3 g(1);
    if (mode == MODE_FIT) {
        switch (mc) {
            case 4: hipLaunchKernelGGL((k_plain<S, MODE_FIT, 4, true>), g, b, lds, st, A); break;
            case 16: hipLaunchKernelGGL((k_plain<S, MODE_FIT, 16, true>), g, b, lds, st, A); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (mc) {
            case 4: hipLaunchKernelGGL((k_plain<S, MODE_EVAL, 4, true>), g, b, lds, st, A); break;
            case 16: hipLaunchKernelGGL((k_plain<S, MODE_EVAL, 16, true>), g, b, lds, st, A); break;
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_plain32f(int mode, int mc, dim3 b, size_t lds, hipStream_t st, const BArgs<float>& A) {
    return launch_plain_tf<float>(mode, mc, b, lds, st, A);
}

hipError_t launch_plain64f(int mode, int mc, dim3 b, size_t lds, hipStream_t st, const BArgs<double>& A) {
    return launch_plain_tf<double>(mode, mc, b, lds, st, A);
}

}  // namespace mt
