// Instantiates the two-pass large-structure kernels of mt_kernels.h.
#include "mt_kernels.h"

namespace mt {

template <typename S>
static hipError_t launch_large_pair(int mc, int mode, dim3 g, dim3 b, hipStream_t st,
                                    const BArgs<S>& A, const LArgs& L) {
    switch (mc) {
        case 4: hipLaunchKernelGGL((k_large_site<S, 4>), g, b, 0, st, A, L); break;
        case 16: hipLaunchKernelGGL((k_large_site<S, 16>), g, b, 0, st, A, L); break;
        default: return hipErrorInvalidValue;
    }
    if (mode == MODE_FIT) hipLaunchKernelGGL((k_large_gather<S, MODE_FIT>), g, b, 0, st, A, L);
    else hipLaunchKernelGGL((k_large_gather<S, MODE_EVAL>), g, b, 0, st, A, L);
    return hipGetLastError();
}

hipError_t launch_large32(int mc, int mode, dim3 g, dim3 b, hipStream_t st, const BArgs<float>& A,
                          const LArgs& L) {
    return launch_large_pair<float>(mc, mode, g, b, st, A, L);
}

hipError_t launch_large64(int mc, int mode, dim3 g, dim3 b, hipStream_t st, const BArgs<double>& A,
                          const LArgs& L) {
    return launch_large_pair<double>(mc, mode, g, b, st, A, L);
}

}  // namespace mt
