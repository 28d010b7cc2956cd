// Instantiates the two-pass large-structure kernels of mt_kernels.h.
#include <type_traits>

#include "mt_kernels.h"

namespace mt {

template <typename S, bool E64, bool Full>
static hipError_t launch_large_site(int mc, dim3 g, dim3 b, hipStream_t st, const BArgs<S>& A,
                                    const LArgs& L) {
    switch (mc) {
        case 4: hipLaunchKernelGGL((k_large_site<S, 4, E64, Full>), g, b, 0, st, A, L); break;
        case 16: hipLaunchKernelGGL((k_large_site<S, 16, E64, Full>), g, b, 0, st, A, L); break;
        default: return hipErrorInvalidValue;
    }
    return hipSuccess;
}

template <typename S, bool Full>
static hipError_t launch_large_form(int mc, int mode, dim3 g, dim3 b, hipStream_t st,
                                    const BArgs<S>& A, const LArgs& L) {
    // float arithmetic evaluates the energy terms in float64 (both modes:
    // the fitness compares per-atom energies at the 1e-6 eV level)
    (void)mode;
    constexpr bool kF32 = std::is_same<S, float>::value;
    return launch_large_site<S, kF32, Full>(mc, g, b, st, A, L);
}

template <typename S>
static hipError_t launch_large_pair(int mc, int mode, int full, dim3 g, dim3 b, hipStream_t st,
                                    const BArgs<S>& A, const LArgs& L) {
    const hipError_t e = full ? launch_large_form<S, true>(mc, mode, g, b, st, A, L)
                              : launch_large_form<S, false>(mc, mode, g, b, st, A, L);
    if (e != hipSuccess) return e;
    if (mode == MODE_STAGE) return hipGetLastError();
    if (mc == 4) {
        if (mode == MODE_FIT) hipLaunchKernelGGL((k_large_gather<S, MODE_FIT, 4>), g, b, 0, st, A, L);
        else hipLaunchKernelGGL((k_large_gather<S, MODE_EVAL, 4>), g, b, 0, st, A, L);
    } else {
        if (mode == MODE_FIT) hipLaunchKernelGGL((k_large_gather<S, MODE_FIT, 16>), g, b, 0, st, A, L);
        else hipLaunchKernelGGL((k_large_gather<S, MODE_EVAL, 16>), g, b, 0, st, A, L);
    }
    return hipGetLastError();
}

hipError_t launch_large32(int mc, int mode, int full, dim3 g, dim3 b, hipStream_t st,
                          const BArgs<float>& A, const LArgs& L) {
    return launch_large_pair<float>(mc, mode, full, g, b, st, A, L);
}

hipError_t launch_large64(int mc, int mode, int full, dim3 g, dim3 b, hipStream_t st,
                          const BArgs<double>& A, const LArgs& L) {
    return launch_large_pair<double>(mc, mode, full, g, b, st, A, L);
}

}  // namespace mt
