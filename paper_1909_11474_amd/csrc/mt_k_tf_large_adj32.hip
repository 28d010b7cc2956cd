// Instantiates the float two-pass fitness-gradient kernels of mt_kernels.h
// (force residuals, dual passes) for the Tersoff form.
#include "mt_kernels.h"

namespace mt {

template <int MC>
static hipError_t large_adj(dim3 g, dim3 b, hipStream_t st, const BArgs<float>& A, const LArgs& L,
                            float* abuf) {
    hipLaunchKernelGGL((k_large_residual<float>), g, b, 0, st, A, L, abuf);
    hipLaunchKernelGGL((k_large_adjoint<float, MC, true>), g, b, 0, st, A, L, (float const*)abuf);
    return hipGetLastError();
}

hipError_t launch_large_adj32f(int mc, dim3 g, dim3 b, hipStream_t st, const BArgs<float>& A,
                               const LArgs& L, float* abuf) {
    if (mc == 4) return large_adj<4>(g, b, st, A, L, abuf);
    if (mc == 16) return large_adj<16>(g, b, st, A, L, abuf);
    return hipErrorInvalidValue;
}

}  // namespace mt
