// Instantiates the double two-pass fitness-gradient kernels of mt_kernels.h
// (force residuals, dual passes) for the Tersoff form.
#include "mt_kernels.h"

namespace mt {

template <int MC>
static hipError_t large_adj(dim3 g, dim3 b, hipStream_t st, const BArgs<double>& A, const LArgs& L,
                            double* abuf) {
    hipLaunchKernelGGL((k_large_residual<double>), g, b, 0, st, A, L, abuf);
    hipLaunchKernelGGL((k_large_adjoint<double, MC, true>), g, b, 0, st, A, L, (double const*)abuf);
    return hipGetLastError();
}

hipError_t launch_large_adj64f(int mc, dim3 g, dim3 b, hipStream_t st, const BArgs<double>& A,
                               const LArgs& L, double* abuf) {
    if (mc == 4) return large_adj<4>(g, b, st, A, L, abuf);
    if (mc == 16) return large_adj<16>(g, b, st, A, L, abuf);
    return hipErrorInvalidValue;
}

}  // namespace mt
