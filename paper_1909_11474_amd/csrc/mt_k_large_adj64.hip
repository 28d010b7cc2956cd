// Instantiates the double two-pass fitness-gradient kernels of mt_kernels.h
// (force residuals, dual passes) for the minimal potential; the Tersoff
// form's are in mt_k_tf_large_adj64.hip.
#include "mt_kernels.h"

namespace mt {

template <int MC>
static hipError_t large_adj(dim3 g, dim3 b, hipStream_t st, const BArgs<double>& A, const LArgs& L,
                            double* abuf) {
    hipLaunchKernelGGL((k_large_residual<double>), g, b, 0, st, A, L, abuf);
    hipLaunchKernelGGL((k_large_adjoint<double, MC, false>), g, b, 0, st, A, L, (double const*)abuf);
    return hipGetLastError();
}

hipError_t launch_large_adj64(int mc, int full, dim3 g, dim3 b, hipStream_t st, const BArgs<double>& Afit,
                              const BArgs<double>& Aadj, const LArgs& L, double* abuf) {
    const hipError_t e = launch_large64(mc, MODE_STAGE, full, g, b, st, Afit, L);
    if (e != hipSuccess) return e;
    if (full) return launch_large_adj64f(mc, g, b, st, Aadj, L, abuf);
    if (mc == 4) return large_adj<4>(g, b, st, Aadj, L, abuf);
    if (mc == 16) return large_adj<16>(g, b, st, Aadj, L, abuf);
    return hipErrorInvalidValue;
}

}  // namespace mt
