// Instantiates the float two-pass fitness-gradient kernels of mt_kernels.h
// (force residuals, dual passes) for the minimal potential; the Tersoff
// form's are in mt_k_tf_large_adj32.hip.
#include "mt_kernels.h"

namespace mt {

template <int MC>
static hipError_t large_adj(dim3 g, dim3 b, hipStream_t st, const BArgs<float>& A, const LArgs& L,
                            float* abuf) {
    hipLaunchKernelGGL((k_large_residual<float>), g, b, 0, st, A, L, abuf);
    hipLaunchKernelGGL((k_large_adjoint<float, MC, false>), g, b, 0, st, A, L, (float const*)abuf);
    return hipGetLastError();
}

hipError_t launch_large_adj32(int mc, int full, dim3 g, dim3 b, hipStream_t st, const BArgs<float>& Afit,
                              const BArgs<float>& Aadj, const LArgs& L, float* abuf) {
    const hipError_t e = launch_large32(mc, MODE_STAGE, full, g, b, st, Afit, L);
    if (e != hipSuccess) return e;
    if (full) return launch_large_adj32f(mc, g, b, st, Aadj, L, abuf);
    if (mc == 4) return large_adj<4>(g, b, st, Aadj, L, abuf);
    if (mc == 16) return large_adj<16>(g, b, st, Aadj, L, abuf);
    return hipErrorInvalidValue;
}

}  // namespace mt
