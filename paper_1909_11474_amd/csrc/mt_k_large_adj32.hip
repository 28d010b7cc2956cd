// Instantiates the float two-pass fitness-gradient kernels of mt_kernels.h
// (force residuals, dual passes) for both potential forms.
#include "mt_kernels.h"

namespace mt {

template <int MC, bool Full>
static hipError_t large_adj(dim3 g, dim3 b, hipStream_t st, const BArgs<float>& A, const LArgs& L,
                            float* abuf) {
    hipLaunchKernelGGL((k_large_residual<float>), g, b, 0, st, A, L, abuf);
    hipLaunchKernelGGL((k_large_adjoint<float, MC, Full>), g, b, 0, st, A, L, (float const*)abuf);
    return hipGetLastError();
}

hipError_t launch_large_adj32(int mc, int full, dim3 g, dim3 b, hipStream_t st, const BArgs<float>& Afit,
                              const BArgs<float>& Aadj, const LArgs& L, float* abuf) {
    const hipError_t e = launch_large32(mc, MODE_STAGE, full, g, b, st, Afit, L);
    if (e != hipSuccess) return e;
    if (mc == 4) return full ? large_adj<4, true>(g, b, st, Aadj, L, abuf) : large_adj<4, false>(g, b, st, Aadj, L, abuf);
    if (mc == 16) return full ? large_adj<16, true>(g, b, st, Aadj, L, abuf) : large_adj<16, false>(g, b, st, Aadj, L, abuf);
    return hipErrorInvalidValue;
}

}  // namespace mt
