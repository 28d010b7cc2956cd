// Molecular-dynamics kernels for the potential's main application (Sec. IV.C:
// equilibrium and driven MD of diamond Si): velocity-Verlet kicks and drifts,
// the homogeneous non-equilibrium driving force built from the per-atom
// virial, and deterministic kinetic-energy / momentum sums.
//
// Units: positions A, velocities A/fs, forces eV/A, masses u, time fs; a force
// F on a mass m accelerates by F / (m * 103.642691) A/fs^2 (1 u A^2/fs^2 =
// 103.642691 eV).  Arrays are SoA [3][N] float64 in the caller's atom order.
#include <hip/hip_runtime.h>

#include "mt_host.h"

namespace mt {
namespace {

constexpr double kAccel = 1.0 / 103.642691;

int blocks_for(int n) { return (n + 255) / 256; }

// v += dt_half (F_i + F_ext,i - <F_ext>) / m_i, with F_ext,i = W_i^T F_e
// (W_i row-major [9][N]) and <F_ext> = W^T F_e / N from the symmetric total
// virial (xx yy zz yz zx xy), so that the driving force adds no momentum.
__global__ __launch_bounds__(256) void k_kick(int N, double* __restrict__ vel,
                                              const double* __restrict__ force,
                                              const double* __restrict__ atom_virial,
                                              const double* __restrict__ virial6, double fe0,
                                              double fe1, double fe2,
                                              const double* __restrict__ inv_mass, double dt_half) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double f[3] = {force[i], force[(size_t)N + i], force[(size_t)2 * N + i]};
    if (atom_virial) {
        const double fe[3] = {fe0, fe1, fe2};
        double W[3][3];
        const double* w = virial6;
        W[0][0] = w[0]; W[1][1] = w[1]; W[2][2] = w[2];
        W[1][2] = W[2][1] = w[3]; W[2][0] = W[0][2] = w[4]; W[0][1] = W[1][0] = w[5];
        for (int b = 0; b < 3; ++b) {
            double ext = 0.0, mean = 0.0;
            for (int a = 0; a < 3; ++a) {
                ext += fe[a] * atom_virial[(size_t)(3 * a + b) * N + i];
                mean += fe[a] * W[a][b];
            }
            f[b] += ext - mean / N;
        }
    }
    const double s = dt_half * kAccel * inv_mass[i];
    for (int k = 0; k < 3; ++k) vel[(size_t)k * N + i] += s * f[k];
}

__global__ __launch_bounds__(256) void k_drift(int N, double* __restrict__ pos,
                                               const double* __restrict__ vel, double dt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    for (int k = 0; k < 3; ++k) pos[(size_t)k * N + i] += dt * vel[(size_t)k * N + i];
}

__global__ __launch_bounds__(256) void k_scale(int N, double* __restrict__ vel, double lambda) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    for (int k = 0; k < 3; ++k) vel[(size_t)k * N + i] *= lambda;
}

// Atoms per thread whose loads are issued together in the single-block
// reductions below (one memory latency per round instead of one per atom).
constexpr int kBatch = 8;

// One block: each thread sums a fixed strided subset (atoms t, t + 1024, ...
// in ascending order), then a fixed tree; the result depends only on N.
// out = [sum m v^2, sum m v_x, sum m v_y, sum m v_z].
__global__ __launch_bounds__(1024) void k_kinetic(int N, const double* __restrict__ vel,
                                                  const double* __restrict__ mass,
                                                  double* __restrict__ out) {
    __shared__ double sh[4][1024];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i0 = threadIdx.x; i0 < N; i0 += kBatch * blockDim.x) {
        double m[kBatch], vx[kBatch], vy[kBatch], vz[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const int i = i0 + b * blockDim.x;
            const bool in = i < N;
            m[b] = in ? mass[i] : 0.0;
            vx[b] = in ? vel[i] : 0.0;
            vy[b] = in ? vel[(size_t)N + i] : 0.0;
            vz[b] = in ? vel[(size_t)2 * N + i] : 0.0;
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            if (i0 + b * (int)blockDim.x >= N) break;
            a[0] += m[b] * (vx[b] * vx[b] + vy[b] * vy[b] + vz[b] * vz[b]);
            a[1] += m[b] * vx[b];
            a[2] += m[b] * vy[b];
            a[3] += m[b] * vz[b];
        }
    }
    for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = a[k];
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 4) out[threadIdx.x] = sh[threadIdx.x][0];
}

// out[0] = max_i |r_i - r0_i|^2 (one block, exact: max is order independent).
__global__ __launch_bounds__(1024) void k_max_disp(int N, const double* __restrict__ pos,
                                                   const double* __restrict__ ref,
                                                   double* __restrict__ out) {
    __shared__ double sh[1024];
    double a = 0.0;
    for (int i0 = threadIdx.x; i0 < N; i0 += kBatch * blockDim.x) {
        double d[kBatch][3];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const int i = i0 + b * blockDim.x;
            const bool in = i < N;
#pragma unroll
            for (int k = 0; k < 3; ++k)
                d[b][k] = in ? pos[(size_t)k * N + i] - ref[(size_t)k * N + i] : 0.0;
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const double d2 = d[b][0] * d[b][0] + d[b][1] * d[b][1] + d[b][2] * d[b][2];
            a = a > d2 ? a : d2;
        }
    }
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

}  // namespace
}  // namespace mt

using namespace mt;

extern "C" {

int mt_md_kick(int N, double* vel, const double* force, const double* atom_virial,
               const double* virial, const double* fe, const double* inv_mass, double dt_half,
               void* stream) {
    if (N <= 0) { set_error("N must be positive"); return MT_EINVAL; }
    if (!vel || !force || !inv_mass) { set_error("vel, force and inv_mass must not be NULL"); return MT_EINVAL; }
    if ((atom_virial != nullptr) != (fe != nullptr) || (atom_virial && !virial)) {
        set_error("the driving force needs fe, atom_virial and virial together");
        return MT_EINVAL;
    }
    const double f0 = fe ? fe[0] : 0.0, f1 = fe ? fe[1] : 0.0, f2 = fe ? fe[2] : 0.0;
    hipLaunchKernelGGL(k_kick, dim3(blocks_for(N)), dim3(256), 0, (hipStream_t)stream, N, vel,
                       force, atom_virial, virial, f0, f1, f2, inv_mass, dt_half);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? MT_OK : hip_fail(e, "k_kick");
}

int mt_md_drift(int N, double* pos, const double* vel, double dt, void* stream) {
    if (N <= 0 || !pos || !vel) { set_error("N must be positive, pos and vel not NULL"); return MT_EINVAL; }
    hipLaunchKernelGGL(k_drift, dim3(blocks_for(N)), dim3(256), 0, (hipStream_t)stream, N, pos, vel, dt);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? MT_OK : hip_fail(e, "k_drift");
}

int mt_md_scale(int N, double* vel, double lambda, void* stream) {
    if (N <= 0 || !vel) { set_error("N must be positive, vel not NULL"); return MT_EINVAL; }
    hipLaunchKernelGGL(k_scale, dim3(blocks_for(N)), dim3(256), 0, (hipStream_t)stream, N, vel, lambda);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? MT_OK : hip_fail(e, "k_scale");
}

int mt_md_max_disp(int N, const double* pos, const double* ref, double* out, void* stream) {
    if (N <= 0 || !pos || !ref || !out) { set_error("N must be positive, pointers not NULL"); return MT_EINVAL; }
    hipLaunchKernelGGL(k_max_disp, dim3(1), dim3(1024), 0, (hipStream_t)stream, N, pos, ref, out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? MT_OK : hip_fail(e, "k_max_disp");
}

int mt_md_kinetic(int N, const double* vel, const double* mass, double* out, void* stream) {
    if (N <= 0 || !vel || !mass || !out) { set_error("N must be positive, pointers not NULL"); return MT_EINVAL; }
    hipLaunchKernelGGL(k_kinetic, dim3(1), dim3(1024), 0, (hipStream_t)stream, N, vel, mass, out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? MT_OK : hip_fail(e, "k_kinetic");
}

}  // extern "C"
