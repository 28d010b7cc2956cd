// Evaluation kernels: parameter decode, the batched candidate x structure
// kernel, the one-launch-per-pair plain path, the two-pass kernels for large
// structures, the adjoint (parameter-gradient) kernel and the finalize kernels
// that turn per-slot partial sums into energies, virials, Z and dZ/dx.
//
// Batched kernel.  A work item is (structure s, candidates c0 .. c0+nc-1).  A
// block of B threads holds R = B / npad_s replicas of the structure (npad_s is
// the atom count rounded up to 8/16/32/64 or to a multiple of 64), one atom per
// thread; replica q evaluates candidates c0 + q, c0 + q + R, ...  The bond
// geometry of the thread's atom is loaded once per item into registers and
// reused for every candidate.  Forces need the other atom's bond gradient
// (F_i = sum_j G_ij - G_ji), exchanged through LDS with one barrier on each
// side.  Per-atom energy, virial and squared force residual are reduced in
// float64 over aligned lane groups with a transpose reduction and written to
// one partial-sum slot per (candidate, structure, wavefront); the finalize
// kernels add the slots in a fixed order, so results are deterministic.
//
// Atoms inside a structure are sorted by coordination, and each wavefront runs
// the variant compiled for its largest coordination, so control flow is
// uniform and padded bonds are rare.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <queue>
#include <vector>

#include "mt_host.h"
#include "mt_site.h"

namespace mt {

#define HIPCHECK(call)                                   \
    do {                                                 \
        hipError_t _e = (call);                          \
        if (_e != hipSuccess) return hip_fail(_e, #call); \
    } while (0)

// ---------------------------------------------------------------------------
// Parameter decode (Sec. II.B): x = [D0, alpha, r0, beta, n, h] with S = 2.
// ---------------------------------------------------------------------------
template <typename S>
__global__ void k_decode(int P, const double* __restrict__ x, S* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= P) return;
    double D0 = x[6 * c + 0], al = x[6 * c + 1], r0 = x[6 * c + 2];
    double be = x[6 * c + 3], n = x[6 * c + 4], h = x[6 * c + 5];
    bool ok = isfinite(D0) && isfinite(al) && isfinite(r0) && isfinite(be) && isfinite(n) &&
              isfinite(h) && D0 > 0.0 && al > 0.0 && n > 0.0 && be >= 0.0;
    if (!ok) {   // a harmless stand-in keeps the arithmetic finite; outputs become NaN
        D0 = 3.0; al = 1.4; r0 = 2.2; be = 0.3; n = 0.6; h = -0.6;
    }
    S* o = out + (size_t)kNParam * c;
    o[P_AL] = (S)(al * 1.4426950408889634);
    const S r0hi = (S)r0;
    o[P_R0HI] = r0hi;
    o[P_R0LO] = (S)(r0 - (double)r0hi);
    o[P_D0] = (S)D0;
    o[P_2D0] = (S)(2.0 * D0);
    o[P_ALPHA] = (S)al;
    o[P_BETA] = (S)be;
    o[P_N] = (S)n;
    o[P_NINV2N] = (S)(-1.0 / (2.0 * n));
    o[P_H] = (S)h;
    o[P_VALID] = ok ? S(1) : S(0);
    for (int k = P_VALID + 1; k < kNParam; ++k) o[k] = S(0);
}

// ---------------------------------------------------------------------------
// Batched kernel
// ---------------------------------------------------------------------------
template <typename S>
struct BArgs {
    SetDev set;
    const Item* items;
    const int* bin_off;
    const S* params;          // [P][kNParam]
    double* partial;          // [P][nslots][nv]
    int nv;
    // MODE_EVAL outputs (caller numbering); may be null
    double* force;            // [P][3][N]
    double* atom_virial;      // [P][9][N]
    const double* vel;        // [3][N]
    // adjoint inputs
    const double* coef;       // [P][S][8]
};

template <typename S>
__device__ __forceinline__ GeomArrays<S> geom_of(const SetDev& d);
template <>
__device__ __forceinline__ GeomArrays<float> geom_of<float>(const SetDev& d) { return d.gf; }
template <>
__device__ __forceinline__ GeomArrays<double> geom_of<double>(const SetDev& d) { return d.gd; }
template <typename S>
__device__ __forceinline__ const S* fref_of(const SetDev& d);
template <>
__device__ __forceinline__ const float* fref_of<float>(const SetDev& d) { return d.fref32; }
template <>
__device__ __forceinline__ const double* fref_of<double>(const SetDev& d) { return d.fref64; }

struct ItemCtx {
    int s, a0, Ns, npad, R, q, la, atom, steps, nbs, slot, g;
    bool active;
};

__device__ __forceinline__ ItemCtx item_ctx(const SetDev& d, const Item& it) {
    ItemCtx x;
    x.s = it.s;
    x.a0 = d.st_off[x.s];
    x.Ns = d.st_off[x.s + 1] - x.a0;
    x.npad = d.st_npad[x.s];
    x.R = blockDim.x / x.npad;
    x.q = threadIdx.x / x.npad;
    x.la = threadIdx.x - x.q * x.npad;
    x.active = (x.q < x.R) && (x.la < x.Ns);
    x.atom = x.a0 + (x.active ? x.la : 0);
    x.steps = (it.nc + x.R - 1) / x.R;
    x.nbs = d.st_boff[x.s + 1] - d.st_boff[x.s];
    x.slot = d.st_slot[x.s] + (x.npad > 64 ? (x.la >> 6) : 0);
    x.g = x.npad < 64 ? x.npad : 64;
    return x;
}

// Store the group sums of v[0..7] into partial[c][slot][off + vidx].
__device__ __forceinline__ void store_group(double* v, const ItemCtx& x, bool group_ok,
                                            double* __restrict__ partial, int nslots, int nv,
                                            int c, int off, int wmask) {
    int vidx;
    const double sum = group_reduce8(v, x.g, &vidx);
    const int lane = threadIdx.x & 63;
    if (group_ok && (lane & ((x.g >> 3) - 1)) == 0 && ((wmask >> vidx) & 1))
        partial[((size_t)c * nslots + x.slot) * nv + off + vidx] = sum;
}

template <typename S, int MODE, int M>
__device__ __noinline__ void run_batched(const BArgs<S>& A, const Item& it, const ItemCtx& x,
                                         S* __restrict__ lds) {
    const SetDev& d = A.set;
    const int N = d.N;
    Geo<S, M> g;
    g.load(geom_of<S>(d), N, x.atom, x.active);
    constexpr int MM = M > 0 ? M : 1;
    int rev[MM];
    const int Mi = x.active ? d.nnb[x.atom] : 0;
    const int lb = x.active ? d.lbo[x.atom] : 0;
#pragma unroll
    for (int m = 0; m < M; ++m) rev[m] = (x.active && m < Mi) ? d.rev[(size_t)m * N + x.atom] : 0;
    const S* fr = fref_of<S>(d);
    S frx = S(0), fry = S(0), frz = S(0);
    if (MODE == MODE_FIT && x.active) {
        frx = fr[x.atom]; fry = fr[(size_t)N + x.atom]; frz = fr[(size_t)2 * N + x.atom];
    }
    const int orig = x.active ? d.perm[x.atom] : 0;
    S vx = S(0), vy = S(0), vz = S(0);
    if (MODE == MODE_EVAL && A.vel && x.active) {
        vx = (S)A.vel[orig]; vy = (S)A.vel[(size_t)N + orig]; vz = (S)A.vel[(size_t)2 * N + orig];
    }
    S* buf = lds + (size_t)x.q * 3 * x.nbs;

    for (int step = 0; step < x.steps; ++step) {
        const int cl = x.q + step * x.R;
        const bool cok = x.active && cl < it.nc;
        const bool group_ok = (x.q < x.R) && cl < it.nc;
        const int c = it.c0 + (cl < it.nc ? cl : 0);
        Cand<S, S> p;
        load_cand(A.params + (size_t)kNParam * c, p);
        S U;
        S Gx[MM], Gy[MM], Gz[MM];
        site_eval<S, S, M>(g, p, U, Gx, Gy, Gz);
        if (cok) {
#pragma unroll
            for (int m = 0; m < M; ++m)
                if (m < Mi) {
                    buf[lb + m] = Gx[m];
                    buf[x.nbs + lb + m] = Gy[m];
                    buf[2 * x.nbs + lb + m] = Gz[m];
                }
        }
        __syncthreads();
        S Fx = S(0), Fy = S(0), Fz = S(0);
        S wi[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) wi[k] = S(0);
        if (cok) {
#pragma unroll
            for (int m = 0; m < M; ++m)
                if (m < Mi) {
                    const S rx = buf[rev[m]], ry = buf[x.nbs + rev[m]], rz = buf[2 * x.nbs + rev[m]];
                    Fx += Gx[m] - rx;
                    Fy += Gy[m] - ry;
                    Fz += Gz[m] - rz;
                    if (MODE == MODE_EVAL) {
                        const S dx = g.rhi[m] * g.ux[m], dy = g.rhi[m] * g.uy[m], dz = g.rhi[m] * g.uz[m];
                        wi[0] += dx * rx; wi[1] += dx * ry; wi[2] += dx * rz;
                        wi[3] += dy * rx; wi[4] += dy * ry; wi[5] += dy * rz;
                        wi[6] += dz * rx; wi[7] += dz * ry; wi[8] += dz * rz;
                    }
                }
        }
        __syncthreads();
        S w6[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) w6[k] = S(0);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const S dx = g.rhi[m] * g.ux[m], dy = g.rhi[m] * g.uy[m], dz = g.rhi[m] * g.uz[m];
            w6[0] -= dx * Gx[m]; w6[1] -= dy * Gy[m]; w6[2] -= dz * Gz[m];
            w6[3] -= dy * Gz[m]; w6[4] -= dz * Gx[m]; w6[5] -= dx * Gy[m];
        }
        double v[8];
        v[0] = cok ? (double)U : 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) v[1 + k] = cok ? (double)w6[k] : 0.0;
        if (MODE == MODE_FIT) {
            const S ax = Fx - frx, ay = Fy - fry, az = Fz - frz;
            v[7] = cok ? (double)(ax * ax + ay * ay + az * az) : 0.0;
            store_group(v, x, group_ok, A.partial, d.nslots, A.nv, c, 0, 0xff);
        } else {
            v[7] = 0.0;
            store_group(v, x, group_ok, A.partial, d.nslots, A.nv, c, 0, 0xff);
            double u[8];
            const S jx = wi[0] * vx + wi[1] * vy + wi[2] * vz;
            const S jy = wi[3] * vx + wi[4] * vy + wi[5] * vz;
            const S jz = wi[6] * vx + wi[7] * vy + wi[8] * vz;
            u[0] = cok ? (double)jx : 0.0;
            u[1] = cok ? (double)jy : 0.0;
            u[2] = cok ? (double)jz : 0.0;
            u[3] = u[4] = u[5] = u[6] = u[7] = 0.0;
            store_group(u, x, group_ok, A.partial, d.nslots, A.nv, c, 8, 0x07);
            if (cok && A.force) {
                double* f = A.force + (size_t)c * 3 * N;
                f[orig] = (double)Fx;
                f[(size_t)N + orig] = (double)Fy;
                f[(size_t)2 * N + orig] = (double)Fz;
            }
            if (cok && A.atom_virial) {
                double* w = A.atom_virial + (size_t)c * 9 * N;
#pragma unroll
                for (int k = 0; k < 9; ++k) w[(size_t)k * N + orig] = (double)wi[k];
            }
        }
    }
}

__device__ __noinline__ void run_idle(int steps) {
    for (int step = 0; step < steps; ++step) {
        __syncthreads();
        __syncthreads();
    }
}

#define MT_DISPATCH_M(FN, ...)                      \
    switch (Mw) {                                   \
        case 0: FN<0>(__VA_ARGS__); break;          \
        case 1: FN<1>(__VA_ARGS__); break;          \
        case 2: FN<2>(__VA_ARGS__); break;          \
        case 3: FN<3>(__VA_ARGS__); break;          \
        case 4: FN<4>(__VA_ARGS__); break;          \
        case 5: FN<5>(__VA_ARGS__); break;          \
        case 6: FN<6>(__VA_ARGS__); break;          \
        case 7: FN<7>(__VA_ARGS__); break;          \
        case 8: FN<8>(__VA_ARGS__); break;          \
        case 9: FN<9>(__VA_ARGS__); break;          \
        case 10: FN<10>(__VA_ARGS__); break;        \
        case 11: FN<11>(__VA_ARGS__); break;        \
        case 12: FN<12>(__VA_ARGS__); break;        \
        case 13: FN<13>(__VA_ARGS__); break;        \
        case 14: FN<14>(__VA_ARGS__); break;        \
        case 15: FN<15>(__VA_ARGS__); break;        \
        default: FN<16>(__VA_ARGS__); break;        \
    }

template <typename S, int MODE>
struct BatchedRun {
    template <int M>
    static __device__ void call(const BArgs<S>& A, const Item& it, const ItemCtx& x, S* lds) {
        run_batched<S, MODE, M>(A, it, x, lds);
    }
};

template <typename S, int MODE>
__device__ __forceinline__ void batched_item(const BArgs<S>& A, const Item& it, S* lds) {
    const ItemCtx x = item_ctx(A.set, it);
    const int Mi = x.active ? A.set.nnb[x.atom] : -1;
    const int Mw = wave_max_int(Mi);
    if (Mw < 0) {
        run_idle(x.steps);
        return;
    }
#define MT_CALL(MV) BatchedRun<S, MODE>::template call<MV>
    switch (Mw) {
        case 0: MT_CALL(0)(A, it, x, lds); break;
        case 1: MT_CALL(1)(A, it, x, lds); break;
        case 2: MT_CALL(2)(A, it, x, lds); break;
        case 3: MT_CALL(3)(A, it, x, lds); break;
        case 4: MT_CALL(4)(A, it, x, lds); break;
        case 5: MT_CALL(5)(A, it, x, lds); break;
        case 6: MT_CALL(6)(A, it, x, lds); break;
        case 7: MT_CALL(7)(A, it, x, lds); break;
        case 8: MT_CALL(8)(A, it, x, lds); break;
        case 9: MT_CALL(9)(A, it, x, lds); break;
        case 10: MT_CALL(10)(A, it, x, lds); break;
        case 11: MT_CALL(11)(A, it, x, lds); break;
        case 12: MT_CALL(12)(A, it, x, lds); break;
        case 13: MT_CALL(13)(A, it, x, lds); break;
        case 14: MT_CALL(14)(A, it, x, lds); break;
        case 15: MT_CALL(15)(A, it, x, lds); break;
        default: MT_CALL(16)(A, it, x, lds); break;
    }
#undef MT_CALL
}

template <typename S, int MODE>
__global__ __launch_bounds__(512) void k_batched(BArgs<S> A) {
    extern __shared__ unsigned char lds_raw[];
    S* lds = reinterpret_cast<S*>(lds_raw);
    const int b0 = A.bin_off[blockIdx.x], b1 = A.bin_off[blockIdx.x + 1];
    for (int i = b0; i < b1; ++i) {
        const Item it = A.items[i];
        batched_item<S, MODE>(A, it, lds);
        __syncthreads();
    }
}

template <typename S, int MODE>
__global__ __launch_bounds__(512) void k_single(BArgs<S> A, Item it) {
    extern __shared__ unsigned char lds_raw[];
    S* lds = reinterpret_cast<S*>(lds_raw);
    batched_item<S, MODE>(A, it, lds);
}

// ---------------------------------------------------------------------------
// Adjoint kernel: dZ/dx of the fitness.  For candidate c and structure s,
//   dZ/dx|_s = sum_i [ k_e U_i' - sum_j G_ij' . delta_ij ],
//   delta_ij = k_f (a_j - a_i) + C_s r_ij,   a = F - F*,
// where ' is the derivative with respect to the six parameters (forward-mode
// dual numbers), k_e = w_e (e_s - e*_s)/(N_s Z_e Q_e), k_f = w_f/(Z_f Q_f) and
// C_s = w_v/(N_s Z_v Q_v) times the symmetric matrix of virial residuals (off
// diagonals halved).  These follow from dF_i/dx = -d/dx dE/dr_i and
// dW/dx = -sum r_ij (x) dG_ij/dx.
// ---------------------------------------------------------------------------
template <typename S, int M>
__device__ __noinline__ void run_adjoint(const BArgs<S>& A, const Item& it, const ItemCtx& x,
                                         S* __restrict__ lds) {
    const SetDev& d = A.set;
    const int N = d.N;
    Geo<S, M> g;
    g.load(geom_of<S>(d), N, x.atom, x.active);
    constexpr int MM = M > 0 ? M : 1;
    int rev[MM], jl[MM];
    const int Mi = x.active ? d.nnb[x.atom] : 0;
    const int lb = x.active ? d.lbo[x.atom] : 0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const bool ok = x.active && m < Mi;
        rev[m] = ok ? d.rev[(size_t)m * N + x.atom] : 0;
        jl[m] = ok ? d.jl[(size_t)m * N + x.atom] : 0;
    }
    const S* fr = fref_of<S>(d);
    S frx = S(0), fry = S(0), frz = S(0);
    if (x.active) { frx = fr[x.atom]; fry = fr[(size_t)N + x.atom]; frz = fr[(size_t)2 * N + x.atom]; }
    S* buf = lds + (size_t)x.q * 3 * x.nbs;
    S* abuf = lds + (size_t)x.R * 3 * x.nbs + (size_t)x.q * 3 * x.npad;

    for (int step = 0; step < x.steps; ++step) {
        const int cl = x.q + step * x.R;
        const bool cok = x.active && cl < it.nc;
        const bool group_ok = (x.q < x.R) && cl < it.nc;
        const int c = it.c0 + (cl < it.nc ? cl : 0);
        Cand<Dual<S>, S> p;
        load_cand(A.params + (size_t)kNParam * c, p);
        Dual<S> U;
        Dual<S> Gx[MM], Gy[MM], Gz[MM];
        site_eval<Dual<S>, S, M>(g, p, U, Gx, Gy, Gz);
        if (cok) {
#pragma unroll
            for (int m = 0; m < M; ++m)
                if (m < Mi) {
                    buf[lb + m] = Gx[m].v;
                    buf[x.nbs + lb + m] = Gy[m].v;
                    buf[2 * x.nbs + lb + m] = Gz[m].v;
                }
        }
        __syncthreads();
        S ax = S(0), ay = S(0), az = S(0);
        if (cok) {
#pragma unroll
            for (int m = 0; m < M; ++m)
                if (m < Mi) {
                    ax += Gx[m].v - buf[rev[m]];
                    ay += Gy[m].v - buf[x.nbs + rev[m]];
                    az += Gz[m].v - buf[2 * x.nbs + rev[m]];
                }
            ax -= frx; ay -= fry; az -= frz;
            abuf[x.la] = ax;
            abuf[x.npad + x.la] = ay;
            abuf[2 * x.npad + x.la] = az;
        }
        __syncthreads();
        const double* cf = A.coef + ((size_t)c * d.S + x.s) * 8;
        const S ke = (S)cf[0], kf = (S)cf[1];
        const S cxx = (S)cf[2], cyy = (S)cf[3], czz = (S)cf[4];
        const S cyz = (S)cf[5], czx = (S)cf[6], cxy = (S)cf[7];
        S phi[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) phi[k] = ke * U.d[k];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            S ajx = S(0), ajy = S(0), ajz = S(0);
            if (cok && m < Mi) {
                ajx = abuf[jl[m]]; ajy = abuf[x.npad + jl[m]]; ajz = abuf[2 * x.npad + jl[m]];
            }
            const S dx = g.rhi[m] * g.ux[m], dy = g.rhi[m] * g.uy[m], dz = g.rhi[m] * g.uz[m];
            const S ex = kf * (ajx - ax) + cxx * dx + cxy * dy + czx * dz;
            const S ey = kf * (ajy - ay) + cxy * dx + cyy * dy + cyz * dz;
            const S ez = kf * (ajz - az) + czx * dx + cyz * dy + czz * dz;
#pragma unroll
            for (int k = 0; k < 6; ++k) phi[k] -= Gx[m].d[k] * ex + Gy[m].d[k] * ey + Gz[m].d[k] * ez;
        }
        __syncthreads();
        double v[8];
#pragma unroll
        for (int k = 0; k < 6; ++k) v[k] = cok ? (double)phi[k] : 0.0;
        v[6] = v[7] = 0.0;
        store_group(v, x, group_ok, A.partial, d.nslots, A.nv, c, 0, 0x3f);
    }
}

template <typename S>
struct AdjointRun {
    template <int M>
    static __device__ void call(const BArgs<S>& A, const Item& it, const ItemCtx& x, S* lds) {
        run_adjoint<S, M>(A, it, x, lds);
    }
};

__device__ __noinline__ void run_idle3(int steps) {
    for (int step = 0; step < steps; ++step) {
        __syncthreads();
        __syncthreads();
        __syncthreads();
    }
}

template <typename S>
__device__ __forceinline__ void adjoint_item(const BArgs<S>& A, const Item& it, S* lds) {
    const ItemCtx x = item_ctx(A.set, it);
    const int Mi = x.active ? A.set.nnb[x.atom] : -1;
    const int Mw = wave_max_int(Mi);
    if (Mw < 0) {
        run_idle3(x.steps);
        return;
    }
#define MT_CALL(MV) AdjointRun<S>::template call<MV>
    switch (Mw) {
        case 0: MT_CALL(0)(A, it, x, lds); break;
        case 1: MT_CALL(1)(A, it, x, lds); break;
        case 2: MT_CALL(2)(A, it, x, lds); break;
        case 3: MT_CALL(3)(A, it, x, lds); break;
        case 4: MT_CALL(4)(A, it, x, lds); break;
        case 5: MT_CALL(5)(A, it, x, lds); break;
        case 6: MT_CALL(6)(A, it, x, lds); break;
        case 7: MT_CALL(7)(A, it, x, lds); break;
        case 8: MT_CALL(8)(A, it, x, lds); break;
        case 9: MT_CALL(9)(A, it, x, lds); break;
        case 10: MT_CALL(10)(A, it, x, lds); break;
        case 11: MT_CALL(11)(A, it, x, lds); break;
        case 12: MT_CALL(12)(A, it, x, lds); break;
        case 13: MT_CALL(13)(A, it, x, lds); break;
        case 14: MT_CALL(14)(A, it, x, lds); break;
        case 15: MT_CALL(15)(A, it, x, lds); break;
        default: MT_CALL(16)(A, it, x, lds); break;
    }
#undef MT_CALL
}

template <typename S>
__global__ __launch_bounds__(512) void k_adjoint(BArgs<S> A) {
    extern __shared__ unsigned char lds_raw[];
    S* lds = reinterpret_cast<S*>(lds_raw);
    const int b0 = A.bin_off[blockIdx.x], b1 = A.bin_off[blockIdx.x + 1];
    for (int i = b0; i < b1; ++i) {
        const Item it = A.items[i];
        adjoint_item<S>(A, it, lds);
        __syncthreads();
    }
}

template <typename S>
__global__ __launch_bounds__(512) void k_adjoint_single(BArgs<S> A, Item it) {
    extern __shared__ unsigned char lds_raw[];
    S* lds = reinterpret_cast<S*>(lds_raw);
    adjoint_item<S>(A, it, lds);
}

// ---------------------------------------------------------------------------
// Large structures (more atoms than one block holds): two passes per
// candidate.  Pass 1 writes every bond gradient to global memory and the
// energy/virial partials; pass 2 gathers forces, per-atom virial, heat
// current and the force residual.
// ---------------------------------------------------------------------------
struct LArgs {
    int s, c0;                 // structure, first candidate of the chunk
    void* gbuf;                // [chunk][3][nbs] of S
};

template <typename S, int M>
__device__ __noinline__ void run_large_site(const BArgs<S>& A, const LArgs& L, int atom, bool active) {
    const SetDev& d = A.set;
    const int N = d.N;
    Geo<S, M> g;
    g.load(geom_of<S>(d), N, atom, active);
    constexpr int MM = M > 0 ? M : 1;
    const int c = L.c0 + blockIdx.y;
    const int a0 = d.st_off[L.s];
    const int nbs = d.st_boff[L.s + 1] - d.st_boff[L.s];
    const int Mi = active ? d.nnb[atom] : 0;
    const int lb = active ? d.lbo[atom] : 0;
    Cand<S, S> p;
    load_cand(A.params + (size_t)kNParam * c, p);
    S U;
    S Gx[MM], Gy[MM], Gz[MM];
    site_eval<S, S, M>(g, p, U, Gx, Gy, Gz);
    S* gb = reinterpret_cast<S*>(L.gbuf) + (size_t)blockIdx.y * 3 * nbs;
    if (active) {
#pragma unroll
        for (int m = 0; m < M; ++m)
            if (m < Mi) {
                gb[lb + m] = Gx[m];
                gb[nbs + lb + m] = Gy[m];
                gb[2 * nbs + lb + m] = Gz[m];
            }
    }
    S w6[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) w6[k] = S(0);
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const S dx = g.rhi[m] * g.ux[m], dy = g.rhi[m] * g.uy[m], dz = g.rhi[m] * g.uz[m];
        w6[0] -= dx * Gx[m]; w6[1] -= dy * Gy[m]; w6[2] -= dz * Gz[m];
        w6[3] -= dy * Gz[m]; w6[4] -= dz * Gx[m]; w6[5] -= dx * Gy[m];
    }
    double v[8];
    v[0] = active ? (double)U : 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) v[1 + k] = active ? (double)w6[k] : 0.0;
    v[7] = 0.0;
    int vidx;
    const double sum = group_reduce8(v, 64, &vidx);
    const int lane = threadIdx.x & 63;
    const int slot = d.st_slot[L.s] + ((atom - a0) >> 6);
    if ((lane & 7) == 0 && vidx < 7)
        A.partial[((size_t)c * d.nslots + slot) * A.nv + vidx] = sum;
}

template <typename S>
struct LargeRun {
    template <int M>
    static __device__ void call(const BArgs<S>& A, const LArgs& L, int atom, bool active) {
        run_large_site<S, M>(A, L, atom, active);
    }
};

template <typename S>
__global__ __launch_bounds__(256) void k_large_site(BArgs<S> A, LArgs L) {
    const SetDev& d = A.set;
    const int a0 = d.st_off[L.s], Ns = d.st_off[L.s + 1] - a0;
    const int la = blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = la < Ns;
    const int atom = a0 + (active ? la : 0);
    const int Mi = active ? d.nnb[atom] : -1;
    const int Mw = wave_max_int(Mi);
    if (Mw < 0) return;
#define MT_CALL(MV) LargeRun<S>::template call<MV>
    switch (Mw) {
        case 0: MT_CALL(0)(A, L, atom, active); break;
        case 1: MT_CALL(1)(A, L, atom, active); break;
        case 2: MT_CALL(2)(A, L, atom, active); break;
        case 3: MT_CALL(3)(A, L, atom, active); break;
        case 4: MT_CALL(4)(A, L, atom, active); break;
        case 5: MT_CALL(5)(A, L, atom, active); break;
        case 6: MT_CALL(6)(A, L, atom, active); break;
        case 7: MT_CALL(7)(A, L, atom, active); break;
        case 8: MT_CALL(8)(A, L, atom, active); break;
        case 9: MT_CALL(9)(A, L, atom, active); break;
        case 10: MT_CALL(10)(A, L, atom, active); break;
        case 11: MT_CALL(11)(A, L, atom, active); break;
        case 12: MT_CALL(12)(A, L, atom, active); break;
        case 13: MT_CALL(13)(A, L, atom, active); break;
        case 14: MT_CALL(14)(A, L, atom, active); break;
        case 15: MT_CALL(15)(A, L, atom, active); break;
        default: MT_CALL(16)(A, L, atom, active); break;
    }
#undef MT_CALL
}

template <typename S, int MODE>
__global__ __launch_bounds__(256) void k_large_gather(BArgs<S> A, LArgs L) {
    const SetDev& d = A.set;
    const int N = d.N;
    const int a0 = d.st_off[L.s], Ns = d.st_off[L.s + 1] - a0;
    const int nbs = d.st_boff[L.s + 1] - d.st_boff[L.s];
    const int la = blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = la < Ns;
    const int atom = a0 + (active ? la : 0);
    const int c = L.c0 + blockIdx.y;
    const S* gb = reinterpret_cast<const S*>(L.gbuf) + (size_t)blockIdx.y * 3 * nbs;
    const GeomArrays<S> G = geom_of<S>(d);
    S Fx = S(0), Fy = S(0), Fz = S(0);
    S wi[9];
    for (int k = 0; k < 9; ++k) wi[k] = S(0);
    if (active) {
        const int Mi = d.nnb[atom], lb = d.lbo[atom];
        for (int m = 0; m < Mi; ++m) {
            const size_t o = (size_t)m * N + atom;
            const int r = d.rev[o];
            const S rx = gb[r], ry = gb[nbs + r], rz = gb[2 * nbs + r];
            Fx += gb[lb + m] - rx;
            Fy += gb[nbs + lb + m] - ry;
            Fz += gb[2 * nbs + lb + m] - rz;
            if (MODE == MODE_EVAL) {
                const S rr = G.rhi[o];
                const S dx = rr * G.ux[o], dy = rr * G.uy[o], dz = rr * G.uz[o];
                wi[0] += dx * rx; wi[1] += dx * ry; wi[2] += dx * rz;
                wi[3] += dy * rx; wi[4] += dy * ry; wi[5] += dy * rz;
                wi[6] += dz * rx; wi[7] += dz * ry; wi[8] += dz * rz;
            }
        }
    }
    const int orig = active ? d.perm[atom] : 0;
    double v[8];
    for (int k = 0; k < 8; ++k) v[k] = 0.0;
    const int lane = threadIdx.x & 63;
    const int slot = d.st_slot[L.s] + (la >> 6);
    int vidx;
    if (MODE == MODE_FIT) {
        const S* fr = fref_of<S>(d);
        if (active) {
            const S ax = Fx - fr[atom], ay = Fy - fr[(size_t)N + atom], az = Fz - fr[(size_t)2 * N + atom];
            v[7] = (double)(ax * ax + ay * ay + az * az);
        }
        const double sum = group_reduce8(v, 64, &vidx);
        if ((lane & 7) == 0 && vidx == 7) A.partial[((size_t)c * d.nslots + slot) * A.nv + 7] = sum;
    } else {
        if (active && A.vel) {
            const S vx = (S)A.vel[orig], vy = (S)A.vel[(size_t)N + orig], vz = (S)A.vel[(size_t)2 * N + orig];
            v[0] = (double)(wi[0] * vx + wi[1] * vy + wi[2] * vz);
            v[1] = (double)(wi[3] * vx + wi[4] * vy + wi[5] * vz);
            v[2] = (double)(wi[6] * vx + wi[7] * vy + wi[8] * vz);
        }
        const double sum = group_reduce8(v, 64, &vidx);
        if ((lane & 7) == 0 && vidx < 3) A.partial[((size_t)c * d.nslots + slot) * A.nv + 8 + vidx] = sum;
        if (active && A.force) {
            double* f = A.force + (size_t)c * 3 * N;
            f[orig] = (double)Fx; f[(size_t)N + orig] = (double)Fy; f[(size_t)2 * N + orig] = (double)Fz;
        }
        if (active && A.atom_virial) {
            double* w = A.atom_virial + (size_t)c * 9 * N;
            for (int k = 0; k < 9; ++k) w[(size_t)k * N + orig] = (double)wi[k];
        }
    }
}

// ---------------------------------------------------------------------------
// Finalize kernels (one block per candidate, fixed summation order).
// ---------------------------------------------------------------------------
template <typename S>
__device__ __forceinline__ bool cand_valid(const S* params, int c) {
    return params[(size_t)kNParam * c + P_VALID] != S(0);
}

__device__ __forceinline__ void block_sum3(double* a, double (*sh)[256]) {
    for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] = a[k];
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + o];
        __syncthreads();
    }
    for (int k = 0; k < 3; ++k) a[k] = sh[k][0];
}

struct FinArgs {
    SetDev set;
    const double* partial;
    int nv;
    const double* eref; const double* wref;
    double Qe, Qv, Qf, we, wv, wf;
    const void* params; int param_double;
    double* Z;                 // [P][4]
    double* coef;              // [P][S][8] or null (gradient coefficients)
    double* energy; double* virial; double* heat;
};

__device__ __forceinline__ void struct_sums(const FinArgs& F, int c, int s, double* e, double* w6,
                                            double* rf, double* j3) {
    const SetDev& d = F.set;
    *e = 0; *rf = 0;
    for (int k = 0; k < 6; ++k) w6[k] = 0;
    for (int k = 0; k < 3; ++k) j3[k] = 0;
    for (int sl = d.st_slot[s]; sl < d.st_slot[s + 1]; ++sl) {
        const double* p = F.partial + ((size_t)c * d.nslots + sl) * F.nv;
        *e += p[0];
        for (int k = 0; k < 6; ++k) w6[k] += p[1 + k];
        *rf += p[7];
        if (F.nv >= 11)
            for (int k = 0; k < 3; ++k) j3[k] += p[8 + k];
    }
}

__global__ __launch_bounds__(256) void k_finalize_fit(FinArgs F) {
    __shared__ double sh[3][256];
    const int c = blockIdx.x;
    const SetDev& d = F.set;
    double acc[3] = {0, 0, 0};
    for (int s = threadIdx.x; s < d.S; s += blockDim.x) {
        double e, w6[6], rf, j3[3];
        struct_sums(F, c, s, &e, w6, &rf, j3);
        const double n = (double)(d.st_off[s + 1] - d.st_off[s]);
        const double de = e / n - F.eref[s];
        acc[0] += de * de;
        for (int k = 0; k < 6; ++k) {
            const double dw = w6[k] / n - F.wref[6 * s + k];
            acc[1] += dw * dw;
        }
        acc[2] += rf;
    }
    block_sum3(acc, sh);
    if (threadIdx.x == 0) {
        const bool ok = F.param_double ? cand_valid((const double*)F.params, c)
                                       : cand_valid((const float*)F.params, c);
        const double Ze = sqrt(acc[0] / F.Qe), Zv = sqrt(acc[1] / F.Qv), Zf = sqrt(acc[2] / F.Qf);
        const double Z = F.we * Ze + F.wv * Zv + F.wf * Zf;
        const double nan = __longlong_as_double(0x7ff8000000000000ll);
        F.Z[4 * c + 0] = ok ? Z : nan;
        F.Z[4 * c + 1] = ok ? Ze : nan;
        F.Z[4 * c + 2] = ok ? Zv : nan;
        F.Z[4 * c + 3] = ok ? Zf : nan;
    }
}

// Gradient coefficients per (candidate, structure), from the forward partials
// and Z: k_e, k_f, and C_s (xx yy zz yz zx xy, off-diagonals halved).
__global__ __launch_bounds__(256) void k_grad_coef(FinArgs F) {
    const int c = blockIdx.x;
    const SetDev& d = F.set;
    const double Ze = F.Z[4 * c + 1], Zv = F.Z[4 * c + 2], Zf = F.Z[4 * c + 3];
    const double ge = Ze > 0 ? F.we / (Ze * F.Qe) : 0.0;
    const double gv = Zv > 0 ? F.wv / (Zv * F.Qv) : 0.0;
    const double gf = Zf > 0 ? F.wf / (Zf * F.Qf) : 0.0;
    for (int s = threadIdx.x; s < d.S; s += blockDim.x) {
        double e, w6[6], rf, j3[3];
        struct_sums(F, c, s, &e, w6, &rf, j3);
        const double n = (double)(d.st_off[s + 1] - d.st_off[s]);
        double* o = F.coef + ((size_t)c * d.S + s) * 8;
        o[0] = ge * (e / n - F.eref[s]) / n;
        o[1] = gf;
        double r[6];
        for (int k = 0; k < 6; ++k) r[k] = gv * (w6[k] / n - F.wref[6 * s + k]) / n;
        o[2] = r[0]; o[3] = r[1]; o[4] = r[2];
        o[5] = 0.5 * r[3]; o[6] = 0.5 * r[4]; o[7] = 0.5 * r[5];
    }
}

__global__ __launch_bounds__(256) void k_finalize_grad(FinArgs F, double* dZdx) {
    __shared__ double sh[6][256];
    const int c = blockIdx.x;
    const SetDev& d = F.set;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int sl = threadIdx.x; sl < d.nslots; sl += blockDim.x) {
        const double* p = F.partial + ((size_t)c * d.nslots + sl) * F.nv;
        for (int k = 0; k < 6; ++k) acc[k] += p[k];
    }
    for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const bool ok = F.param_double ? cand_valid((const double*)F.params, c)
                                       : cand_valid((const float*)F.params, c);
        const double nan = __longlong_as_double(0x7ff8000000000000ll);
        for (int k = 0; k < 6; ++k) dZdx[6 * c + k] = ok ? sh[k][0] : nan;
    }
}

__global__ __launch_bounds__(256) void k_finalize_eval(FinArgs F) {
    __shared__ double sh[3][256];
    const int c = blockIdx.x;
    const SetDev& d = F.set;
    const bool ok = F.param_double ? cand_valid((const double*)F.params, c)
                                   : cand_valid((const float*)F.params, c);
    const double nan = __longlong_as_double(0x7ff8000000000000ll);
    double jacc[3] = {0, 0, 0};
    for (int s = threadIdx.x; s < d.S; s += blockDim.x) {
        double e, w6[6], rf, j3[3];
        struct_sums(F, c, s, &e, w6, &rf, j3);
        if (F.energy) F.energy[(size_t)c * d.S + s] = ok ? e : nan;
        if (F.virial)
            for (int k = 0; k < 6; ++k) F.virial[((size_t)c * d.S + s) * 6 + k] = ok ? w6[k] : nan;
        for (int k = 0; k < 3; ++k) jacc[k] += j3[k];
    }
    block_sum3(jacc, sh);
    if (threadIdx.x == 0 && F.heat)
        for (int k = 0; k < 3; ++k) F.heat[3 * c + k] = ok ? jacc[k] : nan;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
namespace {

template <typename S>
BArgs<S> make_args(mt_set* set, double* partial, int nv) {
    BArgs<S> A{};
    A.set = set->dev();
    A.params = sizeof(S) == 8 ? (const S*)set->params_d.p : (const S*)set->params_f.p;
    A.partial = partial;
    A.nv = nv;
    return A;
}

FinArgs make_fin(mt_set* set, int nv, const double* partial) {
    FinArgs F{};
    F.set = set->dev();
    F.partial = partial;
    F.nv = nv;
    F.eref = set->eref.as<double>();
    F.wref = set->wref.as<double>();
    F.Qe = set->Q[0]; F.Qv = set->Q[1]; F.Qf = set->Q[2];
    return F;
}

int grid_of(long long n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

size_t lds_bytes(const mt_set* set, int block, int elem) {
    size_t best = 0;
    for (int s = 0; s < set->S; ++s) {
        if (set->h_large[s]) continue;
        const int npad = set->h_npad[s];
        const int R = block / npad;
        const size_t nbs = (size_t)(set->h_boff[s + 1] - set->h_boff[s]);
        // bond-gradient exchange, plus the force-residual exchange of the adjoint
        const size_t b = (size_t)R * 3 * (nbs + npad) * elem;
        best = std::max(best, b);
    }
    return std::max<size_t>(best, 16);
}

LaunchCfg default_cfg(const mt_set* set, int P, int precision) {
    (void)precision;
    LaunchCfg c;
    int maxpad = 8;
    for (int s = 0; s < set->S; ++s)
        if (!set->h_large[s]) maxpad = std::max(maxpad, set->h_npad[s]);
    c.block = std::max(64, ((maxpad + 63) / 64) * 64);
    if (c.block < 256 && maxpad <= 64) c.block = 256;
    // aim for about 4 work items per compute unit
    long long pairs = (long long)P * std::max(1, set->n_batched);
    long long tile = std::max<long long>(1, pairs / 1024);
    tile = std::min<long long>(tile, P);
    c.tile = (int)std::max<long long>(1, tile);
    c.persistent = 0;
    return c;
}

ItemPlan* get_plan(mt_set* set, int P, const LaunchCfg& cfg, int precision) {
    auto key = std::make_tuple(P, cfg.block, cfg.tile, cfg.persistent, precision);
    auto itp = set->plans.find(key);
    if (itp != set->plans.end()) return itp->second.get();
    auto plan = std::make_unique<ItemPlan>();
    std::vector<Item> items;
    for (int s = 0; s < set->S; ++s) {
        if (set->h_large[s]) continue;
        const int npad = set->h_npad[s];
        const int R = cfg.block / npad;
        if (R < 1) return nullptr;
        int tile = std::max(cfg.tile, 1);
        tile = ((tile + R - 1) / R) * R;      // whole steps of the replicas
        const int ns = set->h_off[s + 1] - set->h_off[s];
        for (int c0 = 0; c0 < P; c0 += tile) {
            Item it;
            it.s = s;
            it.c0 = c0;
            it.nc = std::min(tile, P - c0);
            const long long steps = (it.nc + R - 1) / R;
            const long long per = set->h_trip[s] + 8ll * ns + 64;
            it.cost = (int)std::min<long long>(steps * per / std::max(1, R) + 1, 1ll << 30);
            items.push_back(it);
        }
    }
    std::stable_sort(items.begin(), items.end(),
                     [](const Item& a, const Item& b) { return a.cost > b.cost; });
    std::vector<int> bin_off;
    std::vector<Item> ordered;
    if (!cfg.persistent) {
        ordered = items;
        bin_off.resize(items.size() + 1);
        std::iota(bin_off.begin(), bin_off.end(), 0);
    } else {
        int dev = 0, ncu = 256;
        (void)hipGetDevice(&dev);
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
            ncu = prop.multiProcessorCount;
        const int per_cu = std::max(1, 1024 / cfg.block);
        const int nbins = (int)std::min<size_t>(items.size(), (size_t)ncu * per_cu);
        std::vector<std::vector<Item>> bins(std::max(nbins, 1));
        using E = std::pair<long long, int>;
        std::priority_queue<E, std::vector<E>, std::greater<E>> heap;
        for (int b = 0; b < (int)bins.size(); ++b) heap.push({0, b});
        for (const Item& it : items) {      // longest first onto the least-loaded bin
            E e = heap.top();
            heap.pop();
            bins[e.second].push_back(it);
            heap.push({e.first + it.cost, e.second});
        }
        bin_off.push_back(0);
        for (auto& b : bins) {
            for (auto& it : b) ordered.push_back(it);
            bin_off.push_back((int)ordered.size());
        }
    }
    plan->n_items = (int)ordered.size();
    plan->n_bins = (int)bin_off.size() - 1;
    if (plan->n_items > 0) {
        if (plan->items.reserve(sizeof(Item) * ordered.size()) != hipSuccess) return nullptr;
        if (hipMemcpy(plan->items.p, ordered.data(), sizeof(Item) * ordered.size(),
                      hipMemcpyHostToDevice) != hipSuccess)
            return nullptr;
    }
    if (plan->bin_off.reserve(sizeof(int) * bin_off.size()) != hipSuccess) return nullptr;
    if (hipMemcpy(plan->bin_off.p, bin_off.data(), sizeof(int) * bin_off.size(),
                  hipMemcpyHostToDevice) != hipSuccess)
        return nullptr;
    plan->lds_f = lds_bytes(set, cfg.block, 4);
    plan->lds_d = lds_bytes(set, cfg.block, 8);
    ItemPlan* raw = plan.get();
    set->plans[key] = std::move(plan);
    return raw;
}

int decode_params(mt_set* set, const double* x, int P, hipStream_t st) {
    HIPCHECK(set->params_f.reserve(sizeof(float) * kNParam * P));
    HIPCHECK(set->params_d.reserve(sizeof(double) * kNParam * P));
    k_decode<float><<<grid_of(P, 128), 128, 0, st>>>(P, x, set->params_f.as<float>());
    HIPCHECK(hipGetLastError());
    k_decode<double><<<grid_of(P, 128), 128, 0, st>>>(P, x, set->params_d.as<double>());
    HIPCHECK(hipGetLastError());
    return MT_OK;
}

template <typename S, int MODE>
static int launch_batched_t(mt_set* set, const ItemPlan& plan, const LaunchCfg& cfg, int nv,
                            const double* vel, double* force, double* atom_virial, hipStream_t st) {
    if (plan.n_items == 0) return MT_OK;
    BArgs<S> A = make_args<S>(set, set->partial.as<double>(), nv);
    A.items = plan.items.as<Item>();
    A.bin_off = plan.bin_off.as<int>();
    A.vel = vel;
    A.force = force;
    A.atom_virial = atom_virial;
    const size_t lds = sizeof(S) == 8 ? plan.lds_d : plan.lds_f;
    hipLaunchKernelGGL((k_batched<S, MODE>), dim3(plan.n_bins), dim3(cfg.block), lds, st, A);
    HIPCHECK(hipGetLastError());
    return MT_OK;
}

int launch_batched(mt_set* set, const ItemPlan& plan, const LaunchCfg& cfg, int P, int precision,
                   int mode, const double* vel, double* force, double* atom_virial,
                   hipStream_t st) {
    (void)P;
    const int nv = mode == MODE_FIT ? kNVFit : kNVEval;
    if (precision == MT_FP64) {
        return mode == MODE_FIT
                   ? launch_batched_t<double, MODE_FIT>(set, plan, cfg, nv, vel, force, atom_virial, st)
                   : launch_batched_t<double, MODE_EVAL>(set, plan, cfg, nv, vel, force, atom_virial, st);
    }
    return mode == MODE_FIT
               ? launch_batched_t<float, MODE_FIT>(set, plan, cfg, nv, vel, force, atom_virial, st)
               : launch_batched_t<float, MODE_EVAL>(set, plan, cfg, nv, vel, force, atom_virial, st);
}

template <typename S, int MODE>
static int launch_plain_t(mt_set* set, int P, int nv, const double* vel, double* force,
                          double* atom_virial, hipStream_t st) {
    BArgs<S> A = make_args<S>(set, set->partial.as<double>(), nv);
    A.vel = vel;
    A.force = force;
    A.atom_virial = atom_virial;
    for (int s = 0; s < set->S; ++s) {
        if (set->h_large[s]) continue;
        const int npad = set->h_npad[s];
        const int block = std::max(64, npad);
        const size_t nbs = (size_t)(set->h_boff[s + 1] - set->h_boff[s]);
        const size_t lds = (size_t)(block / npad) * 3 * (nbs + npad) * sizeof(S);
        for (int c = 0; c < P; ++c) {
            Item it{s, c, 1, 0};
            hipLaunchKernelGGL((k_single<S, MODE>), dim3(1), dim3(block), lds, st, A, it);
        }
    }
    HIPCHECK(hipGetLastError());
    return MT_OK;
}

int launch_plain(mt_set* set, int P, int precision, int mode, const double* vel, double* force,
                 double* atom_virial, hipStream_t st) {
    const int nv = mode == MODE_FIT ? kNVFit : kNVEval;
    if (precision == MT_FP64)
        return mode == MODE_FIT ? launch_plain_t<double, MODE_FIT>(set, P, nv, vel, force, atom_virial, st)
                                : launch_plain_t<double, MODE_EVAL>(set, P, nv, vel, force, atom_virial, st);
    return mode == MODE_FIT ? launch_plain_t<float, MODE_FIT>(set, P, nv, vel, force, atom_virial, st)
                            : launch_plain_t<float, MODE_EVAL>(set, P, nv, vel, force, atom_virial, st);
}

template <typename S, int MODE>
static int launch_large_t(mt_set* set, int P, int nv, const double* vel, double* force,
                          double* atom_virial, hipStream_t st) {
    BArgs<S> A = make_args<S>(set, set->partial.as<double>(), nv);
    A.vel = vel;
    A.force = force;
    A.atom_virial = atom_virial;
    for (int s = 0; s < set->S; ++s) {
        if (!set->h_large[s]) continue;
        const int ns = set->h_off[s + 1] - set->h_off[s];
        const size_t nbs = (size_t)(set->h_boff[s + 1] - set->h_boff[s]);
        const size_t per = 3 * nbs * sizeof(S);
        int chunk = (int)std::max<size_t>(1, std::min<size_t>((size_t)P, (256ull << 20) / std::max<size_t>(per, 1)));
        chunk = std::min(chunk, 65535);
        HIPCHECK(set->gbuf.reserve(per * chunk));
        for (int c0 = 0; c0 < P; c0 += chunk) {
            const int nc = std::min(chunk, P - c0);
            LArgs L{s, c0, set->gbuf.p};
            dim3 grid(grid_of(ns, 256), nc);
            hipLaunchKernelGGL((k_large_site<S>), grid, dim3(256), 0, st, A, L);
            hipLaunchKernelGGL((k_large_gather<S, MODE>), grid, dim3(256), 0, st, A, L);
        }
    }
    HIPCHECK(hipGetLastError());
    return MT_OK;
}

int launch_large(mt_set* set, int P, int precision, int mode, const double* vel, double* force,
                 double* atom_virial, hipStream_t st) {
    if (set->n_large == 0) return MT_OK;
    const int nv = mode == MODE_FIT ? kNVFit : kNVEval;
    if (precision == MT_FP64)
        return mode == MODE_FIT ? launch_large_t<double, MODE_FIT>(set, P, nv, vel, force, atom_virial, st)
                                : launch_large_t<double, MODE_EVAL>(set, P, nv, vel, force, atom_virial, st);
    return mode == MODE_FIT ? launch_large_t<float, MODE_FIT>(set, P, nv, vel, force, atom_virial, st)
                            : launch_large_t<float, MODE_EVAL>(set, P, nv, vel, force, atom_virial, st);
}

int launch_finalize_fit(mt_set* set, int P, const double* w, double* Z, hipStream_t st) {
    FinArgs F = make_fin(set, kNVFit, set->partial.as<double>());
    F.we = w[0]; F.wv = w[1]; F.wf = w[2];
    F.params = set->params_d.p;
    F.param_double = 1;
    F.Z = Z;
    hipLaunchKernelGGL(k_finalize_fit, dim3(P), dim3(256), 0, st, F);
    HIPCHECK(hipGetLastError());
    return MT_OK;
}

int launch_finalize_eval(mt_set* set, int P, double* energy, double* virial, double* heat,
                         hipStream_t st) {
    FinArgs F = make_fin(set, kNVEval, set->partial.as<double>());
    F.params = set->params_d.p;
    F.param_double = 1;
    F.energy = energy;
    F.virial = virial;
    F.heat = heat;
    hipLaunchKernelGGL(k_finalize_eval, dim3(P), dim3(256), 0, st, F);
    HIPCHECK(hipGetLastError());
    return MT_OK;
}

static int launch_grad_coef(mt_set* set, int P, const double* w, const double* Z, hipStream_t st) {
    HIPCHECK(set->zwork.reserve(sizeof(double) * 8 * (size_t)P * set->S));
    FinArgs F = make_fin(set, kNVFit, set->partial.as<double>());
    F.we = w[0]; F.wv = w[1]; F.wf = w[2];
    F.Z = const_cast<double*>(Z);
    F.coef = set->zwork.as<double>();
    hipLaunchKernelGGL(k_grad_coef, dim3(P), dim3(256), 0, st, F);
    HIPCHECK(hipGetLastError());
    return MT_OK;
}

template <typename S>
static int launch_adjoint_t(mt_set* set, const ItemPlan* plan, const LaunchCfg& cfg, int P,
                            hipStream_t st) {
    HIPCHECK(set->partial2.reserve(sizeof(double) * kNVGrad * (size_t)P * set->nslots));
    BArgs<S> A = make_args<S>(set, set->partial2.as<double>(), kNVGrad);
    A.coef = set->zwork.as<double>();
    if (plan) {
        if (plan->n_items == 0) return MT_OK;
        A.items = plan->items.as<Item>();
        A.bin_off = plan->bin_off.as<int>();
        const size_t lds = sizeof(S) == 8 ? plan->lds_d : plan->lds_f;
        hipLaunchKernelGGL((k_adjoint<S>), dim3(plan->n_bins), dim3(cfg.block), lds, st, A);
    } else {
        for (int s = 0; s < set->S; ++s) {
            const int npad = set->h_npad[s];
            const int block = std::max(64, npad);
            const size_t nbs = (size_t)(set->h_boff[s + 1] - set->h_boff[s]);
            const size_t lds = (size_t)(block / npad) * 3 * (nbs + npad) * sizeof(S);
            for (int c = 0; c < P; ++c) {
                Item it{s, c, 1, 0};
                hipLaunchKernelGGL((k_adjoint_single<S>), dim3(1), dim3(block), lds, st, A, it);
            }
        }
    }
    HIPCHECK(hipGetLastError());
    return MT_OK;
}

int launch_adjoint(mt_set* set, const ItemPlan& plan, const LaunchCfg& cfg, int P, int precision,
                   const double* w, const double* Z, hipStream_t st) {
    int rc = launch_grad_coef(set, P, w, Z, st);
    if (rc) return rc;
    return precision == MT_FP64 ? launch_adjoint_t<double>(set, &plan, cfg, P, st)
                                : launch_adjoint_t<float>(set, &plan, cfg, P, st);
}

int launch_adjoint_plain(mt_set* set, int P, int precision, const double* w, const double* Z,
                         hipStream_t st) {
    int rc = launch_grad_coef(set, P, w, Z, st);
    if (rc) return rc;
    LaunchCfg cfg;
    return precision == MT_FP64 ? launch_adjoint_t<double>(set, nullptr, cfg, P, st)
                                : launch_adjoint_t<float>(set, nullptr, cfg, P, st);
}

int launch_finalize_grad(mt_set* set, int P, const double* Z, double* dZdx, hipStream_t st) {
    (void)Z;
    FinArgs F = make_fin(set, kNVGrad, set->partial2.as<double>());
    F.params = set->params_d.p;
    F.param_double = 1;
    hipLaunchKernelGGL(k_finalize_grad, dim3(P), dim3(256), 0, st, F, dZdx);
    HIPCHECK(hipGetLastError());
    return MT_OK;
}

}  // namespace mt
