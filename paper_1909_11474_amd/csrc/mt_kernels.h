// Device code of the evaluation kernels, shared by the per-family translation
// units (each instantiates the kernels of one precision / mode).
//
// Batched kernel.  A work item is (structure s, candidates c0 .. c0+nc-1).  A
// block of B threads holds R = B / npad_s replicas of the structure (npad_s is
// the atom count rounded up to 8/16/32/64 or to a multiple of 64), one atom per
// thread; replica q evaluates candidates c0 + q, c0 + q + R, ...  At the start
// of an item the block decodes the item's parameter sets into LDS; the bond
// geometry of the thread's atom is loaded once into registers and reused for
// every candidate.  Forces need the other atom's bond gradient
// (F_i = sum_j G_ij - G_ji): every thread writes its bond gradients to its
// exchange slots in LDS and reads back the reverse bonds.  A replica of up to
// 64 atoms lives inside one wavefront, whose LDS accesses are ordered, so it
// needs no barrier; larger replicas synchronise the block.  Per-atom energy,
// virial and squared force residual are reduced in float64 over aligned lane
// groups (transpose reduction over DPP / permlane exchanges) and written to one
// partial-sum slot per (candidate, structure, wavefront); the finalize kernels
// add the slots in a fixed order, so results are deterministic.
//
// Coordination classes.  Atoms inside a structure are sorted by coordination
// and each wavefront runs the variant compiled for its largest coordination M,
// so control flow is uniform.  A kernel instance serves one class MC: it holds
// the variants M = LO..MC (a wavefront with M < LO runs the LO variant with
// padded bonds), and a structure is routed to the smallest class that covers
// its largest coordination.  Register allocation then follows the class, so
// diamond-like structures (M <= 4) run at high occupancy.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "mt_host.h"
#include "mt_site.h"

namespace mt {

// ---------------------------------------------------------------------------
// Parameter decode (Sec. II.B): x = [D0, alpha, r0, beta, n, h] with S = 2,
// so lambda = 2 alpha, mu = alpha, f_R = D0 e^{-2 alpha (r - r0)},
// f_A = 2 D0 e^{-alpha (r - r0)}.  A candidate outside the potential's domain
// is replaced by a harmless stand-in so the arithmetic stays finite; its
// outputs are set to NaN by the finalize kernels.
// ---------------------------------------------------------------------------
// Parameter vectors: minimal [D0, alpha, r0, beta, n, h]; Tersoff form
// [D0, alpha, r0, S, gamma, n, c, d, h].
template <bool Full>
struct Form {
    static constexpr int nx = Full ? 9 : 6;
};

template <bool Full>
__device__ __forceinline__ bool params_valid(const double* __restrict__ x) {
    bool fin = true;
#pragma unroll
    for (int k = 0; k < Form<Full>::nx; ++k) fin = fin && isfinite(x[k]);
    if constexpr (Full) {
        return fin && x[0] > 0.0 && x[1] > 0.0 && x[3] > 1.0 && x[4] >= 0.0 && x[5] > 0.0 &&
               x[7] != 0.0;
    } else {
        return fin && x[0] > 0.0 && x[1] > 0.0 && x[4] > 0.0 && x[3] >= 0.0;
    }
}

template <typename S>
__device__ __forceinline__ void put_split(S* __restrict__ o, int hi, int lo, double v) {
    const S h = (S)v;
    o[hi] = h;
    o[lo] = (S)(v - (double)h);
}

// x -> the record of the form-independent site routine (see ParamIndex).
template <typename S, bool Full>
__device__ __forceinline__ void decode_record(const double* __restrict__ x, S* __restrict__ o) {
    const double log2e = 1.4426950408889634;
    const bool ok = params_valid<Full>(x);
    if constexpr (Full) {
        double D0 = x[0], al = x[1], r0 = x[2], Sl = x[3], gam = x[4], n = x[5], c = x[6],
               d = x[7], h = x[8];
        if (!ok) { D0 = 3.0; al = 1.4; r0 = 2.2; Sl = 2.0; gam = 0.3; n = 0.6; c = 1.0; d = 1.0; h = -0.6; }
        const double mu = al * sqrt(2.0 / Sl), lam = al * sqrt(2.0 * Sl);
        put_split(o, P_AA, P_AALO, mu * log2e);
        put_split(o, P_AR, P_ARLO, lam * log2e);
        put_split(o, P_R0HI, P_R0LO, r0);
        put_split(o, P_DR, P_DRLO, D0 / (Sl - 1.0));
        put_split(o, P_DA, P_DALO, Sl * D0 / (Sl - 1.0));
        put_split(o, P_N, P_NLO, n);
        put_split(o, P_NINV2N, P_NINV2NLO, -1.0 / (2.0 * n));
        put_split(o, P_H, P_HLO, h);
        o[P_VALID] = ok ? S(1) : S(0);
        o[P_HMU] = (S)(0.5 * mu);
        o[P_HLAMBDA] = (S)(0.5 * lam);
        o[P_ZS] = S(1);
        o[P_CCS] = S(0.5);
        const double K = gam * c * c / (d * d);
        o[P_GAM] = (S)gam;
        o[P_K] = (S)K;
        o[P_D2] = (S)(d * d);
        o[P_KD2] = (S)(K * d * d);
    } else {
        // S = 2: mu = alpha, lambda = 2 alpha, DR = D0, DA = 2 D0.  The slots
        // that only the Tersoff form reads (P_AR, P_ARLO, P_DALO, P_HLAMBDA,
        // P_GAM .. P_KD2) are left unwritten: writing them changes the
        // register allocation of the float fitness kernel's candidate loop
        // (three more spilled values there, 4 % slower).
        double D0 = x[0], al = x[1], r0 = x[2], be = x[3], n = x[4], h = x[5];
        if (!ok) { D0 = 3.0; al = 1.4; r0 = 2.2; be = 0.3; n = 0.6; h = -0.6; }
        o[P_AA] = (S)(al * log2e);
        const S r0hi = (S)r0;
        o[P_R0HI] = r0hi;
        o[P_R0LO] = (S)(r0 - (double)r0hi);
        o[P_DR] = (S)D0;
        o[P_DA] = (S)(2.0 * D0);
        o[P_ZS] = (S)be;
        o[P_N] = (S)n;
        o[P_NINV2N] = (S)(-1.0 / (2.0 * n));
        put_split(o, P_H, P_HLO, h);
        o[P_VALID] = ok ? S(1) : S(0);
        o[P_HMU] = (S)(0.5 * al);
        o[P_CCS] = (S)(0.5 * be);
        const double aA = al * log2e, ni = -1.0 / (2.0 * n);
        o[P_AALO] = (S)(aA - (double)(S)aA);
        o[P_DRLO] = (S)(D0 - (double)(S)D0);
        o[P_NLO] = (S)(n - (double)(S)n);
        o[P_NINV2NLO] = (S)(ni - (double)(S)ni);
    }
}

template <typename S>
struct alignas(4 * sizeof(S)) Vec4 {
    S x, y, z, w;
};

template <typename S>
struct BArgs {
    SetDev set;
    const Item* items;
    const int* bin_off;
    const double* x;          // [P][6] (minimal) or [P][9] (Tersoff form) parameter sets
    double* partial;          // [P][nslots][nv]
    int nv;
    // MODE_EVAL outputs (caller numbering); may be null
    double* force;            // [P][3][N]
    double* atom_virial;      // [P][9][N]
    const double* vel;        // [3][N]
    // adjoint inputs
    const double* coef;       // [P][S][8]
    // force residuals F - F* of the batched atoms, [P][3][N] (sorted atom
    // order): written by the fitness kernel when non-null, read by the adjoint
    S* resid;
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
    int s, a0, Ns, npad, R, q, la, atom, steps, slot, g, xsz, own;
    bool active, block_sync;
};

__device__ __forceinline__ ItemCtx item_ctx(const SetDev& d, const Item& it) {
    // Item fields are uniform across the block; npad is 8, 16, 32, 64 or a
    // multiple of 64, so lane -> (replica, atom) needs no vector division.
    ItemCtx x;
    x.s = it.s;
    x.a0 = d.st_off[x.s];
    x.Ns = d.st_off[x.s + 1] - x.a0;
    x.npad = d.st_npad[x.s];
    const int tid = threadIdx.x;
    if (x.npad <= 64) {
        const int sh = 31 - __clz(x.npad);
        x.R = blockDim.x >> sh;
        x.q = tid >> sh;
        x.la = tid & (x.npad - 1);
        x.g = x.npad;
    } else {
        const int wpr = x.npad >> 6;                       // wavefronts per replica
        const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
        x.R = (blockDim.x >> 6) / wpr;
        const int qw = wid / wpr;                          // scalar division
        x.q = qw;
        x.la = ((wid - qw * wpr) << 6) + (tid & 63);
        x.g = 64;
    }
    x.active = (x.q < x.R) && (x.la < x.Ns);
    x.atom = x.a0 + (x.active ? x.la : 0);
    x.steps = (it.nc + x.R - 1) / x.R;
    x.slot = d.st_slot[x.s] + (x.npad > 64 ? (x.la >> 6) : 0);
    x.xsz = d.st_xsize[x.s];
    x.block_sync = x.npad > 64;
    // own exchange slot base: the chunk's first atom is always a real atom
    const int first = x.la & ~(x.g - 1);
    x.own = (x.q < x.R) ? (d.xbase[x.a0 + first] + (x.la - first) + x.q * x.xsz) : 0;
    return x;
}

// LDS ordering: a replica inside one wavefront only needs the compiler not to
// move LDS accesses across this point; larger replicas need the block barrier.
__device__ __forceinline__ void exchange_sync(bool block) {
    if (block) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Store the group sums of v[0..7] into partial[c][slot][off + vidx].  GF is
// the group size when known at compile time (0: x.g at run time).
template <int GF = 0>
__device__ __forceinline__ void store_group(double* v, const ItemCtx& x, bool group_ok,
                                            double* __restrict__ partial, int nslots, int nv,
                                            int c, int off, int wmask) {
    int vidx;
    const double sum = GF ? group_reduce8_t<(GF ? GF : 64)>(v, &vidx) : group_reduce8(v, x.g, &vidx);
    const int lane = threadIdx.x & 63;
    if (group_ok && (lane & ((x.g >> 3) - 1)) == 0 && ((wmask >> vidx) & 1))
        partial[((size_t)c * nslots + x.slot) * nv + off + vidx] = sum;
}

// LDS layout of a block while it works on an item: [it.nc x kNParam parameter
// records][R x xsz exchange slots (Vec4)][adjoint: R x npad force residuals
// (Vec4)].  The exchange follows the item's own records, so the LDS a launch
// gets for the largest (records + exchange) of its structures covers every
// item, whatever the candidate tiles of the other structures in the launch.
template <typename S>
__device__ __forceinline__ size_t lds_param_bytes(int nc) {
    return ((size_t)nc * kNParam * sizeof(S) + 31) & ~(size_t)31;
}

// Resid (fitness mode): also write each atom's force residual to A.resid (the
// gradient's fitness call; a separate instance, so the fitness alone carries
// no trace of it).
template <typename S, int MODE, int M, int GF = 0, bool Full = false, bool Resid = false>
__device__ __forceinline__ void run_batched(const BArgs<S>& A, const Item& it, const ItemCtx& x,
                                            unsigned char* __restrict__ lds) {
    const SetDev& d = A.set;
    const int N = d.N;
    const S* __restrict__ pbuf = reinterpret_cast<const S*>(lds);
    Vec4<S>* __restrict__ xb = reinterpret_cast<Vec4<S>*>(lds + lds_param_bytes<S>(it.nc));
    Geo<S, M> g;
    g.load(geom_of<S>(d), N, x.atom, x.active, d.gcs);
    constexpr int MM = M > 0 ? M : 1;
    int rv[MM];
#pragma unroll
    for (int m = 0; m < M; ++m)
        rv[m] = x.active ? d.rev[(size_t)m * N + x.atom] + x.q * x.xsz : x.own + m * x.g;
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

    for (int step = 0; step < x.steps; ++step) {
        const int cl = x.q + step * x.R;
        const bool group_ok = cl < it.nc;
        const bool cok = x.active && group_ok;
        const int clv = group_ok ? cl : 0;
        const int c = it.c0 + clv;
        Cand<S, S, Full> p;
        load_cand(pbuf + kNParam * clv, p);
        // Each bond gradient G_j goes to its exchange slot as soon as the site
        // routine emits it and is folded into this atom's own force sum and
        // the virial, so no bond-gradient array stays live across the exchange.
        double U;
        S Fx = S(0), Fy = S(0), Fz = S(0);
        S w6[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) w6[k] = S(0);
        site_eval_sink<S, S, M, true, (M > kPairwiseMax), false, Full>(
            g, p, U, [&](int m, S gx, S gy, S gz) {
                S* slot = &xb[x.own + m * x.g].x;     // the fourth component is never read
                slot[0] = gx;
                slot[1] = gy;
                slot[2] = gz;
                Fx += gx; Fy += gy; Fz += gz;
                const S dx = g.rhi[m] * g.ux[m], dy = g.rhi[m] * g.uy[m], dz = g.rhi[m] * g.uz[m];
                w6[0] -= dx * gx; w6[1] -= dy * gy; w6[2] -= dz * gz;
                w6[3] -= dy * gz; w6[4] -= dz * gx; w6[5] -= dx * gy;
            });
        exchange_sync(x.block_sync);
        S wi[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) wi[k] = S(0);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const Vec4<S> r = xb[rv[m]];
            Fx -= r.x;
            Fy -= r.y;
            Fz -= r.z;
            if (MODE == MODE_EVAL) {
                const S dx = g.rhi[m] * g.ux[m], dy = g.rhi[m] * g.uy[m], dz = g.rhi[m] * g.uz[m];
                wi[0] += dx * r.x; wi[1] += dx * r.y; wi[2] += dx * r.z;
                wi[3] += dy * r.x; wi[4] += dy * r.y; wi[5] += dy * r.z;
                wi[6] += dz * r.x; wi[7] += dz * r.y; wi[8] += dz * r.z;
            }
        }
        exchange_sync(x.block_sync);
        // Lanes outside the structure have zero geometry and zero reference
        // forces, so their energy, virial and residual are exactly zero.
        double v[8];
        v[0] = (double)U;
#pragma unroll
        for (int k = 0; k < 6; ++k) v[1 + k] = (double)w6[k];
        if (MODE == MODE_FIT) {
            const S ax = Fx - frx, ay = Fy - fry, az = Fz - frz;
            v[7] = (double)(ax * ax + ay * ay + az * az);
            if (Resid && cok) {
                S* r = A.resid + (size_t)c * 3 * N;
                r[x.atom] = ax;
                r[(size_t)N + x.atom] = ay;
                r[(size_t)2 * N + x.atom] = az;
            }
            store_group<GF>(v, x, group_ok, A.partial, d.nslots, A.nv, c, 0, 0xff);
        } else {
            v[7] = 0.0;
            store_group<GF>(v, x, group_ok, A.partial, d.nslots, A.nv, c, 0, 0xff);
            double u[8];
            const S jx = wi[0] * vx + wi[1] * vy + wi[2] * vz;
            const S jy = wi[3] * vx + wi[4] * vy + wi[5] * vz;
            const S jz = wi[6] * vx + wi[7] * vy + wi[8] * vz;
            u[0] = (double)jx;
            u[1] = (double)jy;
            u[2] = (double)jz;
            u[3] = u[4] = u[5] = u[6] = u[7] = 0.0;
            store_group<GF>(u, x, group_ok, A.partial, d.nslots, A.nv, c, 8, 0x07);
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

__device__ __forceinline__ void run_idle(int steps, int barriers) {
    for (int step = 0; step < steps; ++step)
        for (int b = 0; b < barriers; ++b) __syncthreads();
}

// Call f(integral_constant<M>) for the variant that serves coordination m.
template <int LO, int HI, typename F>
__device__ __forceinline__ void dispatch_m(int m, F&& f) {
    if constexpr (LO >= HI) {
        f(std::integral_constant<int, HI>{});
    } else {
        if (m <= LO) f(std::integral_constant<int, LO>{});
        else dispatch_m<LO + 1, HI>(m, f);
    }
}

// Lowest compiled variant of a class; the exchange-slot layout of the set
// reserves at least this many slots per atom for structures of the class.
template <int MC>
struct ClassLo {
    static constexpr int value = MC <= 4 ? 0 : 3;
};

// Decode the item's parameter sets into the LDS records (all threads take part).
template <typename S, bool Full = false>
__device__ __forceinline__ void decode_item(const BArgs<S>& A, const Item& it, unsigned char* lds) {
    S* pbuf = reinterpret_cast<S*>(lds);
    for (int t = threadIdx.x; t < it.nc; t += blockDim.x)
        decode_record<S, Full>(A.x + Form<Full>::nx * (size_t)(it.c0 + t), pbuf + kNParam * t);
    __syncthreads();
}

template <typename S, int MODE, int MC, bool Full, bool Resid = false>
__device__ __forceinline__ void batched_item(const BArgs<S>& A, const Item& it, unsigned char* lds) {
    decode_item<S, Full>(A, it, lds);
    const ItemCtx x = item_ctx(A.set, it);
    const int Mi = x.active ? A.set.nnb[x.atom] : -1;
    const int Mw = wave_max_int(Mi);
    if (Mw < 0) {
        // whole wavefront outside every replica: only larger replicas have such
        // wavefronts, and they synchronise the block twice per step
        run_idle(x.steps, 2);
        return;
    }
    dispatch_m<ClassLo<MC>::value, MC>(Mw, [&](auto mv) {
        // the float fitness kernel of the minimal potential gets a copy with
        // 64-lane groups (structures of 64 atoms or more) fixed at compile
        // time: the reduction then needs no branches and no copies around the
        // in-place lane swaps
        if constexpr (MODE == MODE_FIT && sizeof(S) == 4 && !Full) {
            if (x.g == 64) {
                run_batched<S, MODE, decltype(mv)::value, 64, Full, Resid>(A, it, x, lds);
                return;
            }
        }
        run_batched<S, MODE, decltype(mv)::value, 0, Full, Resid>(A, it, x, lds);
    });
}

// Occupancy target per class: the float fitness kernel of the M <= 4 class
// fits 4 wavefronts per SIMD (128 registers).
template <typename S, int MODE, int MC>
struct WavesPerEU {
    static constexpr int value = (MC <= 4 && sizeof(S) == 4 && MODE == MODE_FIT) ? 4 : 1;
};

template <typename S, int MODE, int MC, bool Full = false, bool Resid = false>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(WavesPerEU<S, MODE, MC>::value)))
void k_batched(BArgs<S> A) {
    extern __shared__ __align__(32) unsigned char lds_raw[];
    const int b0 = A.bin_off[blockIdx.x], b1 = A.bin_off[blockIdx.x + 1];
    for (int i = b0; i < b1; ++i) {
        const Item it = A.items[i];
        batched_item<S, MODE, MC, Full, Resid>(A, it, lds_raw);
        __syncthreads();
    }
}

// The plain schedule: one launch per (candidate, structure), a single block
// that evaluates the item A.items[0].  The same device code as k_batched,
// under a kernel name of its own so that profiles keep the two apart.
template <typename S, int MODE, int MC, bool Full = false>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(WavesPerEU<S, MODE, MC>::value)))
void k_plain(BArgs<S> A) {
    extern __shared__ __align__(32) unsigned char lds_raw[];
    batched_item<S, MODE, MC, Full>(A, A.items[0], lds_raw);
}

// ---------------------------------------------------------------------------
// Adjoint kernel: dZ/dx of the fitness.  For candidate c and structure s,
//   dZ/dx|_s = sum_i [ k_e U_i' - sum_j G_ij' . delta_ij ],
//   delta_ij = k_f (a_j - a_i) + C_s r_ij,   a = F - F*,
// where ' is the derivative with respect to the parameters (six, or nine for
// the Tersoff form; forward-mode dual numbers), k_e = w_e (e_s - e*_s)/(N_s Z_e Q_e), k_f = w_f/(Z_f Q_f) and
// C_s = w_v/(N_s Z_v Q_v) times the symmetric matrix of virial residuals (off
// diagonals halved).  These follow from dF_i/dx = -d/dx dE/dr_i and
// dW/dx = -sum r_ij (x) dG_ij/dx.
//
// Per candidate: a plain pass gives the force residuals a_i, shared through
// LDS; then dual passes over K of the parameters at a time contract each
// G_ij' with delta_ij as soon as the site routine emits it, so no bond
// gradient derivative is held across the exchange.
// ---------------------------------------------------------------------------

// Tangents per dual pass: six for small coordination (one pass for the six
// minimal parameters; six and three for the nine of the Tersoff form), three
// where six would not fit in registers.
template <typename S, int M>
struct AdjointTangents {
    static constexpr int value = (M <= 4 && sizeof(S) == 4) ? 6 : 3;
};

// pass(Base, K') for consecutive blocks of at most K of the NX parameters.
template <int Base, int NX, int K, typename F>
__device__ __forceinline__ void for_passes(F&& pass) {
    if constexpr (Base < NX) {
        constexpr int KK = (NX - Base) < K ? (NX - Base) : K;
        pass(std::integral_constant<int, Base>{}, std::integral_constant<int, KK>{});
        for_passes<Base + KK, NX, K>(pass);
    }
}

// The parameter derivatives of one atom's site terms contracted with its
// residual directions: phi[p] = k_e dU_i/dx_p - sum_j dG_ij/dx_p . delta_ij,
// delta_ij = k_f (a_j - a_i) + C_s r_ij, by dual passes over KK parameters at a
// time.  rec: the candidate's decoded record, xrow its parameters (Tersoff
// form), (ax, ay, az) this atom's force residual, aj(m) the residual of the
// atom at the far end of bond m, cf the coefficients k_e, k_f, C_s (xx yy zz yz
// zx xy, off-diagonals halved) of the (candidate, structure).
template <typename S, int M, bool Full, typename Aj>
__device__ __forceinline__ void adjoint_phi(Geo<S, M>& g, const S* __restrict__ rec,
                                            const double* __restrict__ xrow, S ax, S ay, S az,
                                            Aj&& aj, const double* __restrict__ cf,
                                            S (&phi)[Form<Full>::nx]) {
    constexpr int K = AdjointTangents<S, M>::value;
    constexpr int NX = Form<Full>::nx;
    const S ke = (S)cf[0], kf = (S)cf[1];
    const S cxx = (S)cf[2], cyy = (S)cf[3], czz = (S)cf[4];
    const S cyz = (S)cf[5], czx = (S)cf[6], cxy = (S)cf[7];
    auto pass = [&](auto base_c, auto k_c) {
        constexpr int Base = decltype(base_c)::value;
        constexpr int KK = decltype(k_c)::value;
        Cand<Dual<S, KK>, S, Full> p;
        if constexpr (Full) load_cand<Base>(rec, xrow, p);
        else load_cand<Base>(rec, p);
        Dual<S, KK> U;
        site_eval_sink<Dual<S, KK>, S, M, false, true, true>(
            g, p, U, [&](int m, const Dual<S, KK>& gx, const Dual<S, KK>& gy, const Dual<S, KK>& gz) {
                const Vec4<S> a = aj(m);
                const S dx = g.rhi[m] * g.ux[m], dy = g.rhi[m] * g.uy[m], dz = g.rhi[m] * g.uz[m];
                const S ex = kf * (a.x - ax) + cxx * dx + cxy * dy + czx * dz;
                const S ey = kf * (a.y - ay) + cxy * dx + cyy * dy + cyz * dz;
                const S ez = kf * (a.z - az) + czx * dx + cyz * dy + czz * dz;
#pragma unroll
                for (int t = 0; t < KK; ++t) phi[Base + t] -= gx.d[t] * ex + gy.d[t] * ey + gz.d[t] * ez;
            });
#pragma unroll
        for (int t = 0; t < KK; ++t) phi[Base + t] += ke * U.d[t];
    };
#pragma unroll
    for (int k = 0; k < NX; ++k) phi[k] = S(0);
    for_passes<0, NX, K>(pass);
}

template <typename S, int M, bool Full = false>
__device__ __forceinline__ void run_adjoint(const BArgs<S>& A, const Item& it, const ItemCtx& x,
                                            unsigned char* __restrict__ lds) {
    const SetDev& d = A.set;
    const int N = d.N;
    const S* __restrict__ pbuf = reinterpret_cast<const S*>(lds);
    Vec4<S>* __restrict__ xb = reinterpret_cast<Vec4<S>*>(lds + lds_param_bytes<S>(it.nc));
    Vec4<S>* __restrict__ ab = xb + (size_t)x.R * x.xsz + (size_t)x.q * x.npad;
    Geo<S, M> g;
    g.load(geom_of<S>(d), N, x.atom, x.active);
    constexpr int MM = M > 0 ? M : 1;
    constexpr int NX = Form<Full>::nx;
    int jl[MM];
#pragma unroll
    for (int m = 0; m < M; ++m) jl[m] = x.active ? d.jl[(size_t)m * N + x.atom] : x.la;

    for (int step = 0; step < x.steps; ++step) {
        const int cl = x.q + step * x.R;
        const bool group_ok = cl < it.nc;
        const int clv = group_ok ? cl : 0;
        const int c = it.c0 + clv;
        const S* prec = pbuf + kNParam * clv;
        // this atom's force residual, from the fitness call (lanes outside the
        // structure: zero, and zero geometry)
        S ax = S(0), ay = S(0), az = S(0);
        if (x.active) {
            const S* r = A.resid + (size_t)c * 3 * N;
            ax = r[x.atom]; ay = r[(size_t)N + x.atom]; az = r[(size_t)2 * N + x.atom];
        }
        ab[x.la] = Vec4<S>{ax, ay, az, S(0)};
        exchange_sync(x.block_sync);
        S phi[NX];
        adjoint_phi<S, M, Full>(
            g, prec, A.x + (size_t)NX * c, ax, ay, az,
            [&](int m) {
                // a fresh read in every pass (a reused one would stay live across passes)
                int jm = jl[m];
                asm volatile("" : "+v"(jm));
                return ab[jm];
            },
            A.coef + ((size_t)c * d.S + x.s) * 8, phi);
        exchange_sync(x.block_sync);
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = k < NX ? (double)phi[k < NX ? k : 0] : 0.0;
        store_group(v, x, group_ok, A.partial, d.nslots, A.nv, c, 0, Full ? 0xff : 0x3f);
        if constexpr (Full) {
            double u[8];
            u[0] = (double)phi[8];
#pragma unroll
            for (int k = 1; k < 8; ++k) u[k] = 0.0;
            store_group(u, x, group_ok, A.partial, d.nslots, A.nv, c, 8, 0x01);
        }
    }
}

template <typename S, int MC, bool Full>
__device__ __forceinline__ void adjoint_item(const BArgs<S>& A, const Item& it, unsigned char* lds) {
    decode_item<S, Full>(A, it, lds);
    const ItemCtx x = item_ctx(A.set, it);
    const int Mi = x.active ? A.set.nnb[x.atom] : -1;
    const int Mw = wave_max_int(Mi);
    if (Mw < 0) {
        run_idle(x.steps, 2);
        return;
    }
    dispatch_m<ClassLo<MC>::value, MC>(Mw, [&](auto mv) {
        run_adjoint<S, decltype(mv)::value, Full>(A, it, x, lds);
    });
}

template <typename S, int MC, bool Full = false>
__global__ __launch_bounds__(512) void k_adjoint(BArgs<S> A) {
    extern __shared__ __align__(32) unsigned char lds_raw[];
    const int b0 = A.bin_off[blockIdx.x], b1 = A.bin_off[blockIdx.x + 1];
    for (int i = b0; i < b1; ++i) {
        const Item it = A.items[i];
        adjoint_item<S, MC, Full>(A, it, lds_raw);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Large structures (more atoms than one block holds): two passes per
// candidate.  Pass 1 writes every bond gradient to global memory and the
// energy/virial partials; pass 2 gathers forces, per-atom virial, heat
// current and the force residual.
// ---------------------------------------------------------------------------
// One staged bond gradient of the two-pass path: x, y, z and an unused
// fourth value, so that the gather reads a partner's reverse bond with one
// vector load (one cache line) instead of three scattered ones.
template <typename S>
struct Stage4;
template <>
struct Stage4<float> {
    using T = float4;
};
template <>
struct Stage4<double> {
    using T = double4;
};

struct LArgs {
    int s, c0;                 // structure, first candidate of the chunk
    void* gbuf;                // [chunk][nbs] of Stage4<S> (x, y, z, unused)
    // 1: the structure has one partial-sum slot per block (a structure over
    // the batching limit); 0: one per wavefront (a batched structure sent to
    // the two-pass path)
    int per_block;
    // the structure's first atom, atom count, bond count, first partial-sum
    // slot and largest coordination, copied from the host tables so no kernel
    // waits on reading them
    int a0, ns, nbs, slot0, kmax;
};

// Store a wavefront's group sums (lanes with (lane & 7) == 0 hold value vidx)
// in the structure's partial-sum slots, values off + k for the k set in mask:
// per wavefront (wavefronts past the structure, wave_in false, write
// nothing), or per block, the block's wavefront sums added in wavefront order
// through LDS.  Every thread of the block calls it; a wavefront with no atom
// passes sum = 0 and vidx = (lane >> 3).
__device__ __forceinline__ void large_store(const SetDev& d, const LArgs& L, double* __restrict__ partial,
                                            int nv, int c, int la, bool wave_in, double sum, int vidx,
                                            unsigned mask, int off, double (*sh)[8]) {
    const int lane = threadIdx.x & 63;
    if (!L.per_block) {
        if (wave_in && (lane & 7) == 0 && ((mask >> vidx) & 1))
            partial[((size_t)c * d.nslots + L.slot0 + (la >> 6)) * nv + off + vidx] = sum;
        return;
    }
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((lane & 7) == 0) sh[w][vidx] = sum;
    __syncthreads();
    const int k = threadIdx.x;
    if (k < 8 && ((mask >> k) & 1)) {
        double t = sh[0][k];
        for (int q = 1; q < nw; ++q) t += sh[q][k];
        partial[((size_t)c * d.nslots + L.slot0 + blockIdx.x) * nv + off + k] = t;
    }
    __syncthreads();
}

template <typename S, int M, bool E64, bool Full>
__device__ __forceinline__ void run_large_site(const BArgs<S>& A, const LArgs& L, int la, int atom,
                                               bool active, double& sum, int& vidx, int rows = M) {
    const SetDev& d = A.set;
    const int N = d.N;
    Geo<S, M> g;
    g.load(geom_of<S>(d), N, atom, active, d.gcs, rows);
    constexpr int MM = M > 0 ? M : 1;
    const int c = L.c0 + blockIdx.y;
    const int nbs = L.nbs;
    const int Mi = active ? d.nnb[atom] : 0;
    const int lb = active ? d.lbo[atom] : 0;
    S rec[kNParam];
    decode_record<S, Full>(A.x + Form<Full>::nx * (size_t)c, rec);
    Cand<S, S, Full> p;
    load_cand(rec, p);
    double U;
    S Gx[MM], Gy[MM], Gz[MM];
    // about one wavefront per SIMD for a large structure: the bonds' float64
    // energy chains interleave
    site_eval<S, S, M, E64, Full, false>(g, p, U, Gx, Gy, Gz);
    using V4 = typename Stage4<S>::T;
    V4* gb = reinterpret_cast<V4*>(L.gbuf) + (size_t)blockIdx.y * nbs;
    if (active) {
#pragma unroll
        for (int m = 0; m < M; ++m)
            if (m < Mi) gb[lb + m] = V4{Gx[m], Gy[m], Gz[m], S(0)};
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
    sum = group_reduce8(v, 64, &vidx);
}

// E64: float64 energy terms (the float path's energy/force/virial mode).
template <typename S, int MC, bool E64, bool Full = false>
__global__ __launch_bounds__(256) void k_large_site(BArgs<S> A, LArgs L) {
    const SetDev& d = A.set;
    const int a0 = L.a0, Ns = L.ns;
    const int la = blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = la < Ns;
    const int atom = a0 + (active ? la : 0);
    __shared__ double sh[kLargeBlock / 64][8];
    double sum = 0.0;
    int vidx = (threadIdx.x & 63) >> 3;
    bool wave_in;
    if constexpr (MC <= 4) {
        // one variant for the class: the geometry rows (up to the structure's
        // largest coordination) are read without first waiting for the
        // wavefront's bond counts
        wave_in = (la & ~63) < Ns;
        if (wave_in) run_large_site<S, MC, E64, Full>(A, L, la, atom, active, sum, vidx, L.kmax);
    } else {
        const int Mi = active ? d.nnb[atom] : -1;
        const int Mw = wave_max_int(Mi);
        wave_in = Mw >= 0;
        if (wave_in)
            dispatch_m<ClassLo<MC>::value, MC>(Mw, [&](auto mv) {
                run_large_site<S, decltype(mv)::value, E64, Full>(A, L, la, atom, active, sum, vidx);
            });
    }
    // no partial sums when only the staged bond gradients are wanted
    if (A.partial)
        large_store(d, L, A.partial, A.nv, L.c0 + blockIdx.y, la, wave_in, sum, vidx, 0x7f, 0, sh);
}

template <typename S, int MODE, int MC>
__global__ __launch_bounds__(256) void k_large_gather(BArgs<S> A, LArgs L) {
    const SetDev& d = A.set;
    const int N = d.N;
    const int a0 = L.a0, Ns = L.ns;
    const int nbs = L.nbs;
    const int la = blockIdx.x * blockDim.x + threadIdx.x;
    // wavefronts past the structure own no per-wavefront slot; they still take
    // part in a block's sums (with zeros)
    const bool wave_in = (la & ~63) < Ns;
    const bool active = la < Ns;
    __shared__ double sh[kLargeBlock / 64][8];
    const int atom = a0 + (active ? la : 0);
    const int c = L.c0 + blockIdx.y;
    using V4 = typename Stage4<S>::T;
    const V4* gb = reinterpret_cast<const V4*>(L.gbuf) + (size_t)blockIdx.y * nbs;
    const GeomArrays<S> G = geom_of<S>(d);
    // The reverse-bond indices (rows up to the structure's largest
    // coordination) are read in the same memory round trip as the atom's
    // bond count; the staged gradients of its bonds in the next.
    const int rows = L.kmax < MC ? L.kmax : MC;
    int rv[MC];
#pragma unroll
    for (int m = 0; m < MC; ++m) rv[m] = active && m < rows ? d.revc[(size_t)m * N + atom] : 0;
    const int Mi = active ? d.nnb[atom] : 0, lb = active ? d.lbo[atom] : 0;
    S Fx = S(0), Fy = S(0), Fz = S(0);
    S wi[9];
    for (int k = 0; k < 9; ++k) wi[k] = S(0);
#pragma unroll
    for (int m = 0; m < MC; ++m) {
        if (m >= Mi) break;
        const size_t o = (size_t)m * N + atom;
        const int r = rv[m];
        const V4 rg = gb[r], og = gb[lb + m];
        const S rx = rg.x, ry = rg.y, rz = rg.z;
        Fx += og.x - rx;
        Fy += og.y - ry;
        Fz += og.z - rz;
        if (MODE == MODE_EVAL) {
            const S rr = G.rhi[o];
            const S dx = rr * G.ux[o], dy = rr * G.uy[o], dz = rr * G.uz[o];
            wi[0] += dx * rx; wi[1] += dx * ry; wi[2] += dx * rz;
            wi[3] += dy * rx; wi[4] += dy * ry; wi[5] += dy * rz;
            wi[6] += dz * rx; wi[7] += dz * ry; wi[8] += dz * rz;
        }
    }
    const int orig = active ? d.perm[atom] : 0;
    double v[8];
    for (int k = 0; k < 8; ++k) v[k] = 0.0;
    int vidx;
    if (MODE == MODE_FIT) {
        const S* fr = fref_of<S>(d);
        if (active) {
            const S ax = Fx - fr[atom], ay = Fy - fr[(size_t)N + atom], az = Fz - fr[(size_t)2 * N + atom];
            v[7] = (double)(ax * ax + ay * ay + az * az);
        }
        const double sum = group_reduce8(v, 64, &vidx);
        large_store(d, L, A.partial, A.nv, c, la, wave_in, sum, vidx, 0x80, 0, sh);
    } else {
        if (active && A.vel) {
            const S vx = (S)A.vel[orig], vy = (S)A.vel[(size_t)N + orig], vz = (S)A.vel[(size_t)2 * N + orig];
            v[0] = (double)(wi[0] * vx + wi[1] * vy + wi[2] * vz);
            v[1] = (double)(wi[3] * vx + wi[4] * vy + wi[5] * vz);
            v[2] = (double)(wi[6] * vx + wi[7] * vy + wi[8] * vz);
        }
        const double sum = group_reduce8(v, 64, &vidx);
        large_store(d, L, A.partial, A.nv, c, la, wave_in, sum, vidx, 0x07, 8, sh);
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
// Fitness gradient of the two-pass structures.  k_large_site stages the bond
// gradients of a candidate chunk (as for the fitness), k_large_residual turns
// them into the force residuals a_i = F_i - F*_i, staged [chunk][3][Ns], and
// k_large_adjoint runs the dual passes of every atom (adjoint_phi) with the
// residuals of its bond partners read from there; its partial sums go to the
// structure's per-wavefront slots as in the batched adjoint.
// ---------------------------------------------------------------------------
template <typename S>
__global__ __launch_bounds__(256) void k_large_residual(BArgs<S> A, LArgs L, S* __restrict__ abuf) {
    const SetDev& d = A.set;
    const int N = d.N;
    const int a0 = L.a0, Ns = L.ns;
    const int nbs = L.nbs;
    const int la = blockIdx.x * blockDim.x + threadIdx.x;
    if (la >= Ns) return;
    const int atom = a0 + la;
    using V4 = typename Stage4<S>::T;
    const V4* gb = reinterpret_cast<const V4*>(L.gbuf) + (size_t)blockIdx.y * nbs;
    S Fx = S(0), Fy = S(0), Fz = S(0);
    const int Mi = d.nnb[atom], lb = d.lbo[atom];
    for (int m = 0; m < Mi; ++m) {
        const int r = d.revc[(size_t)m * N + atom];
        const V4 rg = gb[r], og = gb[lb + m];
        Fx += og.x - rg.x;
        Fy += og.y - rg.y;
        Fz += og.z - rg.z;
    }
    const S* fr = fref_of<S>(d);
    S* a = abuf + (size_t)blockIdx.y * 3 * Ns;
    a[la] = Fx - fr[atom];
    a[Ns + la] = Fy - fr[(size_t)N + atom];
    a[2 * Ns + la] = Fz - fr[(size_t)2 * N + atom];
}

template <typename S, int M, bool Full>
__device__ __forceinline__ void run_large_adjoint(const BArgs<S>& A, const LArgs& L, int la, int atom,
                                                  bool active, int Ns, const S* __restrict__ abuf,
                                                  double& sum, int& vidx, double& sum2, int& vidx2) {
    const SetDev& d = A.set;
    const int N = d.N;
    constexpr int MM = M > 0 ? M : 1;
    constexpr int NX = Form<Full>::nx;
    Geo<S, M> g;
    g.load(geom_of<S>(d), N, atom, active, nullptr, d.kcap);
    int jl[MM];
#pragma unroll
    for (int m = 0; m < M; ++m) jl[m] = (active && m < d.kcap) ? d.jl[(size_t)m * N + atom] : 0;
    const int c = L.c0 + blockIdx.y;
    S rec[kNParam];
    decode_record<S, Full>(A.x + (size_t)NX * c, rec);
    const S* a = abuf + (size_t)blockIdx.y * 3 * Ns;
    const S ax = active ? a[la] : S(0), ay = active ? a[Ns + la] : S(0), az = active ? a[2 * Ns + la] : S(0);
    S phi[NX];
    // lanes past the structure have zero geometry: phi = 0
    adjoint_phi<S, M, Full>(
        g, rec, A.x + (size_t)NX * c, ax, ay, az,
        [&](int m) {
            int jm = jl[m];
            asm volatile("" : "+v"(jm));
            return Vec4<S>{a[jm], a[Ns + jm], a[2 * Ns + jm], S(0)};
        },
        A.coef + ((size_t)c * d.S + L.s) * 8, phi);
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = k < NX ? (double)phi[k < NX ? k : 0] : 0.0;
    sum = group_reduce8(v, 64, &vidx);
    if constexpr (Full) {
        double u[8];
        u[0] = (double)phi[8];
#pragma unroll
        for (int k = 1; k < 8; ++k) u[k] = 0.0;
        sum2 = group_reduce8(u, 64, &vidx2);
    }
}

template <typename S, int MC, bool Full>
__global__ __launch_bounds__(256) void k_large_adjoint(BArgs<S> A, LArgs L, const S* __restrict__ abuf) {
    const SetDev& d = A.set;
    const int a0 = L.a0, Ns = L.ns;
    const int la = blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = la < Ns;
    const int atom = a0 + (active ? la : 0);
    const int Mi = active ? d.nnb[atom] : -1;
    const int Mw = wave_max_int(Mi);
    __shared__ double sh[kLargeBlock / 64][8];
    double sum = 0.0, sum2 = 0.0;
    int vidx = (threadIdx.x & 63) >> 3, vidx2 = vidx;
    auto run = [&](auto mv) {
        run_large_adjoint<S, decltype(mv)::value, Full>(A, L, la, atom, active, Ns, abuf, sum, vidx, sum2, vidx2);
    };
    if (Mw >= 0) {                              // a wavefront with no atom adds zeros
        if constexpr (MC <= 4) {
            dispatch_m<0, MC>(Mw, run);
        } else {
            // two variants only: the dual passes of a wide variant take minutes to
            // compile, and rows past the wave's coordination are padding bonds
            if (Mw <= 8) run(std::integral_constant<int, 8>{});
            else run(std::integral_constant<int, MC>{});
        }
    }
    constexpr int NX = Form<Full>::nx;
    const int c = L.c0 + blockIdx.y;
    large_store(d, L, A.partial, A.nv, c, la, Mw >= 0, sum, vidx, (1u << (NX < 8 ? NX : 8)) - 1, 0, sh);
    if constexpr (Full) large_store(d, L, A.partial, A.nv, c, la, Mw >= 0, sum2, vidx2, 0x01, 8, sh);
}

// Launchers, one per kernel family (defined in the mt_k_*.hip units).
hipError_t launch_fit32(int mc, dim3 g, dim3 b, size_t lds, hipStream_t st, const BArgs<float>& A,
                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_eval32(int mc, dim3 g, dim3 b, size_t lds, hipStream_t st, const BArgs<float>& A,
                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_fit64(int mc, dim3 g, dim3 b, size_t lds, hipStream_t st, const BArgs<double>& A,
                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_eval64(int mc, dim3 g, dim3 b, size_t lds, hipStream_t st, const BArgs<double>& A,
                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_adj32(int mc, dim3 g, dim3 b, size_t lds, hipStream_t st, const BArgs<float>& A,
                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_adj64(int mc, dim3 g, dim3 b, size_t lds, hipStream_t st, const BArgs<double>& A,
                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_adj32f(int mc, dim3 g, dim3 b, size_t lds, hipStream_t st, const BArgs<float>& A,
                         hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_adj64f(int mc, dim3 g, dim3 b, size_t lds, hipStream_t st, const BArgs<double>& A,
                         hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// The fitness kernels that also write the force residuals (A.resid), for the
// gradient's fitness call; the launch_fit* launchers pick them when A.resid
// is set.
hipError_t launch_fitr32(int mc, int full, dim3 g, dim3 b, size_t lds, hipStream_t st,
                         const BArgs<float>& A, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_fitr64(int mc, int full, dim3 g, dim3 b, size_t lds, hipStream_t st,
                         const BArgs<double>& A, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_fitr32f(int mc, dim3 g, dim3 b, size_t lds, hipStream_t st, const BArgs<float>& A,
                          hipEvent_t e0, hipEvent_t e1);
// Tersoff-form (nine-parameter) batched families.
hipError_t launch_fit32f(int mc, dim3 g, dim3 b, size_t lds, hipStream_t st, const BArgs<float>& A,
                         hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_eval32f(int mc, dim3 g, dim3 b, size_t lds, hipStream_t st, const BArgs<float>& A,
                          hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_fit64f(int mc, dim3 g, dim3 b, size_t lds, hipStream_t st, const BArgs<double>& A,
                         hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_eval64f(int mc, dim3 g, dim3 b, size_t lds, hipStream_t st, const BArgs<double>& A,
                          hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Plain-schedule launchers (one block, one item); mode is MODE_FIT or MODE_EVAL,
// full selects the Tersoff form.
hipError_t launch_plain32(int mode, bool full, int mc, dim3 b, size_t lds, hipStream_t st,
                          const BArgs<float>& A);
hipError_t launch_plain64(int mode, bool full, int mc, dim3 b, size_t lds, hipStream_t st,
                          const BArgs<double>& A);
hipError_t launch_plain32f(int mode, int mc, dim3 b, size_t lds, hipStream_t st, const BArgs<float>& A);
hipError_t launch_plain64f(int mode, int mc, dim3 b, size_t lds, hipStream_t st, const BArgs<double>& A);
hipError_t launch_large32(int mc, int mode, int full, dim3 g, dim3 b, hipStream_t st,
                          const BArgs<float>& A, const LArgs& L);
hipError_t launch_large64(int mc, int mode, int full, dim3 g, dim3 b, hipStream_t st,
                          const BArgs<double>& A, const LArgs& L);
// Two-pass fitness gradient of one structure and candidate chunk: force
// residuals into abuf from the bond gradients staged by launch_large* in
// MODE_STAGE, then the dual passes.
hipError_t launch_large_adj32(int mc, int full, dim3 g, dim3 b, hipStream_t st, const BArgs<float>& Afit,
                              const BArgs<float>& Aadj, const LArgs& L, float* abuf);
hipError_t launch_large_adj64(int mc, int full, dim3 g, dim3 b, hipStream_t st, const BArgs<double>& Afit,
                              const BArgs<double>& Aadj, const LArgs& L, double* abuf);
// The Tersoff form's residual and dual-pass kernels of the two-pass gradient.
hipError_t launch_large_adj32f(int mc, dim3 g, dim3 b, hipStream_t st, const BArgs<float>& A,
                               const LArgs& L, float* abuf);
hipError_t launch_large_adj64f(int mc, dim3 g, dim3 b, hipStream_t st, const BArgs<double>& A,
                               const LArgs& L, double* abuf);

}  // namespace mt
