// Host side of the evaluation path: parameter decode, work lists per
// coordination class (batched, persistent LPT bins, or one item per launch for
// the plain path), launches of the kernel families of mt_kernels.h, and the
// finalize kernels that turn per-slot partial sums into energies, virials, Z
// and dZ/dx in a fixed summation order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <queue>
#include <string>
#include <vector>

#include "mt_kernels.h"

namespace mt {

#define HIPCHECK(call)                                   \
    do {                                                 \
        hipError_t _e = (call);                          \
        if (_e != hipSuccess) return hip_fail(_e, #call); \
    } while (0)
#define TRY_RC(call)                  \
    do {                              \
        int _rc = (call);             \
        if (_rc != MT_OK) return _rc; \
    } while (0)

// ---------------------------------------------------------------------------
// Finalize kernels (one block per candidate, fixed summation order).
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool cand_valid(const double* x, int c, int full) {
    return full ? params_valid<true>(x + 9 * (size_t)c) : params_valid<false>(x + 6 * (size_t)c);
}

// Block sums of three values: an xor butterfly inside each wavefront, then
// the wavefront totals added in wavefront order (fixed, so deterministic).
__device__ __forceinline__ void block_sum3_waves(double* a, double (*sh)[256]) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int k = 0; k < 3; ++k) a[k] += __shfl_xor(a[k], o, 64);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 3; ++k) sh[k][w] = a[k];
    __syncthreads();
    for (int k = 0; k < 3; ++k) {
        double t = sh[k][0];
        for (int q = 1; q < nw; ++q) t += sh[k][q];
        a[k] = t;
    }
}

struct FinArgs {
    SetDev set;
    const double* partial;
    int nv;
    const double* eref; const double* wref;
    double Qe, Qv, Qf, we, wv, wf;
    const double* x;           // [P][6] (minimal) or [P][9] (Tersoff form)
    int full;                  // 1: x holds Tersoff-form parameter sets
    double* Z;                 // [P][4]
    double* coef;              // [P][S][8] or null (gradient coefficients)
    double* energy; double* virial; double* heat;
    int coop;                  // 1 if some structure has more than kCoopSlots slots
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

// Structures with more partial-sum slots than this (over 2,048 atoms: a
// structure over the batching limit has one slot per 256-atom block, a batched
// one at most 8) are summed by the whole block; smaller ones by one thread each.
constexpr int kCoopSlots = 8;

// Block-wide slot sums of structure s (all threads call; the result is valid
// in every thread).  The structure's [slots][nv] partial sums are read as one
// flat array, consecutive threads on consecutive values (coalesced: a strided
// read of whole slots per thread makes every load instruction touch 64 cache
// lines).  With nv (8 or 16) dividing the block, thread t only ever sees value
// t % nv; an xor butterfly over the lanes of equal value index and the
// wavefront totals in wavefront order finish the sums, so the order depends
// only on the sizes.
template <int NV>
__device__ void coop_sums_n(const FinArgs& F, int c, int s0, int s1, double* a, double (*sh)[256]) {
    const SetDev& d = F.set;
    const int nv = F.nv;                           // 8 or 16, a power of two
    const double* base = F.partial + ((size_t)c * d.nslots + s0) * nv;
    const int total = (s1 - s0) * nv;
    const int bd = blockDim.x;
    double acc = 0.0;
    // sixteen loads in flight per thread before their adds (the last batch
    // predicated: a serial tail would wait for each load in turn)
    for (int e = threadIdx.x; e < total; e += 16 * bd) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = e + u * bd < total ? base[e + u * bd] : 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u) acc += v[u];
    }
    for (int o = nv; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = bd >> 6;
    __syncthreads();                       // sh may still be read by an earlier call
    if (lane < nv && lane < 11) sh[lane][w] = acc;   // values 11.. of a slot are unused
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 11; ++k) {
        double t = 0.0;
        if (k < NV) {
            t = sh[k][0];
            for (int q = 1; q < nw; ++q) t += sh[k][q];
        }
        a[k] = t;
    }
    __syncthreads();
}

__device__ void coop_struct_sums(const FinArgs& F, int c, int s, double* e, double* w6, double* rf,
                                 double* j3, double (*sh)[256]) {
    double a[11];
    const SetDev& d = F.set;
    // a set of one structure owns every slot: no table lookup
    const int s0 = d.S == 1 ? 0 : d.st_slot[s], s1 = d.S == 1 ? d.nslots : d.st_slot[s + 1];
    if (F.nv >= 11) coop_sums_n<11>(F, c, s0, s1, a, sh);
    else coop_sums_n<8>(F, c, s0, s1, a, sh);
    *e = a[0];
    for (int k = 0; k < 6; ++k) w6[k] = a[1 + k];
    *rf = a[7];
    for (int k = 0; k < 3; ++k) j3[k] = a[8 + k];
}

__device__ __forceinline__ bool coop_struct(const SetDev& d, int s) {
    return d.st_slot[s + 1] - d.st_slot[s] > kCoopSlots;
}

__global__ __launch_bounds__(256) void k_finalize_fit(FinArgs F) {
    __shared__ double sh[11][256];
    const int c = blockIdx.x;
    const SetDev& d = F.set;
    double acc[3] = {0, 0, 0};
    for (int s = 0; F.coop && s < d.S; ++s) {
        if (!coop_struct(d, s)) continue;
        double e, w6[6], rf, j3[3];
        coop_struct_sums(F, c, s, &e, w6, &rf, j3, sh);
        if (threadIdx.x == 0) {
            const double n = (double)(d.st_off[s + 1] - d.st_off[s]);
            const double de = e / n - F.eref[s];
            acc[0] += de * de;
            for (int k = 0; k < 6; ++k) {
                const double dw = w6[k] / n - F.wref[6 * s + k];
                acc[1] += dw * dw;
            }
            acc[2] += rf;
        }
    }
    for (int s = threadIdx.x; s < d.S; s += blockDim.x) {
        if (F.coop && coop_struct(d, s)) continue;
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
    block_sum3_waves(acc, sh);
    if (threadIdx.x == 0) {
        const bool ok = cand_valid(F.x, c, F.full);
        const double Ze = sqrt(acc[0] / F.Qe), Zv = sqrt(acc[1] / F.Qv), Zf = sqrt(acc[2] / F.Qf);
        const double Z = F.we * Ze + F.wv * Zv + F.wf * Zf;
        const double nan = __longlong_as_double(0x7ff8000000000000ll);
        F.Z[4 * c + 0] = ok ? Z : nan;
        F.Z[4 * c + 1] = ok ? Ze : nan;
        F.Z[4 * c + 2] = ok ? Zv : nan;
        F.Z[4 * c + 3] = ok ? Zf : nan;
    }
}

// Z for sets of at most 64 structures without block-wide ones: one wavefront
// per candidate (four per block), lanes over structures, then a fixed xor
// butterfly, after which every lane holds the same sums.  OneSlot as for
// k_finalize_fit_block below.
template <bool OneSlot>
__global__ __launch_bounds__(256) void k_finalize_fit_wave(FinArgs F, int P) {
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= P) return;
    const SetDev& d = F.set;
    double acc[3] = {0, 0, 0};
    for (int s = lane; s < d.S; s += 64) {
        double e, w6[6], rf, j3[3];
        if constexpr (OneSlot) {
            const double* p = F.partial + ((size_t)c * d.nslots + s) * F.nv;
            e = p[0];
            for (int k = 0; k < 6; ++k) w6[k] = p[1 + k];
            rf = p[7];
        } else {
            struct_sums(F, c, s, &e, w6, &rf, j3);
        }
        const double n = (double)(d.st_off[s + 1] - d.st_off[s]);
        const double de = e / n - F.eref[s];
        acc[0] += de * de;
        for (int k = 0; k < 6; ++k) {
            const double dw = w6[k] / n - F.wref[6 * s + k];
            acc[1] += dw * dw;
        }
        acc[2] += rf;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[k] += __shfl_xor(acc[k], o, 64);
    if (lane == 0) {
        const bool ok = cand_valid(F.x, c, F.full);
        const double Ze = sqrt(acc[0] / F.Qe), Zv = sqrt(acc[1] / F.Qv), Zf = sqrt(acc[2] / F.Qf);
        const double Z = F.we * Ze + F.wv * Zv + F.wf * Zf;
        const double nan = __longlong_as_double(0x7ff8000000000000ll);
        F.Z[4 * c + 0] = ok ? Z : nan;
        F.Z[4 * c + 1] = ok ? Ze : nan;
        F.Z[4 * c + 2] = ok ? Zv : nan;
        F.Z[4 * c + 3] = ok ? Zf : nan;
    }
}

// Z for sets without block-wide structures when S is small: one block per
// candidate, one thread per structure (strided beyond the block), then a fixed
// LDS tree.  Every thread issues its structure's table and partial-sum loads
// at once, so a generation pays two memory round trips here instead of the
// four or five of a wavefront looping over the structures.  OneSlot: every
// structure has exactly one partial-sum slot (slot s), so the partial sums
// load without the slot table, in the same round trip as the rest.
template <bool OneSlot>
__global__ __launch_bounds__(256) void k_finalize_fit_block(FinArgs F) {
    __shared__ double sh[3][256];
    const int c = blockIdx.x;
    const SetDev& d = F.set;
    double acc[3] = {0, 0, 0};
    for (int s = threadIdx.x; s < d.S; s += blockDim.x) {
        double e, w6[6], rf, j3[3];
        if constexpr (OneSlot) {
            const double* p = F.partial + ((size_t)c * d.nslots + s) * F.nv;
            e = p[0];
            for (int k = 0; k < 6; ++k) w6[k] = p[1 + k];
            rf = p[7];
        } else {
            struct_sums(F, c, s, &e, w6, &rf, j3);
        }
        const double n = (double)(d.st_off[s + 1] - d.st_off[s]);
        const double de = e / n - F.eref[s];
        acc[0] += de * de;
        for (int k = 0; k < 6; ++k) {
            const double dw = w6[k] / n - F.wref[6 * s + k];
            acc[1] += dw * dw;
        }
        acc[2] += rf;
    }
    block_sum3_waves(acc, sh);
    if (threadIdx.x == 0) {
        const bool ok = cand_valid(F.x, c, F.full);
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

// dZ/dx [P][nx], nx = 6 (minimal) or 9 (Tersoff form).
__global__ __launch_bounds__(256) void k_finalize_grad(FinArgs F, double* dZdx) {
    __shared__ double sh[9][256];
    const int c = blockIdx.x;
    const SetDev& d = F.set;
    const int nx = F.full ? 9 : 6;
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int sl = threadIdx.x; sl < d.nslots; sl += blockDim.x) {
        const double* p = F.partial + ((size_t)c * d.nslots + sl) * F.nv;
        for (int k = 0; k < nx; ++k) acc[k] += p[k];
    }
    for (int k = 0; k < 9; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < 9; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const bool ok = cand_valid(F.x, c, F.full);
        const double nan = __longlong_as_double(0x7ff8000000000000ll);
        for (int k = 0; k < nx; ++k) dZdx[(size_t)nx * c + k] = ok ? sh[k][0] : nan;
    }
}

// Per-structure terms of the fitness partial sums: e_s = E_s / N_s,
// w_s = W_s / N_s and the squared force residual of the structure; NaN rows
// for candidates outside the potential's domain.
__global__ __launch_bounds__(256) void k_fitness_terms(FinArgs F, double* e_out, double* w_out,
                                                       double* rf_out) {
    const int c = blockIdx.x;
    const SetDev& d = F.set;
    const bool ok = cand_valid(F.x, c, F.full);
    const double nan = __longlong_as_double(0x7ff8000000000000ll);
    for (int s = threadIdx.x; s < d.S; s += blockDim.x) {
        double e, w6[6], rf, j3[3];
        struct_sums(F, c, s, &e, w6, &rf, j3);
        const double n = (double)(d.st_off[s + 1] - d.st_off[s]);
        const size_t o = (size_t)c * d.S + s;
        if (e_out) e_out[o] = ok ? e / n : nan;
        if (w_out)
            for (int k = 0; k < 6; ++k) w_out[6 * o + k] = ok ? w6[k] / n : nan;
        if (rf_out) rf_out[o] = ok ? rf : nan;
    }
}

__global__ __launch_bounds__(256) void k_finalize_eval(FinArgs F) {
    __shared__ double sh[11][256];
    const int c = blockIdx.x;
    const SetDev& d = F.set;
    const bool ok = cand_valid(F.x, c, F.full);
    const double nan = __longlong_as_double(0x7ff8000000000000ll);
    double jacc[3] = {0, 0, 0};
    if (d.S == 1) {
        // one structure (a large cell): the whole block sums its slots, no
        // slot-table reads and no block reduction of the heat current
        double e, w6[6], rf, j3[3];
        coop_struct_sums(F, c, 0, &e, w6, &rf, j3, sh);
        if (threadIdx.x == 0) {
            if (F.energy) F.energy[c] = ok ? e : nan;
            if (F.virial)
                for (int k = 0; k < 6; ++k) F.virial[(size_t)c * 6 + k] = ok ? w6[k] : nan;
            if (F.heat)
                for (int k = 0; k < 3; ++k) F.heat[3 * c + k] = ok ? j3[k] : nan;
        }
        return;
    }
    for (int s = 0; F.coop && s < d.S; ++s) {
        if (!coop_struct(d, s)) continue;
        double e, w6[6], rf, j3[3];
        coop_struct_sums(F, c, s, &e, w6, &rf, j3, sh);
        if (threadIdx.x == 0) {
            if (F.energy) F.energy[(size_t)c * d.S + s] = ok ? e : nan;
            if (F.virial)
                for (int k = 0; k < 6; ++k) F.virial[((size_t)c * d.S + s) * 6 + k] = ok ? w6[k] : nan;
            for (int k = 0; k < 3; ++k) jacc[k] += j3[k];
        }
    }
    for (int s = threadIdx.x; s < d.S; s += blockDim.x) {
        if (F.coop && coop_struct(d, s)) continue;
        double e, w6[6], rf, j3[3];
        struct_sums(F, c, s, &e, w6, &rf, j3);
        if (F.energy) F.energy[(size_t)c * d.S + s] = ok ? e : nan;
        if (F.virial)
            for (int k = 0; k < 6; ++k) F.virial[((size_t)c * d.S + s) * 6 + k] = ok ? w6[k] : nan;
        for (int k = 0; k < 3; ++k) jacc[k] += j3[k];
    }
    block_sum3_waves(jacc, sh);
    if (threadIdx.x == 0 && F.heat)
        for (int k = 0; k < 3; ++k) F.heat[3 * c + k] = ok ? jacc[k] : nan;
}


// ---------------------------------------------------------------------------
// Host side: work lists per coordination class, launches, finalize.
// ---------------------------------------------------------------------------
namespace {

int grid_of(long long n, int b) { return (int)((n + b - 1) / b); }

template <typename S>
BArgs<S> make_args(mt_set* set, double* partial, int nv) {
    BArgs<S> A{};
    A.set = set->dev();
    A.x = set->cur_x;
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
    F.x = set->cur_x;
    F.full = set->cur_form;
    F.coop = 0;
    for (int s = 0; s < set->S; ++s)
        if (set->h_slot[s + 1] - set->h_slot[s] > kCoopSlots) F.coop = 1;
    return F;
}

bool family_f64(int fam) {
    return fam == FAM_FIT64 || fam == FAM_EVAL64 || fam == FAM_ADJ64 || fam == FAM_FIT64F ||
           fam == FAM_EVAL64F || fam == FAM_ADJ64F;
}
bool family_fit(int fam) {
    return fam == FAM_FIT32 || fam == FAM_FIT64 || fam == FAM_FIT32F || fam == FAM_FIT64F;
}
bool family_full(int fam) {
    return fam == FAM_FIT32F || fam == FAM_EVAL32F || fam == FAM_FIT64F || fam == FAM_EVAL64F ||
           fam == FAM_ADJ32F || fam == FAM_ADJ64F;
}
int family_elem(int fam) { return family_f64(fam) ? 8 : 4; }
bool family_adjoint(int fam) {
    return fam == FAM_ADJ32 || fam == FAM_ADJ64 || fam == FAM_ADJ32F || fam == FAM_ADJ64F;
}

// LDS of one item of nc candidates: parameter records, bond-gradient exchange
// slots (4 values each) and, for the adjoint, the force-residual exchange.
size_t item_lds(const mt_set* set, int s, int block, int fam, int nc) {
    const int npad = set->h_npad[s];
    const int R = block / npad;
    const size_t e = (size_t)family_elem(fam);
    const size_t par = ((size_t)nc * kNParam * e + 31) & ~(size_t)31;
    const size_t xs = (size_t)R * set->h_xsize[s] * 4 * e;
    const size_t ad = family_adjoint(fam) ? (size_t)R * npad * 4 * e : 0;
    return par + xs + ad;
}

hipError_t launch_family(int fam, int mc, dim3 g, dim3 b, size_t lds, hipStream_t st,
                         const BArgs<float>& Af, const BArgs<double>& Ad,
                         hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
    switch (fam) {
        case FAM_FIT32: return launch_fit32(mc, g, b, lds, st, Af, e0, e1);
        case FAM_EVAL32: return launch_eval32(mc, g, b, lds, st, Af, e0, e1);
        case FAM_FIT64: return launch_fit64(mc, g, b, lds, st, Ad, e0, e1);
        case FAM_EVAL64: return launch_eval64(mc, g, b, lds, st, Ad, e0, e1);
        case FAM_ADJ32: return launch_adj32(mc, g, b, lds, st, Af, e0, e1);
        case FAM_ADJ64: return launch_adj64(mc, g, b, lds, st, Ad, e0, e1);
        case FAM_FIT32F: return launch_fit32f(mc, g, b, lds, st, Af, e0, e1);
        case FAM_EVAL32F: return launch_eval32f(mc, g, b, lds, st, Af, e0, e1);
        case FAM_FIT64F: return launch_fit64f(mc, g, b, lds, st, Ad, e0, e1);
        case FAM_EVAL64F: return launch_eval64f(mc, g, b, lds, st, Ad, e0, e1);
        case FAM_ADJ32F: return launch_adj32f(mc, g, b, lds, st, Af, e0, e1);
        case FAM_ADJ64F: return launch_adj64f(mc, g, b, lds, st, Ad, e0, e1);
    }
    return hipErrorInvalidValue;
}

}  // namespace

int family_for(int precision, int mode, int form) {
    const bool f64 = precision == MT_FP64;
    if (form) {
        if (mode == MODE_FIT) return f64 ? FAM_FIT64F : FAM_FIT32F;
        return f64 ? FAM_EVAL64F : FAM_EVAL32F;
    }
    if (mode == MODE_FIT) return f64 ? FAM_FIT64 : FAM_FIT32;
    return f64 ? FAM_EVAL64 : FAM_EVAL32;
}

const std::vector<int>& family_classes(int fam) {
    static const std::vector<int> k[NFAM] = {
        {4, 6, 8, 12, 16},   // FIT32
        {4, 8, 16},          // EVAL32
        {4, 16},             // FIT64
        {4, 16},             // EVAL64
        {4, 8, 12},          // ADJ32
        {4, 12},             // ADJ64
        {4, 16},             // FIT32F
        {4, 16},             // EVAL32F
        {4, 16},             // FIT64F
        {4, 16},             // EVAL64F
        {4, 12},             // ADJ32F
        {4, 12},             // ADJ64F
    };
    return k[fam];
}

int class_of(int fam, int kmax) {
    for (int mc : family_classes(fam))
        if (kmax <= mc) return mc;
    return family_classes(fam).back();
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

static bool upload_class(ClassPlan& cp, const std::vector<Item>& ordered, const std::vector<int>& bin_off) {
    cp.h_items = ordered;
    cp.n_items = (int)ordered.size();
    cp.n_bins = (int)bin_off.size() - 1;
    if (cp.n_items > 0) {
        if (cp.items.reserve(sizeof(Item) * ordered.size()) != hipSuccess) return false;
        if (hipMemcpy(cp.items.p, ordered.data(), sizeof(Item) * ordered.size(), hipMemcpyHostToDevice) != hipSuccess)
            return false;
    }
    if (cp.bin_off.reserve(sizeof(int) * bin_off.size()) != hipSuccess) return false;
    return hipMemcpy(cp.bin_off.p, bin_off.data(), sizeof(int) * bin_off.size(), hipMemcpyHostToDevice) == hipSuccess;
}

// Candidate tile of structure s at R replicas per block (whole steps of the replicas).
static int tile_for(const LaunchCfg& cfg, int P, int R, bool plain) {
    int tile = plain ? 1 : std::max(cfg.tile, 1);
    if (!plain) tile = ((tile + R - 1) / R) * R;
    return std::min(tile, ((P + R - 1) / R) * R);
}

// Block size for structure s: the requested one when its LDS fits the device
// (replicas that do not fill the block leave whole wavefronts idle), else the
// largest smaller multiple of 64 threads, at least the padded size, that fits;
// 0 when a single replica does not fit.  Keeping the requested size keeps
// every structure of a class in one launch.
static int block_for(const mt_set* set, int s, const LaunchCfg& cfg, int P, int fam, bool plain) {
    const int npad = set->h_npad[s];
    const int least = std::max(64, npad);
    for (int block = plain ? least : cfg.block; block >= least; block -= 64) {
        const int R = block / npad;
        if (item_lds(set, s, block, fam, std::min(tile_for(cfg, P, R, plain), P)) <= set->lds_max)
            return block;
    }
    return 0;
}

// The blocks of a launch go to the XCDs round robin (block b to XCD b mod 8),
// and each XCD has its own L2.  Within every run of equal-cost items (the
// order across runs is kept), order the items structure by structure and deal
// each XCD a contiguous share of the run: the candidate tiles of a structure
// then run on one XCD, and its bond geometry comes from HBM about once instead
// of once per XCD it lands on.  Only the placement changes, not any result.
static std::vector<Item> xcd_grouped(const std::vector<Item>& items) {
    constexpr size_t kXcd = 8;
    std::vector<Item> out(items.size());
    size_t a = 0;
    while (a < items.size()) {
        size_t e = a;
        while (e < items.size() && items[e].cost == items[a].cost) ++e;
        std::vector<Item> run(items.begin() + a, items.begin() + e);
        std::stable_sort(run.begin(), run.end(), [](const Item& x, const Item& y) {
            return x.s != y.s ? x.s < y.s : x.c0 < y.c0;
        });
        size_t next = 0;
        for (size_t k = 0; k < kXcd; ++k)
            for (size_t b = a; b < e; ++b)
                if (b % kXcd == k) out[b] = run[next++];
        a = e;
    }
    return out;
}

ItemPlan* find_plan(mt_set* set, int P, const LaunchCfg& cfg, int fam) {
    auto itp = set->plans.find(std::make_tuple(P, cfg.block, cfg.tile, cfg.persistent, fam));
    return itp != set->plans.end() ? itp->second.get() : nullptr;
}

// cfg.block == 0 requests the plain plan: one item per (structure, candidate).
ItemPlan* get_plan(mt_set* set, int P, const LaunchCfg& cfg, int fam) {
    auto key = std::make_tuple(P, cfg.block, cfg.tile, cfg.persistent, fam);
    auto itp = set->plans.find(key);
    if (itp != set->plans.end()) return itp->second.get();
    auto plan = std::make_unique<ItemPlan>();
    const bool plain = cfg.block == 0;
    int ncu = 256;
    if (!plain) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
            ncu = prop.multiProcessorCount;
    }
    struct Group {
        std::vector<Item> items;
        size_t lds = 16;
    };
    // Launch class of each structure.  A class above 4 whose work items would
    // fill fewer blocks than the device has compute units joins the next
    // larger class that has work: on its own its launch leaves most of the
    // device idle, and the larger class's kernel runs the same compiled
    // variants (chosen per wavefront by the largest coordination, never
    // below 3) on the same exchange-slot layout, so results are unchanged.
    const std::vector<int>& classes = family_classes(fam);
    std::vector<int> cls(set->S, 0);
    std::map<int, long long> nitems;
    for (int s = 0; s < set->S; ++s) {
        if (set->h_large[s]) continue;
        if (set->h_kmax[s] > classes.back()) {
            // above the family's widest class (the adjoint's 12): two-pass
            plan->twopass.push_back(s);
            continue;
        }
        cls[s] = class_of(fam, set->h_kmax[s]);
        if (!plain) {
            const int tile = tile_for(cfg, P, std::max(1, cfg.block / set->h_npad[s]), plain);
            nitems[cls[s]] += (P + tile - 1) / tile;
        }
    }
    for (size_t i = 0; !plain && i < classes.size(); ++i) {
        const int mc = classes[i];
        if (mc <= 4 || nitems[mc] == 0 || nitems[mc] >= ncu) continue;
        for (size_t j = i + 1; j < classes.size(); ++j) {
            const int to = classes[j];
            if (nitems[to] == 0) continue;
            for (int s = 0; s < set->S; ++s)
                if (!set->h_large[s] && cls[s] == mc) cls[s] = to;
            nitems[to] += nitems[mc];
            nitems[mc] = 0;
            break;
        }
    }
    for (int mc : classes) {
        std::map<int, Group> groups;          // launch block size -> work items
        for (int s = 0; s < set->S; ++s) {
            if (set->h_large[s] || cls[s] != mc) continue;
            const int npad = set->h_npad[s];
            if (!plain && cfg.block < npad) return nullptr;
            const int block = block_for(set, s, cfg, P, fam, plain);
            if (block == 0) {
                plan->twopass.push_back(s);
                continue;
            }
            const int R = block / npad;
            const int tile = tile_for(cfg, P, R, plain);
            Group& g = groups[block];
            g.lds = std::max(g.lds, item_lds(set, s, block, fam, std::min(tile, P)));
            const int ns = set->h_off[s + 1] - set->h_off[s];
            for (int c0 = 0; c0 < P; c0 += tile) {
                Item it;
                it.s = s;
                it.c0 = c0;
                it.nc = std::min(tile, P - c0);
                const long long steps = (it.nc + R - 1) / R;
                const long long per = set->h_trip[s] + 8ll * ns + 64;
                it.cost = (int)std::min<long long>(steps * per / std::max(1, R) + 1, 1ll << 30);
                g.items.push_back(it);
            }
        }
        for (auto it = groups.rbegin(); it != groups.rend(); ++it) {
            std::vector<Item>& items = it->second.items;
            auto cp = std::make_unique<ClassPlan>();
            cp->mc = mc;
            cp->block = it->first;
            cp->lds = it->second.lds;
            std::vector<int> bin_off;
            std::vector<Item> ordered;
            if (plain) {
                ordered = items;
                bin_off = {0, 1};
            } else {
                // longest first; equal costs grouped by XCD (bins, one per block,
                // take the items in this order)
                std::stable_sort(items.begin(), items.end(),
                                 [](const Item& a, const Item& b) { return a.cost > b.cost; });
                items = xcd_grouped(items);
                if (!cfg.persistent) {
                    ordered = items;
                    bin_off.resize(items.size() + 1);
                    std::iota(bin_off.begin(), bin_off.end(), 0);
                } else {
                    const int per_cu = std::max(1, 1024 / cp->block);
                    const int nbins = (int)std::min<size_t>(items.size(), (size_t)ncu * per_cu);
                    std::vector<std::vector<Item>> bins(std::max(nbins, 1));
                    using E = std::pair<long long, int>;
                    std::priority_queue<E, std::vector<E>, std::greater<E>> heap;
                    for (int b = 0; b < (int)bins.size(); ++b) heap.push({0, b});
                    for (const Item& w : items) {       // longest first onto the least-loaded bin
                        E e = heap.top();
                        heap.pop();
                        bins[e.second].push_back(w);
                        heap.push({e.first + w.cost, e.second});
                    }
                    bin_off.push_back(0);
                    for (auto& b : bins) {
                        for (auto& w : b) ordered.push_back(w);
                        bin_off.push_back((int)ordered.size());
                    }
                }
            }
            if (!upload_class(*cp, ordered, bin_off)) return nullptr;
            if (plain) cp->n_bins = 1;
            plan->cls.push_back(std::move(cp));
        }
    }
    ItemPlan* raw = plan.get();
    set->plans[key] = std::move(plan);
    return raw;
}


// Launch every class of a plan (batched: one launch per class; plain: one per item).
static int run_plan(mt_set* set, ItemPlan* plan, const LaunchCfg& cfg, int fam, BArgs<float> Af,
                    BArgs<double> Ad, int prof_kind, hipStream_t st) {
    const bool plain = cfg.block == 0;
    for (auto& cpp : plan->cls) {
        ClassPlan& cp = *cpp;
        if (!plain) {
            Af.items = Ad.items = cp.items.as<Item>();
            Af.bin_off = Ad.bin_off = cp.bin_off.as<int>();
            ProfScope prof(set, prof_kind < 0 ? -1 : prof_kind);
            HIPCHECK(launch_family(fam, cp.mc, dim3(cp.n_bins), dim3(cp.block), cp.lds, st, Af, Ad,
                                   prof.e0, prof.e1));
        } else {
            const bool f64 = family_f64(fam);
            const bool full = family_full(fam);
            const int mode = family_fit(fam) ? MODE_FIT : MODE_EVAL;
            for (int k = 0; k < cp.n_items; ++k) {
                const int s = cp.h_items[k].s;
                const dim3 block(cp.block);
                const size_t lds = item_lds(set, s, block.x, fam, 1);
                Af.items = Ad.items = cp.items.as<Item>() + k;
                HIPCHECK(f64 ? launch_plain64(mode, full, cp.mc, block, lds, st, Ad)
                             : launch_plain32(mode, full, cp.mc, block, lds, st, Af));
            }
        }
    }
    return MT_OK;
}

static int launch_twopass(mt_set* set, const std::vector<int>& structs, int P, int precision,
                          int mode, const double* vel, double* force, double* atom_virial,
                          hipStream_t st);

int launch_batched(mt_set* set, const LaunchCfg& cfg, int P, int precision, int mode,
                   const double* vel, double* force, double* atom_virial, hipStream_t st) {
    const int fam = family_for(precision, mode, set->cur_form);
    ItemPlan* plan = get_plan(set, P, cfg, fam);
    if (!plan) {
        set_error("could not build the work list (block smaller than a structure?)");
        return MT_EINVAL;
    }
    const int nv = mode == MODE_FIT ? kNVFit : kNVEval;
    BArgs<float> Af = make_args<float>(set, set->partial.as<double>(), nv);
    BArgs<double> Ad = make_args<double>(set, set->partial.as<double>(), nv);
    Af.vel = Ad.vel = vel;
    Af.force = Ad.force = force;
    Af.atom_virial = Ad.atom_virial = atom_virial;
    if (mode == MODE_FIT && set->grad_resid) {
        Af.resid = static_cast<float*>(set->grad_resid);
        Ad.resid = static_cast<double*>(set->grad_resid);
    }
    TRY_RC(run_plan(set, plan, cfg, fam, Af, Ad, 0, st));
    if (plan->twopass.empty()) return MT_OK;
    TRY_RC(reserve_twopass(set, plan, P, precision));     // no-op once reserved
    return launch_twopass(set, plan->twopass, P, precision, mode, vel, force, atom_virial, st);
}

int launch_plan_fit(mt_set* set, ItemPlan* plan, const LaunchCfg& cfg, int precision, double* partial,
                    hipStream_t st) {
    const int fam = family_for(precision, MODE_FIT, set->cur_form);
    BArgs<float> Af = make_args<float>(set, partial, kNVFit);
    BArgs<double> Ad = make_args<double>(set, partial, kNVFit);
    return run_plan(set, plan, cfg, fam, Af, Ad, -1, st);
}

int launch_plain(mt_set* set, int P, int precision, int mode, const double* vel, double* force,
                 double* atom_virial, hipStream_t st) {
    LaunchCfg plain;      // block = 0
    return launch_batched(set, plain, P, precision, mode, vel, force, atom_virial, st);
}

// reps back-to-back passes of the batched fitness kernels (the launches of
// run_plan only: no two-pass structures, no finalize) between one event pair;
// the per-pass average in ms and the launches per pass.  Synchronises st.
int time_batched_kernels(mt_set* set, const LaunchCfg& cfg, int P, int precision, int reps,
                         hipStream_t st, double* ms, int64_t* launches) {
    const int fam = family_for(precision, MODE_FIT, set->cur_form);
    ItemPlan* plan = get_plan(set, P, cfg, fam);
    if (!plan) {
        set_error("could not build the work list (block smaller than a structure?)");
        return MT_EINVAL;
    }
    BArgs<float> Af = make_args<float>(set, set->partial.as<double>(), kNVFit);
    BArgs<double> Ad = make_args<double>(set, set->partial.as<double>(), kNVFit);
    hipEvent_t e[2] = {nullptr, nullptr};
    int rc = MT_OK;
    hipError_t he = hipSuccess;
    for (auto& ev : e)
        if (rc == MT_OK && (he = hipEventCreate(&ev)) != hipSuccess) rc = hip_fail(he, "hipEventCreate");
    if (rc == MT_OK && (he = hipEventRecord(e[0], st)) != hipSuccess) rc = hip_fail(he, "hipEventRecord");
    for (int r = 0; r < reps && rc == MT_OK; ++r) rc = run_plan(set, plan, cfg, fam, Af, Ad, 0, st);
    if (rc == MT_OK && (he = hipEventRecord(e[1], st)) != hipSuccess) rc = hip_fail(he, "hipEventRecord");
    if (rc == MT_OK && (he = hipEventSynchronize(e[1])) != hipSuccess) rc = hip_fail(he, "hipEventSynchronize");
    float t = 0.f;
    if (rc == MT_OK && (he = hipEventElapsedTime(&t, e[0], e[1])) != hipSuccess)
        rc = hip_fail(he, "hipEventElapsedTime");
    for (auto& ev : e)
        if (ev) (void)hipEventDestroy(ev);
    if (rc != MT_OK) return rc;
    *ms = (double)t / reps;
    *launches = 0;
    for (auto& cp : plan->cls) *launches += cfg.block == 0 ? cp->n_items : 1;
    return MT_OK;
}

// Each launch of the batched fitness plan timed on its own: reps back-to-back
// launches of it between one event pair; per launch the average ms, its
// coordination class, and for every structure the launch that evaluates it
// (-1: two-pass path).  Synchronises st.
int time_class_launches(mt_set* set, const LaunchCfg& cfg, int P, int precision, int reps,
                        hipStream_t st, int max_launches, double* ms, int* mc, int* struct_launch,
                        int* n_launches) {
    const int fam = family_for(precision, MODE_FIT, set->cur_form);
    ItemPlan* plan = get_plan(set, P, cfg, fam);
    if (!plan) {
        set_error("could not build the work list (block smaller than a structure?)");
        return MT_EINVAL;
    }
    if (cfg.block == 0) {
        set_error("per-launch timing covers the batched schedule only");
        return MT_EINVAL;
    }
    const int n = (int)plan->cls.size();
    *n_launches = n;
    if (n > max_launches) {
        set_error("more launches than max_launches");
        return MT_EINVAL;
    }
    if (struct_launch) {
        for (int s = 0; s < set->S; ++s) struct_launch[s] = -1;
        for (int k = 0; k < n; ++k)
            for (const Item& it : plan->cls[k]->h_items) struct_launch[it.s] = k;
    }
    BArgs<float> Af = make_args<float>(set, set->partial.as<double>(), kNVFit);
    BArgs<double> Ad = make_args<double>(set, set->partial.as<double>(), kNVFit);
    hipEvent_t e[2] = {nullptr, nullptr};
    int rc = MT_OK;
    hipError_t he = hipSuccess;
    for (auto& ev : e)
        if (rc == MT_OK && (he = hipEventCreate(&ev)) != hipSuccess) rc = hip_fail(he, "hipEventCreate");
    for (int k = 0; k < n && rc == MT_OK; ++k) {
        ClassPlan& cp = *plan->cls[k];
        Af.items = Ad.items = cp.items.as<Item>();
        Af.bin_off = Ad.bin_off = cp.bin_off.as<int>();
        if ((he = hipEventRecord(e[0], st)) != hipSuccess) { rc = hip_fail(he, "hipEventRecord"); break; }
        for (int r = 0; r < reps && rc == MT_OK; ++r)
            if ((he = launch_family(fam, cp.mc, dim3(cp.n_bins), dim3(cp.block), cp.lds, st, Af, Ad)) !=
                hipSuccess)
                rc = hip_fail(he, "kernel launch");
        if (rc != MT_OK) break;
        if ((he = hipEventRecord(e[1], st)) != hipSuccess) { rc = hip_fail(he, "hipEventRecord"); break; }
        if ((he = hipEventSynchronize(e[1])) != hipSuccess) { rc = hip_fail(he, "hipEventSynchronize"); break; }
        float t = 0.f;
        if ((he = hipEventElapsedTime(&t, e[0], e[1])) != hipSuccess) { rc = hip_fail(he, "hipEventElapsedTime"); break; }
        ms[k] = (double)t / reps;
        mc[k] = cp.mc;
    }
    for (auto& ev : e)
        if (ev) (void)hipEventDestroy(ev);
    return rc;
}

// Candidates per launch of the two-pass path for structure s: bounded so that
// the bond-gradient staging buffer stays within 256 MB.
static int twopass_chunk(const mt_set* set, int s, int P, size_t elem) {
    const size_t per = 4 * (size_t)(set->h_boff[s + 1] - set->h_boff[s]) * elem;
    const size_t chunk = std::min<size_t>((size_t)P, (256ull << 20) / std::max<size_t>(per, 1));
    return (int)std::min<size_t>(std::max<size_t>(chunk, 1), 65535);
}

int reserve_twopass(mt_set* set, const ItemPlan* plan, int P, int precision) {
    const size_t elem = precision == MT_FP64 ? sizeof(double) : sizeof(float);
    size_t need = 0;
    auto add = [&](int s) {
        const size_t per = 4 * (size_t)(set->h_boff[s + 1] - set->h_boff[s]) * elem;
        need = std::max(need, per * twopass_chunk(set, s, P, elem));
    };
    for (int s = 0; s < set->S; ++s)
        if (set->h_large[s]) add(s);
    if (plan)
        for (int s : plan->twopass) add(s);
    // a captured fitness graph holds the buffer's address in its two-pass
    // launches: growing the buffer frees that memory, so those graphs go too
    const void* before = set->gbuf.p;
    if (need) HIPCHECK(set->gbuf.reserve(need));
    if (set->gbuf.p != before) clear_graphs(set);
    return MT_OK;
}

// Two-pass evaluation (bond gradients staged in global memory, then gathered)
// of the listed structures, for structures too large for one block's LDS.
template <typename S>
static int launch_twopass_t(mt_set* set, const std::vector<int>& structs, int P, int mode, int nv,
                            const double* vel, double* force, double* atom_virial, hipStream_t st) {
    BArgs<S> A = make_args<S>(set, set->partial.as<double>(), nv);
    A.vel = vel;
    A.force = force;
    A.atom_virial = atom_virial;
    for (int s : structs) {
        const int mc = set->h_kmax[s] <= 4 ? 4 : 16;
        const int ns = set->h_off[s + 1] - set->h_off[s];
        const size_t per = 4 * (size_t)(set->h_boff[s + 1] - set->h_boff[s]) * sizeof(S);
        const int chunk = twopass_chunk(set, s, P, sizeof(S));
        if (set->gbuf.bytes < per * chunk) {
            set_error("two-pass staging buffer not reserved");
            return MT_ESTATE;
        }
        for (int c0 = 0; c0 < P; c0 += chunk) {
            const int nc = std::min(chunk, P - c0);
            LArgs L{s, c0, set->gbuf.p, set->h_large[s] ? 1 : 0, set->h_off[s], set->h_off[s + 1] - set->h_off[s],
                    set->h_boff[s + 1] - set->h_boff[s], set->h_slot[s], set->h_kmax[s]};
            dim3 grid(grid_of(ns, kLargeBlock), nc);
            hipError_t e;
            if constexpr (std::is_same<S, double>::value)
                e = launch_large64(mc, mode, set->cur_form, grid, dim3(kLargeBlock), st, A, L);
            else
                e = launch_large32(mc, mode, set->cur_form, grid, dim3(kLargeBlock), st, A, L);
            HIPCHECK(e);
        }
    }
    return MT_OK;
}

static int launch_twopass(mt_set* set, const std::vector<int>& structs, int P, int precision,
                          int mode, const double* vel, double* force, double* atom_virial,
                          hipStream_t st) {
    if (structs.empty()) return MT_OK;
    const int nv = mode == MODE_FIT ? kNVFit : kNVEval;
    return precision == MT_FP64
               ? launch_twopass_t<double>(set, structs, P, mode, nv, vel, force, atom_virial, st)
               : launch_twopass_t<float>(set, structs, P, mode, nv, vel, force, atom_virial, st);
}

int launch_large(mt_set* set, int P, int precision, int mode, const double* vel, double* force,
                 double* atom_virial, hipStream_t st) {
    if (set->n_large == 0) return MT_OK;
    std::vector<int> structs;
    for (int s = 0; s < set->S; ++s)
        if (set->h_large[s]) structs.push_back(s);
    TRY_RC(reserve_twopass(set, nullptr, P, precision));
    return launch_twopass(set, structs, P, precision, mode, vel, force, atom_virial, st);
}

int launch_finalize_fit(mt_set* set, int P, const double* w, double* Z, hipStream_t st,
                        const double* partial) {
    FinArgs F = make_fin(set, kNVFit, partial ? partial : set->partial.as<double>());
    F.we = w[0]; F.wv = w[1]; F.wf = w[2];
    F.Z = Z;
    if (F.coop) {
        hipLaunchKernelGGL(k_finalize_fit, dim3(P), dim3(256), 0, st, F);
    } else if (set->S > 64) {
        // power-of-two block (the LDS tree halves it), at least one thread per
        // structure up to 256
        int block = 128;
        while (block < set->S && block < 256) block *= 2;
        if (set->nslots == set->S)
            hipLaunchKernelGGL(k_finalize_fit_block<true>, dim3(P), dim3(block), 0, st, F);
        else
            hipLaunchKernelGGL(k_finalize_fit_block<false>, dim3(P), dim3(block), 0, st, F);
    } else {
        if (set->nslots == set->S)
            hipLaunchKernelGGL(k_finalize_fit_wave<true>, dim3((P + 3) / 4), dim3(256), 0, st, F, P);
        else
            hipLaunchKernelGGL(k_finalize_fit_wave<false>, dim3((P + 3) / 4), dim3(256), 0, st, F, P);
    }
    HIPCHECK(hipGetLastError());
    return MT_OK;
}

int launch_finalize_eval(mt_set* set, int P, double* energy, double* virial, double* heat,
                         hipStream_t st) {
    FinArgs F = make_fin(set, kNVEval, set->partial.as<double>());
    F.energy = energy;
    F.virial = virial;
    F.heat = heat;
    hipLaunchKernelGGL(k_finalize_eval, dim3(P), dim3(256), 0, st, F);
    HIPCHECK(hipGetLastError());
    return MT_OK;
}

int launch_fitness_terms(mt_set* set, int P, double* e, double* w, double* rf, hipStream_t st) {
    FinArgs F = make_fin(set, kNVFit, set->partial.as<double>());
    hipLaunchKernelGGL(k_fitness_terms, dim3(P), dim3(256), 0, st, F, e, w, rf);
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

// Two-pass fitness gradient of the listed structures, one candidate chunk at a
// time: bond gradients staged as for the two-pass fitness (no partial sums),
// force residuals staged [chunk][3][Ns] in abuf, then the dual passes.
template <typename S>
static int launch_twopass_adjoint(mt_set* set, const std::vector<int>& structs, int P, int nv,
                                  hipStream_t st) {
    size_t abytes = 0;
    for (int s : structs) {
        const int ns = set->h_off[s + 1] - set->h_off[s];
        abytes = std::max(abytes, 3 * (size_t)ns * sizeof(S) * twopass_chunk(set, s, P, sizeof(S)));
    }
    HIPCHECK(set->abuf.reserve(abytes));
    BArgs<S> Afit = make_args<S>(set, nullptr, kNVFit);
    BArgs<S> Aadj = make_args<S>(set, set->partial2.as<double>(), nv);
    Aadj.coef = set->zwork.as<double>();
    for (int s : structs) {
        const int mc = set->h_kmax[s] <= 4 ? 4 : 16;
        const int ns = set->h_off[s + 1] - set->h_off[s];
        const size_t per = 4 * (size_t)(set->h_boff[s + 1] - set->h_boff[s]) * sizeof(S);
        const int chunk = twopass_chunk(set, s, P, sizeof(S));
        if (set->gbuf.bytes < per * chunk || set->abuf.bytes < 3 * (size_t)ns * sizeof(S) * chunk) {
            set_error("two-pass staging buffers not reserved");
            return MT_ESTATE;
        }
        for (int c0 = 0; c0 < P; c0 += chunk) {
            const int nc = std::min(chunk, P - c0);
            LArgs L{s, c0, set->gbuf.p, set->h_large[s] ? 1 : 0, set->h_off[s], set->h_off[s + 1] - set->h_off[s],
                    set->h_boff[s + 1] - set->h_boff[s], set->h_slot[s], set->h_kmax[s]};
            dim3 grid(grid_of(ns, kLargeBlock), nc);
            hipError_t e;
            if constexpr (std::is_same<S, double>::value)
                e = launch_large_adj64(mc, set->cur_form, grid, dim3(kLargeBlock), st, Afit, Aadj, L,
                                       set->abuf.as<double>());
            else
                e = launch_large_adj32(mc, set->cur_form, grid, dim3(kLargeBlock), st, Afit, Aadj, L,
                                       set->abuf.as<float>());
            HIPCHECK(e);
        }
    }
    return MT_OK;
}

static int adjoint_common(mt_set* set, const LaunchCfg& cfg, int P, int precision, const double* w,
                          const double* Z, hipStream_t st) {
    TRY_RC(launch_grad_coef(set, P, w, Z, st));
    const int nv = set->cur_form ? kNVGradTF : kNVGrad;
    HIPCHECK(set->partial2.reserve(sizeof(double) * nv * (size_t)P * set->nslots));
    const bool f64 = precision == MT_FP64;
    const int fam = set->cur_form ? (f64 ? FAM_ADJ64F : FAM_ADJ32F) : (f64 ? FAM_ADJ64 : FAM_ADJ32);
    ItemPlan* plan = get_plan(set, P, cfg, fam);
    if (!plan) {
        set_error("could not build the adjoint work list");
        return MT_EINVAL;
    }
    BArgs<float> Af = make_args<float>(set, set->partial2.as<double>(), nv);
    BArgs<double> Ad = make_args<double>(set, set->partial2.as<double>(), nv);
    Af.coef = Ad.coef = set->zwork.as<double>();
    // the fitness call before this one wrote the batched atoms' residuals (a
    // structure the adjoint batches needs no more LDS in the fitness, so the
    // fitness batched it too)
    Af.resid = set->resid.as<float>();
    Ad.resid = set->resid.as<double>();
    TRY_RC(run_plan(set, plan, cfg, fam, Af, Ad, 1, st));
    // structures over the batched limit, and those whose adjoint does not fit
    // one block's LDS, take the two-pass adjoint
    std::vector<int> structs;
    for (int s = 0; s < set->S; ++s)
        if (set->h_large[s]) structs.push_back(s);
    structs.insert(structs.end(), plan->twopass.begin(), plan->twopass.end());
    if (structs.empty()) return MT_OK;
    TRY_RC(reserve_twopass(set, plan, P, precision));
    return f64 ? launch_twopass_adjoint<double>(set, structs, P, nv, st)
               : launch_twopass_adjoint<float>(set, structs, P, nv, st);
}

int launch_adjoint(mt_set* set, const LaunchCfg& cfg, int P, int precision, const double* w,
                   const double* Z, hipStream_t st) {
    return adjoint_common(set, cfg, P, precision, w, Z, st);
}

int launch_finalize_grad(mt_set* set, int P, const double* Z, double* dZdx, hipStream_t st) {
    (void)Z;
    FinArgs F = make_fin(set, set->cur_form ? kNVGradTF : kNVGrad, set->partial2.as<double>());
    hipLaunchKernelGGL(k_finalize_grad, dim3(P), dim3(256), 0, st, F, dZdx);
    HIPCHECK(hipGetLastError());
    return MT_OK;
}

}  // namespace mt
