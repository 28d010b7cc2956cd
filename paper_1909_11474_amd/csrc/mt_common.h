// Internal declarations shared by the HIP translation units of the library.
//
// Data layout in HBM (all "sorted" atom indices: inside each structure the atoms
// are reordered by descending coordination number, so that the atoms of one
// wavefront have nearly the same number of neighbours; `perm` maps back to the
// caller's numbering):
//
//   per structure s : st_off[s]     first sorted atom, st_off[S] = N
//                     st_boff[s]    first bond (CSR over sorted atoms)
//                     st_npad[s]    atoms rounded up to 8/16/32/64 or a multiple of 64
//                     st_kmax[s]    largest coordination in s
//                     st_slot[s]    first partial-sum slot of s
//   per atom a      : perm[a], nnb[a] (coordination), lbo[a] (first bond of a,
//                     relative to st_boff[s]), xbase[a] (exchange slot, below)
//   per bond slot   : slot-major arrays [m][N] (m < kcap) of float and double
//                     geometry: unit vector, length (float: hi+lo split), 1/r,
//                     f_C(r), f_C'(r)/2; int: exchange slot and CSR index of the
//                     reverse bond, neighbour atom (structure-local sorted index).
//
// Exchange slots (LDS of the batched kernels).  A replica of structure s is cut
// into chunks of G = min(npad, 64) lanes; chunk c reserves K_c * G slots, K_c
// being the largest coordination in the chunk (at least the lowest variant of
// the structure's class), and bond m of the atom in lane l of the chunk uses
// slot off_c + m * G + l.  Padded bonds (m >= coordination) own a slot too and
// their reverse index is that slot, so the exchange needs no predicates.
//
// Geometry is candidate independent (R1, R2 are fixed, not fitted), so it is
// built once per structure set and reused by every candidate.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace mt {

constexpr int kMaxNbr = 16;        // template limit on coordination
constexpr int kMaxBatched = 512;   // largest structure of the batched kernel
// Threads per block of the two-pass kernels; a structure over the batching
// limit has one partial-sum slot per such block.
constexpr int kLargeBlock = 256;
constexpr int kNVFit = 8;          // partial sums per slot: E, W6, |F - F*|^2
constexpr int kNVEval = 16;        // E, W6, |F-F*|^2, J3, unused
constexpr int kNVGrad = 8;         // dZ/dx (6), unused (2)
constexpr int kNVGradTF = 16;      // Tersoff form: dZ/dx (9), unused (7)
constexpr int kNParam = 26;        // per-candidate decoded parameter record (25 used)

// Decoded parameter record (float or double), filled per work item in LDS.
// Both potential forms share it: f_R = DR e^{-lambda (r - r0)},
// f_A = DA e^{-mu (r - r0)} with lambda = alpha sqrt(2S), mu = alpha sqrt(2/S),
// DR = D0/(S-1), DA = S D0/(S-1) (Sec. II.B Eqs. 11-14; S = 2 in the minimal
// potential); zeta = ZS sum_k f_C g(theta) with g = (cos - h)^2 and ZS = beta
// (minimal), or g = g^T = gamma + K t^2 / (d^2 + t^2), t = cos - h,
// K = gamma c^2 / d^2 and ZS = 1 (Tersoff form, Sec. II.A Eq. 8).
enum ParamIndex {
    P_AA = 0,       // mu log2(e)
    P_R0HI = 1,     // r0 (float: high part)
    P_R0LO = 2,     // r0 - r0_hi (float only)
    P_DR = 3,
    P_DA = 4,
    P_AR = 5,       // lambda log2(e)
    P_ZS = 6,       // zeta scale: beta, or 1
    P_N = 7,
    P_NINV2N = 8,   // -1 / (2 n)
    P_H = 9,
    P_VALID = 10,   // 1 if the candidate is inside the potential's domain
    P_HMU = 11,     // mu / 2
    P_CCS = 12,     // gradient coefficient scale: beta / 2, or 1 / 2
    // float records: low parts (value - float(value)) of the parameters the
    // float64 energy terms use; zero in double records
    P_AALO = 13,
    P_DRLO = 14,
    P_NLO = 15,
    P_NINV2NLO = 16,
    P_ARLO = 17,
    P_DALO = 18,
    P_HLAMBDA = 19, // lambda / 2
    // Tersoff angular function
    P_GAM = 20,     // gamma
    P_K = 21,       // gamma c^2 / d^2
    P_D2 = 22,      // d^2
    P_KD2 = 23,     // K d^2
    P_HLO = 24      // h - float(h) (float records; zero in double records)
};

struct Item {       // one (structure, candidate range) work item of the batched kernel
    int s;
    int c0;
    int nc;
    int cost;       // relative cost used for scheduling
};

template <typename S>
struct GeomArrays {
    const S* ux; const S* uy; const S* uz;
    const S* rhi; const S* rlo; const S* rinv;
    const S* fc; const S* hfcp;     // f_C and f_C'/2
    // float only: the same geometry packed per bond slot as two 4-vectors,
    // (ux, uy, uz, r_hi) and (r_lo, 1/r, f_C, f_C'/2), [kcap][N] each
    const float4* pk0; const float4* pk1;
};

struct SetDev {
    int S, N, kcap, nb, nslots;
    const int* st_off; const int* st_boff; const int* st_npad; const int* st_kmax;
    const int* st_slot;
    const int* st_xsize;                        // exchange slots of one replica
    const int* perm; const int* nnb; const int* lbo;
    const int* xbase;                           // [N] first exchange slot of the atom
    const int* rev;                             // [kcap][N] exchange slot of the reverse bond
    const int* revc;                            // [kcap][N] structure-local CSR index of it
    const int* jl;                              // [kcap][N] structure-local neighbour atom
    GeomArrays<float> gf;
    GeomArrays<double> gd;
    // [15][N] cos(theta_jk) of the bond pairs j < k < 6, pair k (k - 1) / 2 + j:
    // float64 unit-vector products rounded once (zero for padding bonds)
    const float* gcs;
    const float* fref32;  const double* fref64; // [3][N] sorted order
};

// Pairs of bonds whose cos(theta) the pair table holds (bonds 0-5).
constexpr int kCosPairs = 15;

// ---------------------------------------------------------------------------
// Device math.  float: the hardware transcendental instructions (v_exp_f32,
// v_log_f32, v_rcp_f32); arguments on the hot path stay in the normal range.
// double: the ROCm device math library.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float dexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float dlog2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float drcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double dexp2(double x) { return exp2(x); }
__device__ __forceinline__ double dlog2(double x) { return log2(x); }
__device__ __forceinline__ double drcp(double x) { return 1.0 / x; }



// float64 2^y for the energy terms of the float path: about 1e-12 relative
// error, finite arguments only.  y = k + f with k = rint(y), |f| <= 1/2;
// 2^f = e^(f ln 2) by its Taylor series to degree 8 (remainder below
// (ln2/2)^9 / 9! e^(ln2/2) < 3e-10: under 5e-9 eV on a 15 eV energy term).
__device__ __forceinline__ double exp2_acc(double y) {
    const double k = __builtin_rint(y);
    const double f = y - k;
    double p = 1.321548679014431e-06;           // (ln 2)^i / i!, i = 8 .. 0
    p = p * f + 1.5252733804059841e-05;
    p = p * f + 0.0001540353039338161;
    p = p * f + 0.0013333558146428443;
    p = p * f + 0.009618129107628477;
    p = p * f + 0.05550410866482158;
    p = p * f + 0.24022650695910072;
    p = p * f + 0.6931471805599453;
    p = p * f + 1.0;
    return __builtin_amdgcn_ldexp(p, (int)k);
}

template <typename S>
struct Consts;
template <>
struct Consts<float> {
    static constexpr float ln2 = 0.693147180559945309f;
};
template <>
struct Consts<double> {
    static constexpr double ln2 = 0.693147180559945309;
};

// Forward-mode derivative with respect to K of the six parameters (which
// ones is set where the parameter record is seeded).
template <typename S, int K = 6>
struct Dual {
    S v;
    S d[K];
};

template <typename T>
struct DualOf { static constexpr int tangents = 0; };
template <typename S, int K>
struct DualOf<Dual<S, K>> { static constexpr int tangents = K; };

template <typename S, int K>
__device__ __forceinline__ Dual<S, K> dconst(S v) {
    Dual<S, K> r;
    r.v = v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = S(0);
    return r;
}

template <typename S> __device__ __forceinline__ S val(S a) { return a; }
template <typename S, int K> __device__ __forceinline__ S val(const Dual<S, K>& a) { return a.v; }

template <typename S, int K>
__device__ __forceinline__ Dual<S, K> operator+(const Dual<S, K>& a, const Dual<S, K>& b) {
    Dual<S, K> r; r.v = a.v + b.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] + b.d[k];
    return r;
}
template <typename S, int K>
__device__ __forceinline__ Dual<S, K> operator-(const Dual<S, K>& a, const Dual<S, K>& b) {
    Dual<S, K> r; r.v = a.v - b.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] - b.d[k];
    return r;
}
template <typename S, int K>
__device__ __forceinline__ Dual<S, K> operator-(const Dual<S, K>& a) {
    Dual<S, K> r; r.v = -a.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = -a.d[k];
    return r;
}
template <typename S, int K>
__device__ __forceinline__ Dual<S, K> operator*(const Dual<S, K>& a, const Dual<S, K>& b) {
    Dual<S, K> r; r.v = a.v * b.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
template <typename S, int K>
__device__ __forceinline__ Dual<S, K> operator*(const Dual<S, K>& a, S b) {
    Dual<S, K> r; r.v = a.v * b;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b;
    return r;
}
template <typename S, int K>
__device__ __forceinline__ Dual<S, K> operator*(S b, const Dual<S, K>& a) { return a * b; }
template <typename S, int K>
__device__ __forceinline__ Dual<S, K> operator+(const Dual<S, K>& a, S b) {
    Dual<S, K> r = a; r.v += b; return r;
}
template <typename S, int K>
__device__ __forceinline__ Dual<S, K> operator+(S b, const Dual<S, K>& a) { return a + b; }
template <typename S, int K>
__device__ __forceinline__ Dual<S, K> operator-(const Dual<S, K>& a, S b) {
    Dual<S, K> r = a; r.v -= b; return r;
}
template <typename S, int K>
__device__ __forceinline__ Dual<S, K> operator-(S b, const Dual<S, K>& a) { return (-a) + b; }
template <typename S, int K>
__device__ __forceinline__ Dual<S, K> dexp2(const Dual<S, K>& a) {
    Dual<S, K> r; r.v = dexp2(a.v);
    const S g = r.v * Consts<S>::ln2;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = g * a.d[k];
    return r;
}
template <typename S, int K>
__device__ __forceinline__ Dual<S, K> dlog2(const Dual<S, K>& a) {
    Dual<S, K> r; r.v = dlog2(a.v);
    const S g = drcp(a.v * Consts<S>::ln2);
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = g * a.d[k];
    return r;
}
template <typename S, int K>
__device__ __forceinline__ Dual<S, K> drcp(const Dual<S, K>& a) {
    Dual<S, K> r; r.v = drcp(a.v);
    const S g = -r.v * r.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = g * a.d[k];
    return r;
}
template <typename S, int K>
__device__ __forceinline__ Dual<S, K> dselect(bool c, const Dual<S, K>& a, const Dual<S, K>& b) {
    Dual<S, K> r; r.v = c ? a.v : b.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = c ? a.d[k] : b.d[k];
    return r;
}
template <typename S>
__device__ __forceinline__ S dselect(bool c, S a, S b) { return c ? a : b; }

template <typename V, typename S>
__device__ __forceinline__ V vconst(S v) {
    if constexpr (sizeof(V) == sizeof(S)) return v; else return dconst<S, DualOf<V>::tangents>(v);
}

// ---------------------------------------------------------------------------
// Host-side helpers shared by the translation units.
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
int hip_fail(hipError_t e, const char* what);

}  // namespace mt
