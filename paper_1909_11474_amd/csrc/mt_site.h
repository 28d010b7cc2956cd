// Per-atom evaluation of the Tersoff site energy for one candidate: the
// minimal potential, or the nine-parameter Tersoff form.
//
// One thread owns one atom i with M bonds (compile-time M, padded bonds have
// f_C = f_C' = 0 and contribute nothing).  For a candidate parameter record it
// computes the site energy U_i and the bond gradients G_ij = dU_i/dr_ij:
//
//   zeta_ij = beta sum_{k != j} f_C(r_ik) (cos theta_ijk - h)^2          (Sec. II.A Eq. 7, Sec. II.B Eq. 10)
//   b_ij = (1 + zeta^n)^(-1/(2n)) (b = 1 at zeta = 0)                    (Sec. II.A Eq. 6)
//   U_i = 1/2 sum_j f_C(r_ij) [f_R - b_ij f_A]                            (Sec. II.A Eqs. 2-3)
//   with S = 2:  f_R = D0 x^2,  f_A = 2 D0 x,  x = exp(-alpha (r - r0))  (Sec. II.B Eqs. 11-14)
//
// G_ij is the exact derivative of U_i.  Writing C_j = -f_C fA b'/2 for the
// coefficient of d zeta_ij, c~_j = 2 beta C_j, t_jk = cos_jk - h and
// q_jk = (c~_j f_C,k + c~_k f_C,j) t_jk, the gradient decomposes into a radial
// part along r^_j and a transverse sum:
//   G_j = [ D_j + f_C'_j/2 sum_k c~_k t_jk^2 - (1/r_j) r^_j . V_j ] r^_j + (1/r_j) V_j,
//   V_j = sum_k q_jk r^_k,
//   D_j = 1/2 [ f_C'_j (f_R - b f_A) + f_C,j alpha (b f_A - 2 f_R) ]
// (the radial term uses sum_k q_jk cos_jk = r^_j . V_j).  Every unordered bond
// pair (j, k) is visited once in each of the forward (zeta) and backward
// (gradient) sweeps.
//
// The Tersoff form (Sec. II.A Eqs. 2-8 with Eqs. 11-14 for general S) replaces
// beta (cos - h)^2 by g^T(theta), t^2 by g^T in the P sums, t by g^T'/2 in q_jk,
// and takes f_R, f_A with their own exponents lambda = alpha sqrt(2S),
// mu = alpha sqrt(2/S); then D_j = 1/2 [f_C' (f_R - b f_A) + f_C (mu b f_A - lambda f_R)].
//
// V is the value type (float, double, or Dual<> for parameter derivatives);
// S is the geometry type.  The code is written once for all of them.
#pragma once

#include <type_traits>

#include "mt_common.h"

namespace mt {

template <typename S, int M>
struct Geo {
    static constexpr int NP = M * (M - 1) / 2;
    static constexpr bool kCache = NP <= 15;       // keep cos(theta) in registers for M <= 6
    S ux[M > 0 ? M : 1], uy[M > 0 ? M : 1], uz[M > 0 ? M : 1];
    S rhi[M > 0 ? M : 1], rlo[M > 0 ? M : 1], rinv[M > 0 ? M : 1];
    S fc[M > 0 ? M : 1], hfcp[M > 0 ? M : 1];     // f_C and f_C'/2
    S cs[kCache && NP > 0 ? NP : 1];

    __device__ __forceinline__ S cosjk(int j, int k, int pidx) const {
        if constexpr (kCache && NP > 0) {
            return cs[pidx];
        } else {
            (void)pidx;
            return ux[j] * ux[k] + uy[j] * uy[k] + uz[j] * uz[k];
        }
    }

    // Gcs (float geometry only): the set's pair table of cos(theta) values,
    // formed from the float64 unit vectors and rounded once; from float unit
    // vectors they carry up to ~2e-7 absolute error, which zeta passes on to
    // the energy through (cos - h)^2.
    // rows: neighbour rows the arrays hold (a variant wider than the set's
    // capacity reads the rows past it as padding bonds)
    __device__ __forceinline__ void load(const GeomArrays<S>& G, int N, int atom, bool active,
                                         const float* Gcs = nullptr, int rows = M) {
        if constexpr (sizeof(S) == 4) {
            if (G.pk0) {
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const size_t o = (size_t)m * N + atom;
                    const bool ok = active && m < rows;
                    const float4 a = ok ? G.pk0[o] : make_float4(0.f, 0.f, 0.f, 3.f);
                    const float4 b = ok ? G.pk1[o] : make_float4(0.f, 0.f, 0.f, 0.f);
                    ux[m] = a.x; uy[m] = a.y; uz[m] = a.z; rhi[m] = a.w;
                    rlo[m] = b.x; rinv[m] = b.y; fc[m] = b.z; hfcp[m] = b.w;
                }
                if constexpr (kCache && NP > 0) {
                    static_assert(M <= 6, "the pair table holds bonds 0-5");
                    if (Gcs && active) {
                        int p = 0;
#pragma unroll
                        for (int j = 0; j < M; ++j)
#pragma unroll
                            for (int k = j + 1; k < M; ++k)
                                cs[p++] = k < rows ? Gcs[(size_t)(k * (k - 1) / 2 + j) * N + atom] : S(0);
                        return;
                    }
                }
                cache_cos();
                return;
            }
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const size_t o = (size_t)m * N + atom;
            const bool ok = active && m < rows;
            ux[m] = ok ? G.ux[o] : S(0);
            uy[m] = ok ? G.uy[o] : S(0);
            uz[m] = ok ? G.uz[o] : S(0);
            rhi[m] = ok ? G.rhi[o] : S(3);
            rlo[m] = (ok && G.rlo) ? G.rlo[o] : S(0);
            rinv[m] = ok ? G.rinv[o] : S(0);
            fc[m] = ok ? G.fc[o] : S(0);
            hfcp[m] = ok ? G.hfcp[o] : S(0);
        }
        cache_cos();
    }

    __device__ __forceinline__ void cache_cos() {
        if constexpr (kCache && NP > 0) {
            int p = 0;
#pragma unroll
            for (int j = 0; j < M; ++j)
#pragma unroll
                for (int k = j + 1; k < M; ++k) cs[p++] = ux[j] * ux[k] + uy[j] * uy[k] + uz[j] * uz[k];
        }
    }
};

// Decoded parameters of one candidate.  Full selects the Tersoff angular
// function g^T and independent pair exponents (the nine-parameter form); the
// minimal potential has g = (cos - h)^2 and lambda = 2 mu.
template <typename V, typename S, bool Full = false>
struct Cand {
    static constexpr bool kFull = Full;
    V aA, aR, r0hi, r0lo, DR, DA, hmu, hlambda, zs, ccs, n, ninv2n, h;
    V gam, K, d2, Kd2;               // g^T = gam + K t^2 / (d2 + t^2)
    S valid;
    S aAlo, aRlo, DRlo, DAlo, nlo, ninv2nlo;   // low parts for the float64 energy terms
    S hlo;                                      // h - float(h): zeta of the float path
};

// Type of the site energy: float64 for the float path (its energy terms are
// evaluated in float64), the value type otherwise.
template <typename V>
struct EnergyOf { using type = V; };
template <>
struct EnergyOf<float> { using type = double; };

// The minimal record leaves the Tersoff-form slots unwritten; its candidate
// takes lambda = 2 mu and does not read them.
template <typename S, bool Full>
__device__ __forceinline__ void load_cand(const S* __restrict__ p, Cand<S, S, Full>& c) {
    c.aA = p[P_AA]; c.r0hi = p[P_R0HI]; c.r0lo = p[P_R0LO];
    c.DR = p[P_DR]; c.DA = p[P_DA]; c.hmu = p[P_HMU];
    c.zs = p[P_ZS]; c.ccs = p[P_CCS]; c.n = p[P_N]; c.ninv2n = p[P_NINV2N]; c.h = p[P_H];
    c.aAlo = p[P_AALO]; c.DRlo = p[P_DRLO]; c.nlo = p[P_NLO]; c.ninv2nlo = p[P_NINV2NLO];
    c.hlo = p[P_HLO];
    c.valid = p[P_VALID];
    if constexpr (Full) {
        c.aR = p[P_AR]; c.hlambda = p[P_HLAMBDA]; c.aRlo = p[P_ARLO]; c.DAlo = p[P_DALO];
        c.gam = p[P_GAM]; c.K = p[P_K]; c.d2 = p[P_D2]; c.Kd2 = p[P_KD2];
    } else {
        c.aR = S(2) * c.aA; c.hlambda = S(2) * c.hmu; c.aRlo = S(2) * c.aAlo; c.DAlo = S(2) * c.DRlo;
        c.gam = S(0); c.K = S(0); c.d2 = S(1); c.Kd2 = S(0);
    }
}

// Seeds K parameter directions, parameters Base .. Base + K - 1 of the
// minimal potential's (D0, alpha, r0, beta, n, h).
template <int Base, typename S, int K>
__device__ __forceinline__ void load_cand(const S* __restrict__ p, Cand<Dual<S, K>, S, false>& c) {
    const S log2e = S(1.4426950408889634);
    c.aA = dconst<S, K>(p[P_AA]);
    c.aR = dconst<S, K>(S(2) * p[P_AA]);
    c.r0hi = dconst<S, K>(p[P_R0HI]);
    c.r0lo = dconst<S, K>(p[P_R0LO]);
    c.DR = dconst<S, K>(p[P_DR]);
    c.DA = dconst<S, K>(p[P_DA]);
    c.hmu = dconst<S, K>(p[P_HMU]);
    c.hlambda = dconst<S, K>(S(2) * p[P_HMU]);
    c.zs = dconst<S, K>(p[P_ZS]);
    c.ccs = dconst<S, K>(p[P_CCS]);
    c.n = dconst<S, K>(p[P_N]);
    c.ninv2n = dconst<S, K>(p[P_NINV2N]);
    c.h = dconst<S, K>(p[P_H]);
#pragma unroll
    for (int t = 0; t < K; ++t) {
        switch (Base + t) {
            // S = 2: DR = D0, DA = 2 D0, mu = alpha, lambda = 2 alpha
            case 0: c.DR.d[t] = S(1); c.DA.d[t] = S(2); break;
            case 1:
                c.aA.d[t] = log2e; c.hmu.d[t] = S(0.5);
                c.aR.d[t] = S(2) * log2e; c.hlambda.d[t] = S(1);
                break;
            case 2: c.r0hi.d[t] = S(1); break;
            case 3: c.zs.d[t] = S(1); c.ccs.d[t] = S(0.5); break;
            // d/dn (-1/(2n)) = 1/(2n^2)
            case 4: c.n.d[t] = S(1); c.ninv2n.d[t] = S(2) * p[P_NINV2N] * p[P_NINV2N]; break;
            case 5: c.h.d[t] = S(1); break;
        }
    }
    c.valid = p[P_VALID];
    c.hlo = S(0);
}

// Seeds K parameter directions, parameters Base .. Base + K - 1 of the
// Tersoff form's (D0, alpha, r0, S, gamma, n, c, d, h): values from the record
// p, tangents of the record's fields from the candidate's x (float64):
//   DR = D0/(S-1), DA = S D0/(S-1), mu = alpha sqrt(2/S), lambda = alpha sqrt(2S),
//   K = gamma c^2/d^2, d^2, K d^2 = gamma c^2, -1/(2n).
template <int Base, typename S, int K>
__device__ __forceinline__ void load_cand(const S* __restrict__ p, const double* __restrict__ x,
                                          Cand<Dual<S, K>, S, true>& c) {
    const double log2e = 1.4426950408889634;
    c.aA = dconst<S, K>(p[P_AA]);
    c.aR = dconst<S, K>(p[P_AR]);
    c.r0hi = dconst<S, K>(p[P_R0HI]);
    c.r0lo = dconst<S, K>(p[P_R0LO]);
    c.DR = dconst<S, K>(p[P_DR]);
    c.DA = dconst<S, K>(p[P_DA]);
    c.hmu = dconst<S, K>(p[P_HMU]);
    c.hlambda = dconst<S, K>(p[P_HLAMBDA]);
    c.zs = dconst<S, K>(p[P_ZS]);
    c.ccs = dconst<S, K>(p[P_CCS]);
    c.n = dconst<S, K>(p[P_N]);
    c.ninv2n = dconst<S, K>(p[P_NINV2N]);
    c.h = dconst<S, K>(p[P_H]);
    c.gam = dconst<S, K>(p[P_GAM]);
    c.K = dconst<S, K>(p[P_K]);
    c.d2 = dconst<S, K>(p[P_D2]);
    c.Kd2 = dconst<S, K>(p[P_KD2]);
    const double D0 = x[0], al = x[1], Sl = x[3], gam = x[4], n = x[5], cc = x[6], d = x[7];
    const double rs = sqrt(2.0 / Sl), rl = sqrt(2.0 * Sl), sm1 = Sl - 1.0;
#pragma unroll
    for (int t = 0; t < K; ++t) {
        switch (Base + t) {
            case 0: c.DR.d[t] = (S)(1.0 / sm1); c.DA.d[t] = (S)(Sl / sm1); break;
            case 1:
                c.aA.d[t] = (S)(rs * log2e); c.aR.d[t] = (S)(rl * log2e);
                c.hmu.d[t] = (S)(0.5 * rs); c.hlambda.d[t] = (S)(0.5 * rl);
                break;
            case 2: c.r0hi.d[t] = S(1); break;
            case 3: {
                // d sqrt(2/S)/dS = -sqrt(2/S)/(2S), d sqrt(2S)/dS = sqrt(2S)/(2S)
                const double dD = -D0 / (sm1 * sm1), ts = 0.5 / Sl;
                c.DR.d[t] = (S)dD; c.DA.d[t] = (S)dD;
                c.aA.d[t] = (S)(-al * rs * log2e * ts); c.aR.d[t] = (S)(al * rl * log2e * ts);
                c.hmu.d[t] = (S)(-0.5 * al * rs * ts); c.hlambda.d[t] = (S)(0.5 * al * rl * ts);
                break;
            }
            case 4: c.gam.d[t] = S(1); c.K.d[t] = (S)(cc * cc / (d * d)); c.Kd2.d[t] = (S)(cc * cc); break;
            // d/dn (-1/(2n)) = 1/(2n^2)
            case 5: c.n.d[t] = S(1); c.ninv2n.d[t] = (S)(0.5 / (n * n)); break;
            case 6: c.K.d[t] = (S)(2.0 * gam * cc / (d * d)); c.Kd2.d[t] = (S)(2.0 * gam * cc); break;
            case 7: c.K.d[t] = (S)(-2.0 * gam * cc * cc / (d * d * d)); c.d2.d[t] = (S)(2.0 * d); break;
            case 8: c.h.d[t] = S(1); break;
        }
    }
    c.valid = p[P_VALID];
    c.hlo = S(0);
}

// Angular function and half its derivative for t = cos(theta) - h:
// minimal g = t^2, g'/2 = t; Tersoff g^T = gam + K t^2 / (d^2 + t^2),
// g'/2 = K d^2 t / (d^2 + t^2)^2 (Sec. II.A Eq. 8, written without the
// cancellation of 1 + c^2/d^2 - c^2/(d^2 + t^2)).
template <bool Full, typename V, typename P>
__device__ __forceinline__ V ang_g(const P& p, const V& t) {
    const V t2 = t * t;
    if constexpr (Full) return p.gam + (p.K * t2) * drcp(p.d2 + t2);
    else return t2;
}
template <bool Full, typename V, typename P>
__device__ __forceinline__ void ang_g_dg(const P& p, const V& t, V& gv, V& hg) {
    const V t2 = t * t;
    if constexpr (Full) {
        const V r = drcp(p.d2 + t2);
        gv = p.gam + (p.K * t2) * r;
        hg = ((p.Kd2 * t) * r) * r;
    } else {
        gv = t2;
        hg = t;
    }
}

// Make the compiler treat the values as changed here (no instruction is
// emitted): expressions of them after this point are recomputed, not reused.
template <typename S, int N>
__device__ __forceinline__ void opaque(S (&a)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) asm volatile("" : "+v"(a[i]));
}

// Largest coordination whose backward sweep runs over unordered bond pairs.
constexpr int kPairwiseMax = 8;

// The site routine.  It hands each bond gradient G_j to sink(j, Gx, Gy, Gz);
// PerBond selects the one-bond-at-a-time backward sweep (for large M, or for
// dual numbers, whose per-bond state is K + 1 times larger), which emits G_j
// as soon as it is complete.
// Fresh: treat the geometry as new, so that nothing computed from it by an
// earlier call in the same loop iteration is kept alive for reuse (repeated
// dual passes over the same site would otherwise hold every shared primal
// value across passes).  The barriers act on the caller's geometry in place
// (they change no value), so no second copy of it becomes live.
// SerialE64: keep the float64 energy chains of the bonds one after another
// (fewer live registers; a kernel with other wavefronts to switch to loses
// nothing), or let them interleave (a kernel that runs about one wavefront per
// SIMD needs the instruction-level parallelism).
template <typename V, typename S, int M, bool Energy64, bool PerBond, bool Fresh = false,
          bool Full = false, bool SerialE64 = true, typename Sink>
__device__ __forceinline__ void site_eval_sink(Geo<S, M>& g, const Cand<V, S, Full>& p,
                                               typename EnergyOf<V>::type& U, Sink&& sink) {
    constexpr int MM = M > 0 ? M : 1;
    if constexpr (Fresh && M > 0) {
        opaque(g.rhi); opaque(g.rlo); opaque(g.rinv); opaque(g.fc); opaque(g.hfcp);
        if constexpr (Geo<S, M>::kCache && Geo<S, M>::NP > 0) opaque(g.cs);
    }
    if constexpr ((Fresh || !Geo<S, M>::kCache) && M > 1) {
        // cos(theta) is not cached for larger M: keep the compiler from
        // hoisting the M (M - 1) / 2 values out of the candidate loop (they
        // would not fit in registers and go to scratch)
        opaque(g.ux);
        opaque(g.uy);
        opaque(g.uz);
    }
    // Energy64 (float path): the pair terms and the bond order of the energy
    // are evaluated with float64 exponentials (below), and zeta takes h as a
    // float hi/lo pair, so that a float rounding of h does not shift every
    // (cos - h)^2 of a candidate the same way.
    constexpr bool kE64 = Energy64 && std::is_same<V, float>::value;
    V zeta[MM];
#pragma unroll
    for (int j = 0; j < M; ++j) zeta[j] = vconst<V, S>(S(0));
    {
        int pidx = 0;
#pragma unroll
        for (int j = 0; j < M; ++j) {
#pragma unroll
            for (int k = j + 1; k < M; ++k) {
                const S c = g.cosjk(j, k, pidx++);
                V t;
                if constexpr (kE64) t = (c - p.h) - p.hlo;
                else t = c - p.h;
                const V gv = ang_g<Full>(p, t);
                zeta[j] = zeta[j] + g.fc[k] * gv;
                zeta[k] = zeta[k] + g.fc[j] * gv;
            }
        }
    }
    // Energy64: in float32 the rounding of f_R and b f_A (up to ~15 eV each
    // for parameters inside the fitting box) and the one-ulp errors of the
    // hardware exponentials reach 1e-6 eV per bond.  The exponentials whose
    // errors reach the energy at full weight, e^{-mu (r - r0)} and b, are
    // taken in float64 (the argument of b from the float logarithm of
    // 1 + zeta^n, whose error enters b damped by zeta^n / (1 + zeta^n) / 2n),
    // and the pair energy is formed in float64.  Their float32 roundings feed
    // the gradient.
    V cc[MM], D[MM];
    V usum = vconst<V, S>(S(0));
    double usum64 = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const V z = zeta[j] * p.zs;
        // zeta = 0 (no other neighbour inside the cutoff, or all at g = 0):
        // zeta^n = 0 exactly, so b = 1 and db/dzeta * zeta^n-terms vanish
        const bool pos = val(z) > S(0);
        const V zsafe = dselect(pos, z, vconst<V, S>(S(1)));
        V eA, zn, b;
        [[maybe_unused]] V eR;
        if constexpr (kE64) {
            // float64 copies of the bond's geometry are made here, per candidate:
            // hoisted out of the candidate loop they would hold 6 M registers
            S rh = g.rhi[j], rl = g.rlo[j], fcj = g.fc[j];
            asm volatile("" : "+v"(rh), "+v"(rl), "+v"(fcj));
            const double dl = ((double)rh - (double)p.r0hi) + ((double)rl - (double)p.r0lo);
            const double eA64 = exp2_acc(-(((double)p.aA + (double)p.aAlo) * dl));
            const float zn32 = pos ? dexp2(p.n * dlog2(zsafe)) : 0.f;
            const double b64 =
                exp2_acc(((double)p.ninv2n + (double)p.ninv2nlo) * (double)dlog2(1.f + zn32));
            const double DR = (double)p.DR + (double)p.DRlo;
            if constexpr (Full) {
                const double eR64 = exp2_acc(-(((double)p.aR + (double)p.aRlo) * dl));
                const double DA = (double)p.DA + (double)p.DAlo;
                usum64 += (double)fcj * (DR * eR64 - b64 * (DA * eA64));
                eR = (float)eR64;
            } else {
                // DA = 2 DR, e_R = e_A^2
                usum64 += (double)fcj * (DR * eA64 * (eA64 - 2.0 * b64));
            }
            eA = (float)eA64;
            zn = zn32;
            b = (float)b64;
        } else {
            const V delta = (g.rhi[j] - p.r0hi) + (g.rlo[j] - p.r0lo);
            eA = dexp2(-(p.aA * delta));
            if constexpr (Full) eR = dexp2(-(p.aR * delta));
            zn = dselect(pos, dexp2(p.n * dlog2(zsafe)), vconst<V, S>(S(0)));
            b = dexp2(p.ninv2n * dlog2(S(1) + zn));
        }
        const V onep = S(1) + zn;
        V fR;
        if constexpr (Full) fR = p.DR * eR;
        else fR = p.DR * (eA * eA);               // e_R = e_A^2
        const V fA = p.DA * eA;
        const V diff = fR - b * fA;           // one rounding (fused multiply-add)
        const V bfA = b * fA;
        if constexpr (!kE64) usum = usum + g.fc[j] * diff;
        // D = 1/2 [f_C' (f_R - b f_A) + f_C (mu b f_A - lambda f_R)]
        if constexpr (Full) D[j] = g.hfcp[j] * diff + g.fc[j] * (p.hmu * bfA - p.hlambda * fR);
        else D[j] = g.hfcp[j] * diff + (p.hmu * g.fc[j]) * (bfA - S(2) * fR);
        // c~ = -ZS f_C f_A db/dzeta with db/dzeta = -b zeta^n / (2 zeta (1 + zeta^n))
        cc[j] = (p.ccs * g.fc[j]) * (bfA * zn) * drcp(zsafe * onep);
        // per-bond sweep: keep the scheduler from interleaving all M bonds' chains
        // (about ten live values each; float64 ones in the energy mode)
        if constexpr (PerBond || (kE64 && SerialE64)) __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (kE64) U = 0.5 * usum64; else U = S(0.5) * usum;
    if constexpr (PerBond) {
        // One bond at a time, visiting each pair from both ends.
        // About 1.5x the backward arithmetic of the pairwise sweep below, but
        // only four running sums are live instead of 4 M, which keeps the
        // kernel out of scratch spills.  The barrier stops the compiler from
        // keeping the forward sweep's per-pair terms (about 2 M^2 values)
        // alive for reuse here.
        opaque(g.ux);
        opaque(g.uy);
        opaque(g.uz);
#pragma unroll
        for (int j = 0; j < M; ++j) {
            V vx = vconst<V, S>(S(0)), vy = vx, vz = vx, pp = vx;
#pragma unroll
            for (int k = 0; k < M; ++k) {
                if (k == j) continue;
                const S c = g.ux[j] * g.ux[k] + g.uy[j] * g.uy[k] + g.uz[j] * g.uz[k];
                const V t = c - p.h;
                V gv, hg;
                ang_g_dg<Full>(p, t, gv, hg);
                const V q = (cc[j] * g.fc[k] + cc[k] * g.fc[j]) * hg;
                vx = vx + q * g.ux[k]; vy = vy + q * g.uy[k]; vz = vz + q * g.uz[k];
                if constexpr (Full) pp = pp + cc[k] * gv;
                else pp = pp + (cc[k] * t) * t;
            }
            const V uv = g.ux[j] * vx + g.uy[j] * vy + g.uz[j] * vz;
            const V rad = D[j] + g.hfcp[j] * pp - uv * g.rinv[j];
            sink(j, rad * g.ux[j] + vx * g.rinv[j], rad * g.uy[j] + vy * g.rinv[j],
                 rad * g.uz[j] + vz * g.rinv[j]);
            __builtin_amdgcn_sched_barrier(0);
        }
        return;
    }
    V Vx[MM], Vy[MM], Vz[MM], Pp[MM];
#pragma unroll
    for (int j = 0; j < M; ++j) {
        Vx[j] = Vy[j] = Vz[j] = Pp[j] = vconst<V, S>(S(0));
    }
    {
        int pidx = 0;
#pragma unroll
        for (int j = 0; j < M; ++j) {
#pragma unroll
            for (int k = j + 1; k < M; ++k) {
                const S c = g.cosjk(j, k, pidx++);
                const V t = c - p.h;
                V gv, hg;
                ang_g_dg<Full>(p, t, gv, hg);
                const V q = (cc[j] * g.fc[k] + cc[k] * g.fc[j]) * hg;
                Vx[j] = Vx[j] + q * g.ux[k]; Vy[j] = Vy[j] + q * g.uy[k]; Vz[j] = Vz[j] + q * g.uz[k];
                Vx[k] = Vx[k] + q * g.ux[j]; Vy[k] = Vy[k] + q * g.uy[j]; Vz[k] = Vz[k] + q * g.uz[j];
                Pp[j] = Pp[j] + cc[k] * gv;
                Pp[k] = Pp[k] + cc[j] * gv;
            }
        }
    }
    // sum_k q_jk cos_jk = u_j . V_j, so the radial part needs no per-pair term
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const V uv = g.ux[j] * Vx[j] + g.uy[j] * Vy[j] + g.uz[j] * Vz[j];
        const V rad = D[j] + g.hfcp[j] * Pp[j] - uv * g.rinv[j];
        sink(j, rad * g.ux[j] + Vx[j] * g.rinv[j], rad * g.uy[j] + Vy[j] * g.rinv[j],
             rad * g.uz[j] + Vz[j] * g.rinv[j]);
    }
}

// The site routine with the bond gradients returned in arrays.
template <typename V, typename S, int M, bool Energy64 = false, bool Full = false, bool SerialE64 = true>
__device__ __forceinline__ void site_eval(Geo<S, M>& g, const Cand<V, S, Full>& p,
                                          typename EnergyOf<V>::type& U,
                                          V* __restrict__ Gx, V* __restrict__ Gy,
                                          V* __restrict__ Gz) {
    site_eval_sink<V, S, M, Energy64, (M > kPairwiseMax), false, Full, SerialE64>(
        g, p, U, [&](int j, const V& x, const V& y, const V& z) {
            Gx[j] = x;
            Gy[j] = y;
            Gz[j] = z;
        });
}

// Cross-lane exchanges of a double, 32 bits at a time.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
constexpr int kDppXor1 = 0xB1;         // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // lane l <-> 7 - l within 8 (opposite bit 2)
constexpr int kDppMirror = 0x140;      // lane l <-> 15 - l within 16 (opposite bit 3)

// Transpose step over lane bit m: lanes with the bit clear keep a (and add the
// partner's a), lanes with it set keep b.  permlane{16,32}_swap exchange the
// upper half of the first operand with the lower half of the second, so the
// two returned halves always sum to own kept value + partner's kept value.
template <int M>
__device__ __forceinline__ double tstep(double a, double b) {
    if constexpr (M == 32 || M == 16) {
        const long long ia = __double_as_longlong(a), ib = __double_as_longlong(b);
        const unsigned alo = (unsigned)ia, ahi = (unsigned)(ia >> 32);
        const unsigned blo = (unsigned)ib, bhi = (unsigned)(ib >> 32);
        unsigned r0lo, r1lo, r0hi, r1hi;
        if constexpr (M == 32) {
            auto l = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
            auto h = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
            r0lo = l[0]; r1lo = l[1]; r0hi = h[0]; r1hi = h[1];
        } else {
            auto l = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
            auto h = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
            r0lo = l[0]; r1lo = l[1]; r0hi = h[0]; r1hi = h[1];
        }
        const double x0 = __longlong_as_double(((long long)r0hi << 32) | r0lo);
        const double x1 = __longlong_as_double(((long long)r1hi << 32) | r1lo);
        return x0 + x1;
    } else {
        const bool h = (threadIdx.x & M) != 0;
        const double send = h ? a : b;
        const double keep = h ? b : a;
        constexpr int ctrl = M == 8 ? kDppMirror : (M == 4 ? kDppHalfMirror : (M == 2 ? kDppXor2 : kDppXor1));
        return keep + dpp_mov<ctrl>(send);
    }
}

template <int M>
__device__ __forceinline__ double bstep(double v) {
    constexpr int ctrl = M == 4 ? kDppHalfMirror : (M == 2 ? kDppXor2 : kDppXor1);
    return v + dpp_mov<ctrl>(v);
}

// Segmented transpose-reduction of 8 doubles over aligned groups of G lanes
// (G in 8, 16, 32, 64): three transpose steps over the top lane bits of the
// group, then butterfly steps over the rest.  Afterwards every lane holds the
// group sum of value index *vidx (bits of the transpose steps); lanes with
// (lane & (G/8 - 1)) == 0 are the writers.
template <int G>
__device__ __forceinline__ double group_reduce8_t(double* v, int* vidx) {
    constexpr int m1 = G / 2, m2 = G / 4, m3 = G / 8;
    const int lane = threadIdx.x & 63;
    double a4[4], a2[2];
#pragma unroll
    for (int k = 0; k < 4; ++k) a4[k] = tstep<m1>(v[k], v[k + 4]);
#pragma unroll
    for (int k = 0; k < 2; ++k) a2[k] = tstep<m2>(a4[k], a4[k + 2]);
    double r = tstep<m3>(a2[0], a2[1]);
    if constexpr (m3 > 4) r = bstep<4>(r);
    if constexpr (m3 > 2) r = bstep<2>(r);
    if constexpr (m3 > 1) r = bstep<1>(r);
    *vidx = ((lane & m1) ? 4 : 0) + ((lane & m2) ? 2 : 0) + ((lane & m3) ? 1 : 0);
    return r;
}

__device__ __forceinline__ double group_reduce8(double* v, int g, int* vidx) {
    switch (g) {
        case 8: return group_reduce8_t<8>(v, vidx);
        case 16: return group_reduce8_t<16>(v, vidx);
        case 32: return group_reduce8_t<32>(v, vidx);
        default: return group_reduce8_t<64>(v, vidx);
    }
}

__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int y = __shfl_xor(v, o, 64);
        v = v > y ? v : y;
    }
    return v;
}

}  // namespace mt
