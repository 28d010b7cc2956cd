// Per-atom evaluation of the minimal Tersoff potential for one candidate.
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
//   G_j = [ D_j + f_C'_j/2 sum_k c~_k t_jk^2 - (1/r_j) sum_k q_jk cos_jk ] r^_j
//         + (1/r_j) sum_k q_jk r^_k,
//   D_j = 1/2 [ f_C'_j (f_R - b f_A) + f_C,j alpha (b f_A - 2 f_R) ].
// Every unordered bond pair (j, k) is visited once in each of the forward
// (zeta) and backward (gradient) sweeps.
//
// V is the value type (float, double, or Dual<> for parameter derivatives);
// S is the geometry type.  The code is written once for all of them.
#pragma once

#include "mt_common.h"

namespace mt {

template <typename S, int M>
struct Geo {
    static constexpr int NP = M * (M - 1) / 2;
    static constexpr bool kCache = NP <= 15;       // keep cos(theta) in registers for M <= 6
    S ux[M > 0 ? M : 1], uy[M > 0 ? M : 1], uz[M > 0 ? M : 1];
    S rhi[M > 0 ? M : 1], rlo[M > 0 ? M : 1], rinv[M > 0 ? M : 1];
    S fc[M > 0 ? M : 1], fcp[M > 0 ? M : 1];
    S cs[kCache && NP > 0 ? NP : 1];

    __device__ __forceinline__ S cosjk(int j, int k, int pidx) const {
        if constexpr (kCache && NP > 0) {
            return cs[pidx];
        } else {
            (void)pidx;
            return ux[j] * ux[k] + uy[j] * uy[k] + uz[j] * uz[k];
        }
    }

    __device__ __forceinline__ void load(const GeomArrays<S>& G, int N, int atom, bool active) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const size_t o = (size_t)m * N + atom;
            ux[m] = active ? G.ux[o] : S(0);
            uy[m] = active ? G.uy[o] : S(0);
            uz[m] = active ? G.uz[o] : S(0);
            rhi[m] = active ? G.rhi[o] : S(3);
            rlo[m] = (active && G.rlo) ? G.rlo[o] : S(0);
            rinv[m] = active ? G.rinv[o] : S(0);
            fc[m] = active ? G.fc[o] : S(0);
            fcp[m] = active ? G.fcp[o] : S(0);
        }
        if constexpr (kCache && NP > 0) {
            int p = 0;
#pragma unroll
            for (int j = 0; j < M; ++j)
#pragma unroll
                for (int k = j + 1; k < M; ++k) cs[p++] = ux[j] * ux[k] + uy[j] * uy[k] + uz[j] * uz[k];
        }
    }
};

template <typename V, typename S>
struct Cand {
    V aL, r0hi, r0lo, D0, twoD0, alpha, beta, n, ninv2n, h;
    S valid;
};

template <typename S>
__device__ __forceinline__ void load_cand(const S* __restrict__ p, Cand<S, S>& c) {
    c.aL = p[P_AL]; c.r0hi = p[P_R0HI]; c.r0lo = p[P_R0LO]; c.D0 = p[P_D0]; c.twoD0 = p[P_2D0];
    c.alpha = p[P_ALPHA]; c.beta = p[P_BETA]; c.n = p[P_N]; c.ninv2n = p[P_NINV2N]; c.h = p[P_H];
    c.valid = p[P_VALID];
}

// Seeds the six parameter directions D0, alpha, r0, beta, n, h.
template <typename S>
__device__ __forceinline__ void load_cand(const S* __restrict__ p, Cand<Dual<S>, S>& c) {
    const S log2e = S(1.4426950408889634);
    c.aL = dconst<S>(p[P_AL]);        c.aL.d[1] = log2e;
    c.r0hi = dconst<S>(p[P_R0HI]);    c.r0hi.d[2] = S(1);
    c.r0lo = dconst<S>(p[P_R0LO]);
    c.D0 = dconst<S>(p[P_D0]);        c.D0.d[0] = S(1);
    c.twoD0 = dconst<S>(p[P_2D0]);    c.twoD0.d[0] = S(2);
    c.alpha = dconst<S>(p[P_ALPHA]);  c.alpha.d[1] = S(1);
    c.beta = dconst<S>(p[P_BETA]);    c.beta.d[3] = S(1);
    c.n = dconst<S>(p[P_N]);          c.n.d[4] = S(1);
    c.ninv2n = dconst<S>(p[P_NINV2N]);
    c.ninv2n.d[4] = S(2) * p[P_NINV2N] * p[P_NINV2N];     // d/dn (-1/(2n)) = 1/(2n^2)
    c.h = dconst<S>(p[P_H]);          c.h.d[5] = S(1);
    c.valid = p[P_VALID];
}

template <typename V, typename S, int M>
__device__ __forceinline__ void site_eval(const Geo<S, M>& g, const Cand<V, S>& p, V& U,
                                          V* __restrict__ Gx, V* __restrict__ Gy,
                                          V* __restrict__ Gz) {
    constexpr int MM = M > 0 ? M : 1;
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
                const V t = c - p.h;
                const V t2 = t * t;
                zeta[j] = zeta[j] + g.fc[k] * t2;
                zeta[k] = zeta[k] + g.fc[j] * t2;
            }
        }
    }
    V cc[MM], D[MM];
    V usum = vconst<V, S>(S(0));
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const V z = zeta[j] * p.beta;
        const V delta = (g.rhi[j] - p.r0hi) + (g.rlo[j] - p.r0lo);
        const V e = dexp2(-(p.aL * delta));
        const V fR = p.D0 * (e * e);
        const V fA = p.twoD0 * e;
        const bool pos = val(z) > S(0);
        const V zs = dselect(pos, z, vconst<V, S>(S(1)));
        const V zn = dexp2(p.n * dlog2(zs));
        const V onep = S(1) + zn;
        V b = dexp2(p.ninv2n * dlog2(onep));
        V bp = S(-0.5) * (b * zn) * drcp(zs * onep);
        b = dselect(pos, b, vconst<V, S>(S(1)));
        bp = dselect(pos, bp, vconst<V, S>(S(0)));
        const V diff = fR - b * fA;
        usum = usum + g.fc[j] * diff;
        D[j] = S(0.5) * (g.fcp[j] * diff + (g.fc[j] * p.alpha) * (b * fA - S(2) * fR));
        cc[j] = -(p.beta * (g.fc[j] * (fA * bp)));
    }
    U = S(0.5) * usum;
    V Vx[MM], Vy[MM], Vz[MM], A[MM], Pp[MM];
#pragma unroll
    for (int j = 0; j < M; ++j) {
        Vx[j] = Vy[j] = Vz[j] = A[j] = Pp[j] = vconst<V, S>(S(0));
    }
    {
        int pidx = 0;
#pragma unroll
        for (int j = 0; j < M; ++j) {
#pragma unroll
            for (int k = j + 1; k < M; ++k) {
                const S c = g.cosjk(j, k, pidx++);
                const V t = c - p.h;
                const V t2 = t * t;
                const V q = (cc[j] * g.fc[k] + cc[k] * g.fc[j]) * t;
                Vx[j] = Vx[j] + q * g.ux[k]; Vy[j] = Vy[j] + q * g.uy[k]; Vz[j] = Vz[j] + q * g.uz[k];
                Vx[k] = Vx[k] + q * g.ux[j]; Vy[k] = Vy[k] + q * g.uy[j]; Vz[k] = Vz[k] + q * g.uz[j];
                const V qc = q * c;
                A[j] = A[j] - qc;
                A[k] = A[k] - qc;
                Pp[j] = Pp[j] + cc[k] * t2;
                Pp[k] = Pp[k] + cc[j] * t2;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const V rad = D[j] + (S(0.5) * g.fcp[j]) * Pp[j] + A[j] * g.rinv[j];
        Gx[j] = rad * g.ux[j] + Vx[j] * g.rinv[j];
        Gy[j] = rad * g.uy[j] + Vy[j] * g.rinv[j];
        Gz[j] = rad * g.uz[j] + Vz[j] * g.rinv[j];
    }
}

// Segmented transpose-reduction of 8 doubles over aligned groups of g lanes
// (g a power of two, 8 <= g <= 64).  Afterwards every lane holds the group sum
// of value index *vidx; lanes with (lane & (g/8 - 1)) == 0 are the writers.
__device__ __forceinline__ double group_reduce8(double* v, int g, int* vidx) {
    const int lane = threadIdx.x & 63;
    int base = 0;
    int m = g >> 1;
    {   // 8 -> 4
        const int h = (lane & m) ? 1 : 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double send = h ? v[k] : v[k + 4];
            const double keep = h ? v[k + 4] : v[k];
            v[k] = keep + __shfl_xor(send, m, 64);
        }
        base += 4 * h;
        m >>= 1;
    }
    {   // 4 -> 2
        const int h = (lane & m) ? 1 : 0;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const double send = h ? v[k] : v[k + 2];
            const double keep = h ? v[k + 2] : v[k];
            v[k] = keep + __shfl_xor(send, m, 64);
        }
        base += 2 * h;
        m >>= 1;
    }
    {   // 2 -> 1
        const int h = (lane & m) ? 1 : 0;
        const double send = h ? v[0] : v[1];
        const double keep = h ? v[1] : v[0];
        v[0] = keep + __shfl_xor(send, m, 64);
        base += h;
        m >>= 1;
    }
    for (; m > 0; m >>= 1) v[0] += __shfl_xor(v[0], m, 64);
    *vidx = base;
    return v[0];
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
