// Structure-set construction: cell-list neighbour search, per-structure
// ordering of atoms by coordination, candidate-independent bond geometry, and
// reference data.
//
// Neighbour search.  The cutoff f_C of the potential (Sec. II.A) vanishes for
// r >= R2, so an atom interacts with every periodic image of every atom closer
// than R2.  Each structure's cell (rows a, b, c) is divided along each axis k
// into nb_k = max(1, floor(w_k / R2)) bins, w_k being the perpendicular width of
// the cell; atoms are binned by their wrapped fractional coordinates.  A point
// within R2 of an atom lies at most m_k = ceil(R2 nb_k / w_k) bins away along
// axis k, and each stencil offset d in [-m_k, m_k] names a distinct (bin,
// image) pair: bin (b + d) mod nb_k, image floor((b + d) / nb_k).  This finds
// all images without duplicates, also when nb_k = 1 and several images of an
// atom (or of the atom itself) are neighbours, which happens in cells narrower
// than 2 R2 and in sheared cells.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "mt_host.h"

namespace mt {

namespace {

constexpr int kMaxBinsAxis = 1024;

struct StructMeta {          // per structure, computed on the device
    double h[9];             // cell rows
    double hinv[9];          // inverse of h (row-vector convention: s = r * hinv)
    int nbin[3];
    int mst[3];              // stencil half width per axis
    int bin_base;            // first global bin (filled after the host prefix)
    int ok;                  // 0: singular cell
};

__global__ void k_struct_meta(int S, const double* __restrict__ cell, double R2,
                              StructMeta* __restrict__ meta) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const double* h = cell + 9 * s;
    StructMeta m;
    for (int k = 0; k < 9; ++k) m.h[k] = h[k];
    // inverse by cofactors
    double a = h[0], b = h[1], c = h[2], d = h[3], e = h[4], f = h[5], g = h[6], hh = h[7], i = h[8];
    double A = e * i - f * hh, B = -(d * i - f * g), C = d * hh - e * g;
    double det = a * A + b * B + c * C;
    m.ok = (det != 0.0 && isfinite(det)) ? 1 : 0;
    double inv = 1.0 / det;
    m.hinv[0] = A * inv;               m.hinv[1] = -(b * i - c * hh) * inv; m.hinv[2] = (b * f - c * e) * inv;
    m.hinv[3] = B * inv;               m.hinv[4] = (a * i - c * g) * inv;    m.hinv[5] = -(a * f - c * d) * inv;
    m.hinv[6] = C * inv;               m.hinv[7] = -(a * hh - b * g) * inv;  m.hinv[8] = (a * e - b * d) * inv;
    // perpendicular widths w_k = |det| / |a_l x a_m|
    double vol = fabs(det);
    for (int k = 0; k < 3; ++k) {
        const double* u = h + 3 * ((k + 1) % 3);
        const double* v = h + 3 * ((k + 2) % 3);
        double cx = u[1] * v[2] - u[2] * v[1];
        double cy = u[2] * v[0] - u[0] * v[2];
        double cz = u[0] * v[1] - u[1] * v[0];
        double w = vol / sqrt(cx * cx + cy * cy + cz * cz);
        int nb = (int)floor(w / R2);
        nb = nb < 1 ? 1 : (nb > kMaxBinsAxis ? kMaxBinsAxis : nb);
        m.nbin[k] = nb;
        m.mst[k] = (int)ceil(R2 * nb / w);
        if (!(w > 0.0) || !isfinite(w)) m.ok = 0;
    }
    m.bin_base = 0;
    meta[s] = m;
}

__device__ __forceinline__ int struct_of(const int* __restrict__ st_off, int S, int atom) {
    int lo = 0, hi = S - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (st_off[mid] <= atom) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int floordiv(int a, int b) {
    int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

// Wrapped fractional coordinates -> bin; count atoms per bin.
__global__ void k_bin_atoms(int N, int S, const int* __restrict__ st_off,
                            const double* __restrict__ pos, const StructMeta* __restrict__ meta,
                            int* __restrict__ atom_bin, int* __restrict__ atom_wrap,
                            int* __restrict__ bin_count) {
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= N) return;
    int s = struct_of(st_off, S, a);
    const StructMeta& m = meta[s];
    double r[3] = {pos[a], pos[N + a], pos[2 * N + a]};
    int bin[3];
    for (int k = 0; k < 3; ++k) {
        double f = r[0] * m.hinv[0 * 3 + k] + r[1] * m.hinv[1 * 3 + k] + r[2] * m.hinv[2 * 3 + k];
        double w = floor(f);
        double fw = f - w;
        int b = (int)floor(fw * m.nbin[k]);
        b = b < 0 ? 0 : (b >= m.nbin[k] ? m.nbin[k] - 1 : b);
        bin[k] = b;
        atom_wrap[3 * a + k] = (int)w;
    }
    int g = m.bin_base + (bin[0] * m.nbin[1] + bin[1]) * m.nbin[2] + bin[2];
    atom_bin[a] = g;
    atomicAdd(&bin_count[g], 1);
}

// Single-block exclusive scan over n ints (in place), chunks of blockDim.
__device__ int block_exclusive_scan(int v, int* sh, int* total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    if (wid == 0) {
        int w = lane < nw ? sh[lane] : 0;
        for (int o = 1; o < 64; o <<= 1) {
            int y = __shfl_up(w, o);
            if (lane >= o) w += y;
        }
        if (lane < nw) sh[lane] = w;
    }
    __syncthreads();
    int prefix = wid ? sh[wid - 1] : 0;
    *total = sh[nw - 1];
    __syncthreads();
    return prefix + x - v;
}

__global__ void k_scan(int n, const int* __restrict__ in, int* __restrict__ out) {
    __shared__ int sh[16];
    int carry = 0;
    for (int base = 0; base < n; base += blockDim.x) {
        int i = base + threadIdx.x;
        int v = i < n ? in[i] : 0;
        int tot;
        int ex = block_exclusive_scan(v, sh, &tot);
        if (i < n) out[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) out[n] = carry;
}

__global__ void k_scatter_bins(int N, const int* __restrict__ atom_bin, const int* __restrict__ bin_start,
                               int* __restrict__ bin_fill, int* __restrict__ bin_atoms) {
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= N) return;
    int g = atom_bin[a];
    int r = atomicAdd(&bin_fill[g], 1);
    bin_atoms[bin_start[g] + r] = a;
}

__device__ __forceinline__ int pack_shift(int n1, int n2, int n3) {
    return ((n1 + 512) << 20) | ((n2 + 512) << 10) | (n3 + 512);
}
__device__ __forceinline__ void unpack_shift(int p, int& n1, int& n2, int& n3) {
    n1 = ((p >> 20) & 1023) - 512;
    n2 = ((p >> 10) & 1023) - 512;
    n3 = (p & 1023) - 512;
}

// Neighbour search over the stencil; entries of each atom sorted by (j, image).
// flags[0] |= 1 on capacity overflow, flags[0] |= 2 on coincident atoms,
// flags[0] |= 4 on a singular cell or an image shift out of range.
__global__ void k_search(int N, int S, int kcap, double R2, const int* __restrict__ st_off,
                         const double* __restrict__ pos, const StructMeta* __restrict__ meta,
                         const int* __restrict__ atom_bin, const int* __restrict__ atom_wrap,
                         const int* __restrict__ bin_start, const int* __restrict__ bin_atoms,
                         int* __restrict__ cnt, int* __restrict__ ent_j, int* __restrict__ ent_sh,
                         int* __restrict__ flags) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int s = struct_of(st_off, S, i);
    const StructMeta& m = meta[s];
    if (!m.ok) { atomicOr(flags, 4); cnt[i] = 0; return; }
    const double ri[3] = {pos[i], pos[N + i], pos[2 * N + i]};
    const int wi[3] = {atom_wrap[3 * i], atom_wrap[3 * i + 1], atom_wrap[3 * i + 2]};
    int local = atom_bin[i] - m.bin_base;
    int bz = local % m.nbin[2];
    int by = (local / m.nbin[2]) % m.nbin[1];
    int bx = local / (m.nbin[2] * m.nbin[1]);
    const int b[3] = {bx, by, bz};
    unsigned long long key[kMaxNbr];
    int count = 0;
    const double R2sq = R2 * R2;
    for (int dx = -m.mst[0]; dx <= m.mst[0]; ++dx)
    for (int dy = -m.mst[1]; dy <= m.mst[1]; ++dy)
    for (int dz = -m.mst[2]; dz <= m.mst[2]; ++dz) {
        const int d[3] = {dx, dy, dz};
        int tb[3], img[3];
        for (int k = 0; k < 3; ++k) {
            int v = b[k] + d[k];
            img[k] = floordiv(v, m.nbin[k]);
            tb[k] = v - img[k] * m.nbin[k];
        }
        int g = m.bin_base + (tb[0] * m.nbin[1] + tb[1]) * m.nbin[2] + tb[2];
        for (int p = bin_start[g]; p < bin_start[g + 1]; ++p) {
            int j = bin_atoms[p];
            int sh[3];
            for (int k = 0; k < 3; ++k) sh[k] = img[k] + wi[k] - atom_wrap[3 * j + k];
            if (j == i && sh[0] == 0 && sh[1] == 0 && sh[2] == 0) continue;
            double dv[3];
            for (int k = 0; k < 3; ++k)
                dv[k] = pos[k * N + j] - ri[k] + sh[0] * m.h[k] + sh[1] * m.h[3 + k] + sh[2] * m.h[6 + k];
            double r2 = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
            if (r2 >= R2sq) continue;
            if (r2 == 0.0) { atomicOr(flags, 2); continue; }
            if (sh[0] < -500 || sh[0] > 500 || sh[1] < -500 || sh[1] > 500 || sh[2] < -500 || sh[2] > 500) {
                atomicOr(flags, 4);
                continue;
            }
            if (count < kcap) {
                unsigned long long kk = ((unsigned long long)(unsigned)j << 32) |
                                        (unsigned)pack_shift(sh[0], sh[1], sh[2]);
                // insertion into the sorted key list
                int q = count;
                while (q > 0 && key[q - 1] > kk) { key[q] = key[q - 1]; --q; }
                key[q] = kk;
            }
            ++count;
        }
    }
    if (count > kcap) atomicOr(flags, 1);
    int n = count < kcap ? count : kcap;
    cnt[i] = n;
    for (int q = 0; q < n; ++q) {
        ent_j[q * N + i] = (int)(key[q] >> 32);
        ent_sh[q * N + i] = (int)(key[q] & 0xffffffffu);
    }
}

// Stable sort of each structure's atoms by descending coordination; one block
// per structure.  perm[sorted] = original, inv[original] = sorted.
__global__ void k_sort_by_coordination(const int* __restrict__ st_off, int kcap,
                                       const int* __restrict__ cnt, int* __restrict__ perm,
                                       int* __restrict__ inv) {
    __shared__ int sh[16];
    const int s = blockIdx.x;
    const int a0 = st_off[s], a1 = st_off[s + 1];
    int base = 0;
    for (int m = kcap; m >= 0; --m) {
        for (int c = a0; c < a1; c += blockDim.x) {
            int a = c + threadIdx.x;
            int flag = (a < a1 && cnt[a] == m) ? 1 : 0;
            int tot;
            int ex = block_exclusive_scan(flag, sh, &tot);
            if (flag) {
                perm[a0 + base + ex] = a;
                inv[a] = a0 + base + ex;
            }
            base += tot;
        }
    }
}

// Per structure (one block each): coordination in sorted order, local bond
// offsets, bonds, largest coordination and ordered triplets.
__global__ void k_struct_tables(const int* __restrict__ st_off, const int* __restrict__ perm,
                                const int* __restrict__ cnt, const int* __restrict__ st_npad,
                                int* __restrict__ nnb, int* __restrict__ lbo,
                                int* __restrict__ st_nbonds, int* __restrict__ st_kmax,
                                long long* __restrict__ st_trip, int* __restrict__ xbase,
                                int* __restrict__ st_xsize) {
    __shared__ int sh[16];
    __shared__ int kmax_sh;
    __shared__ unsigned long long trip_sh;
    const int s = blockIdx.x;
    const int a0 = st_off[s], a1 = st_off[s + 1];
    if (threadIdx.x == 0) { kmax_sh = 0; trip_sh = 0; }
    __syncthreads();
    int base = 0;
    for (int c = a0; c < a1; c += blockDim.x) {
        int a = c + threadIdx.x;
        int m = a < a1 ? cnt[perm[a]] : 0;
        int tot;
        int ex = block_exclusive_scan(m, sh, &tot);
        if (a < a1) {
            nnb[a] = m;
            lbo[a] = base + ex;
            atomicMax(&kmax_sh, m);
            atomicAdd(&trip_sh, (unsigned long long)(m * (m - 1 > 0 ? m - 1 : 0)));
        }
        base += tot;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        st_nbonds[s] = base;
        st_kmax[s] = kmax_sh;
        st_trip[s] = (long long)trip_sh;
    }
    // Exchange slots of the batched kernels (structures up to kMaxBatched atoms):
    // chunks of G lanes, chunk c holds K_c * G slots.
    __shared__ int choff[kMaxBatched / 8 + 1];
    const int npad = st_npad[s];
    const int ns = a1 - a0;
    if (npad > 0) {
        const int G = npad < 64 ? npad : 64;
        const int nch = npad / G;
        const int lo = kmax_sh <= 4 ? 0 : 3;     // lowest variant of the structure's class
        if (threadIdx.x == 0) {
            int off = 0;
            for (int c = 0; c < nch; ++c) {
                int K = lo;
                for (int l = c * G; l < (c + 1) * G && l < ns; ++l) K = max(K, nnb[a0 + l]);
                choff[c] = off;
                off += K * G;
            }
            choff[nch] = off;
            st_xsize[s] = off;
        }
        __syncthreads();
        for (int l = threadIdx.x; l < ns; l += blockDim.x) xbase[a0 + l] = choff[l / G] + (l % G);
    } else {
        for (int l = threadIdx.x; l < ns; l += blockDim.x) xbase[a0 + l] = 0;
        if (threadIdx.x == 0) st_xsize[s] = 0;
    }
}

// cos(theta_jk) of every pair of the first six bond slots of a sorted atom, the
// float64 unit vectors' product rounded once to float (pair k (k - 1) / 2 + j;
// zero where a slot is past the capacity, and padding slots have zero unit
// vectors).  The float kernels read their cached angle cosines from here.
__global__ void k_pair_cos(int N, int kcap, const double* __restrict__ gd, float* __restrict__ gcs) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= N) return;
    const size_t KN = (size_t)kcap * N;
    double vx[6], vy[6], vz[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        const bool ok = m < kcap;
        vx[m] = ok ? gd[(size_t)m * N + a] : 0.0;
        vy[m] = ok ? gd[KN + (size_t)m * N + a] : 0.0;
        vz[m] = ok ? gd[2 * KN + (size_t)m * N + a] : 0.0;
    }
#pragma unroll
    for (int k = 1; k < 6; ++k)
#pragma unroll
        for (int j = 0; j < k; ++j)
            gcs[(size_t)(k * (k - 1) / 2 + j) * N + a] = (float)(vx[j] * vx[k] + vy[j] * vy[k] + vz[j] * vz[k]);
}

// Bond geometry for every (sorted atom, slot).  Padded slots (m >= coordination)
// get f_C = f_C' = 0 and a zero unit vector, so they add nothing anywhere.
__global__ void k_geometry(int N, int S, int kcap, double R1, double R2,
                           const int* __restrict__ st_off, const double* __restrict__ pos,
                           const StructMeta* __restrict__ meta, const int* __restrict__ perm,
                           const int* __restrict__ inv, const int* __restrict__ cnt,
                           const int* __restrict__ ent_j, const int* __restrict__ ent_sh,
                           const int* __restrict__ lbo, const int* __restrict__ xbase,
                           const int* __restrict__ st_npad,
                           float* __restrict__ gf, float* __restrict__ gf_rlo, float4* __restrict__ gpk,
                           double* __restrict__ gd,
                           int* __restrict__ rev, int* __restrict__ revc, int* __restrict__ jl,
                           int* __restrict__ nbr_j, int* __restrict__ nbr_sh, int* __restrict__ flags) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * kcap) return;
    const int a = idx % N;          // sorted atom
    const int m = idx / N;          // slot
    const size_t KN = (size_t)kcap * N;
    const int i = perm[a];
    const int M = cnt[i];
    const int o = m * N + a;
    float* f_ux = gf;         float* f_uy = gf + KN;    float* f_uz = gf + 2 * KN;
    float* f_rhi = gf + 3 * KN; float* f_rinv = gf + 4 * KN;
    float* f_fc = gf + 5 * KN;  float* f_hfcp = gf + 6 * KN;
    double* d_ux = gd;        double* d_uy = gd + KN;   double* d_uz = gd + 2 * KN;
    double* d_r = gd + 3 * KN;  double* d_rinv = gd + 4 * KN;
    double* d_fc = gd + 5 * KN; double* d_hfcp = gd + 6 * KN;
    const int s = struct_of(st_off, S, a);
    const int npad = st_npad[s];
    const int G = npad < 64 ? npad : 64;
    if (m >= M) {
        f_ux[o] = f_uy[o] = f_uz[o] = 0.f; f_rhi[o] = 3.0f; gf_rlo[o] = 0.f;
        f_rinv[o] = 0.f; f_fc[o] = 0.f; f_hfcp[o] = 0.f;
        d_ux[o] = d_uy[o] = d_uz[o] = 0.0; d_r[o] = 3.0; d_rinv[o] = 0.0;
        d_fc[o] = 0.0; d_hfcp[o] = 0.0;
        // a padded bond reads back its own (zero) slot and its own atom
        gpk[o] = make_float4(0.f, 0.f, 0.f, 3.0f);
        gpk[KN + o] = make_float4(0.f, 0.f, 0.f, 0.f);
        rev[o] = npad > 0 ? xbase[a] + m * G : 0;
        revc[o] = 0;
        jl[o] = a - st_off[s];
        nbr_j[o] = -1; nbr_sh[o] = 0;
        return;
    }
    const StructMeta& me = meta[s];
    const int j = ent_j[m * N + i];
    const int shp = ent_sh[m * N + i];
    int n1, n2, n3;
    unpack_shift(shp, n1, n2, n3);
    double dv[3];
    for (int k = 0; k < 3; ++k)
        dv[k] = pos[k * N + j] - pos[k * N + i] + n1 * me.h[k] + n2 * me.h[3 + k] + n3 * me.h[6 + k];
    const double r = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    const double rinv = 1.0 / r;
    double fc, hfcp;                 // f_C and f_C'/2 (the kernels only use half the slope)
    if (r <= R1) { fc = 1.0; hfcp = 0.0; }
    else if (r >= R2) { fc = 0.0; hfcp = 0.0; }
    else {
        const double w = M_PI / (R2 - R1);
        const double ph = w * (r - R1);
        fc = 0.5 * (1.0 + cos(ph));
        hfcp = -0.25 * w * sin(ph);
    }
    const double ux = dv[0] * rinv, uy = dv[1] * rinv, uz = dv[2] * rinv;
    d_ux[o] = ux; d_uy[o] = uy; d_uz[o] = uz; d_r[o] = r; d_rinv[o] = rinv;
    d_fc[o] = fc; d_hfcp[o] = hfcp;
    const float rhi = (float)r;
    f_ux[o] = (float)ux; f_uy[o] = (float)uy; f_uz[o] = (float)uz;
    f_rhi[o] = rhi; gf_rlo[o] = (float)(r - (double)rhi);
    f_rinv[o] = (float)rinv; f_fc[o] = (float)fc; f_hfcp[o] = (float)hfcp;
    gpk[o] = make_float4((float)ux, (float)uy, (float)uz, rhi);
    gpk[KN + o] = make_float4((float)(r - (double)rhi), (float)rinv, (float)fc, (float)hfcp);
    // reverse entry: (j -> i, -shift) in j's sorted list
    const int want = pack_shift(-n1, -n2, -n3);
    const int Mj = cnt[j];
    int mr = -1;
    for (int q = 0; q < Mj; ++q)
        if (ent_j[q * N + j] == i && ent_sh[q * N + j] == want) { mr = q; break; }
    if (mr < 0) atomicOr(flags, 8);
    const int js = inv[j];
    if (mr < 0) mr = 0;
    rev[o] = npad > 0 ? xbase[js] + mr * G : 0;
    revc[o] = lbo[js] + mr;
    jl[o] = js - st_off[s];
    nbr_j[o] = j;
    nbr_sh[o] = shp;
}

__global__ void k_export(int N, int kcap, const int* __restrict__ perm, const int* __restrict__ nnb,
                         const int* __restrict__ lbo, const int* __restrict__ st_off, int S,
                         const int* __restrict__ st_boff,
                         const int* __restrict__ nbr_j, const int* __restrict__ nbr_sh,
                         int nb, int32_t* __restrict__ oi, int32_t* __restrict__ oj,
                         int32_t* __restrict__ osh) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * kcap) return;
    const int a = idx % N, m = idx / N;
    if (m >= nnb[a]) return;
    const int s = struct_of(st_off, S, a);
    const int e = st_boff[s] + lbo[a] + m;
    int n1, n2, n3;
    unpack_shift(nbr_sh[m * N + a], n1, n2, n3);
    oi[e] = perm[a];
    oj[e] = nbr_j[m * N + a];
    osh[e] = n1; osh[nb + e] = n2; osh[2 * nb + e] = n3;
}

__global__ void k_permute_forces(int N, const int* __restrict__ perm, const double* __restrict__ f,
                                 double* __restrict__ f64, float* __restrict__ f32) {
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= N) return;
    const int i = perm[a];
    for (int k = 0; k < 3; ++k) {
        double v = f[(size_t)k * N + i];
        f64[(size_t)k * N + a] = v;
        f32[(size_t)k * N + a] = (float)v;
    }
}

// Q_e, Q_v, Q_f: sums of squares of the reference data in a fixed order
// (one block; each thread strides, then a fixed tree).
__global__ void k_ref_norms(int S, int N, const double* __restrict__ e, const double* __restrict__ w,
                            const double* __restrict__ f, double* __restrict__ out) {
    __shared__ double sh[3][256];
    double q[3] = {0, 0, 0};
    for (int s = threadIdx.x; s < S; s += blockDim.x) {
        q[0] += e[s] * e[s];
        for (int c = 0; c < 6; ++c) q[1] += w[6 * s + c] * w[6 * s + c];
    }
    for (size_t k = threadIdx.x; k < (size_t)3 * N; k += blockDim.x) q[2] += f[k] * f[k];
    for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] = q[c];
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) out[c] = sh[c][0];
}

int grid_of(long long n, int block) { return (int)((n + block - 1) / block); }

}  // namespace

#define HIPCHECK(call)                                   \
    do {                                                 \
        hipError_t _e = (call);                          \
        if (_e != hipSuccess) return hip_fail(_e, #call); \
    } while (0)

int build_set(mt_set* set, const int64_t* atom_offset, const double* pos, const double* cell,
              hipStream_t st) {
    const int S = set->S, N = set->N, kcap = set->kcap;
    int dev = 0, lds_max = 0;
    HIPCHECK(hipGetDevice(&dev));
    HIPCHECK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    set->lds_max = (size_t)lds_max;
    set->h_off.assign(S + 1, 0);
    for (int s = 0; s <= S; ++s) set->h_off[s] = (int)atom_offset[s];

    HIPCHECK(set->pos.reserve(sizeof(double) * 3 * N));
    HIPCHECK(set->cell.reserve(sizeof(double) * 9 * S));
    // a rebuild passes the set's own cell (mt_set_update_positions)
    if (pos != set->pos.p)
        HIPCHECK(hipMemcpyAsync(set->pos.p, pos, sizeof(double) * 3 * N, hipMemcpyDeviceToDevice, st));
    if (cell != set->cell.p)
        HIPCHECK(hipMemcpyAsync(set->cell.p, cell, sizeof(double) * 9 * S, hipMemcpyDeviceToDevice, st));
    HIPCHECK(set->st_off.reserve(sizeof(int) * (S + 1)));
    HIPCHECK(hipMemcpyAsync(set->st_off.p, set->h_off.data(), sizeof(int) * (S + 1),
                            hipMemcpyHostToDevice, st));

    BuildScratch& B = set->build;
    DevBuf &meta = B.meta, &atom_bin = B.atom_bin, &atom_wrap = B.atom_wrap, &bin_count = B.bin_count,
           &bin_start = B.bin_start, &bin_fill = B.bin_fill, &bin_atoms = B.bin_atoms, &cnt = B.cnt,
           &ent_j = B.ent_j, &ent_sh = B.ent_sh, &inv = B.inv, &flags = B.flags, &st_nb = B.st_nb,
           &st_trip = B.st_trip;
    HIPCHECK(meta.reserve(sizeof(StructMeta) * S));
    const double rlist = set->R2 + set->skin;
    k_struct_meta<<<grid_of(S, 128), 128, 0, st>>>(S, set->cell.as<double>(), rlist,
                                                    meta.as<StructMeta>());
    HIPCHECK(hipGetLastError());
    std::vector<StructMeta> hm(S);
    HIPCHECK(hipMemcpyAsync(hm.data(), meta.p, sizeof(StructMeta) * S, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    long long nbins = 0;
    for (int s = 0; s < S; ++s) {
        if (!hm[s].ok) {
            set_error("structure " + std::to_string(s) + " has a singular or non-finite cell");
            return MT_EINVAL;
        }
        hm[s].bin_base = (int)nbins;
        nbins += (long long)hm[s].nbin[0] * hm[s].nbin[1] * hm[s].nbin[2];
    }
    if (nbins > (1ll << 28)) {
        set_error("cell list too large");
        return MT_EINVAL;
    }
    HIPCHECK(hipMemcpyAsync(meta.p, hm.data(), sizeof(StructMeta) * S, hipMemcpyHostToDevice, st));

    HIPCHECK(atom_bin.reserve(sizeof(int) * N));
    HIPCHECK(atom_wrap.reserve(sizeof(int) * 3 * N));
    HIPCHECK(bin_count.reserve(sizeof(int) * (nbins + 1)));
    HIPCHECK(bin_start.reserve(sizeof(int) * (nbins + 1)));
    HIPCHECK(bin_fill.reserve(sizeof(int) * (nbins + 1)));
    HIPCHECK(bin_atoms.reserve(sizeof(int) * N));
    HIPCHECK(hipMemsetAsync(bin_count.p, 0, sizeof(int) * (nbins + 1), st));
    HIPCHECK(hipMemsetAsync(bin_fill.p, 0, sizeof(int) * (nbins + 1), st));
    k_bin_atoms<<<grid_of(N, 256), 256, 0, st>>>(N, S, set->st_off.as<int>(), set->pos.as<double>(),
                                                  meta.as<StructMeta>(), atom_bin.as<int>(),
                                                  atom_wrap.as<int>(), bin_count.as<int>());
    HIPCHECK(hipGetLastError());
    k_scan<<<1, 1024, 0, st>>>((int)nbins, bin_count.as<int>(), bin_start.as<int>());
    HIPCHECK(hipGetLastError());
    k_scatter_bins<<<grid_of(N, 256), 256, 0, st>>>(N, atom_bin.as<int>(), bin_start.as<int>(),
                                                     bin_fill.as<int>(), bin_atoms.as<int>());
    HIPCHECK(hipGetLastError());

    HIPCHECK(cnt.reserve(sizeof(int) * N));
    HIPCHECK(ent_j.reserve(sizeof(int) * (size_t)kcap * N));
    HIPCHECK(ent_sh.reserve(sizeof(int) * (size_t)kcap * N));
    HIPCHECK(flags.reserve(sizeof(int) * 4));
    HIPCHECK(hipMemsetAsync(flags.p, 0, sizeof(int) * 4, st));
    k_search<<<grid_of(N, 128), 128, 0, st>>>(N, S, kcap, rlist, set->st_off.as<int>(),
                                               set->pos.as<double>(), meta.as<StructMeta>(),
                                               atom_bin.as<int>(), atom_wrap.as<int>(),
                                               bin_start.as<int>(), bin_atoms.as<int>(), cnt.as<int>(),
                                               ent_j.as<int>(), ent_sh.as<int>(), flags.as<int>());
    HIPCHECK(hipGetLastError());
    int hflags = 0;
    HIPCHECK(hipMemcpyAsync(&hflags, flags.p, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    if (hflags & 2) { set_error("coincident atoms (distance 0 between an atom and a neighbour image)"); return MT_ECOINCIDENT; }
    if (hflags & 4) { set_error("invalid cell or image shift out of range"); return MT_EINVAL; }
    if (hflags & 1) {
        set_error("an atom has more than max_nbr = " + std::to_string(kcap) +
                  " neighbours within R2 + skin");
        return MT_ENBR_OVERFLOW;
    }

    // padded sizes depend on atom counts only
    set->h_npad.assign(S, 0);
    set->h_large.assign(S, 0);
    for (int s = 0; s < S; ++s) {
        const int ns = set->h_off[s + 1] - set->h_off[s];
        int npad;
        if (ns <= 8) npad = 8;
        else if (ns <= 16) npad = 16;
        else if (ns <= 32) npad = 32;
        else npad = ((ns + 63) / 64) * 64;
        const bool large = ns > kMaxBatched;
        set->h_large[s] = large ? 1 : 0;
        set->h_npad[s] = large ? 0 : npad;
    }
    HIPCHECK(set->st_npad.reserve(sizeof(int) * S));
    HIPCHECK(hipMemcpyAsync(set->st_npad.p, set->h_npad.data(), sizeof(int) * S, hipMemcpyHostToDevice, st));

    HIPCHECK(set->perm.reserve(sizeof(int) * N));
    HIPCHECK(inv.reserve(sizeof(int) * N));
    k_sort_by_coordination<<<S, 256, 0, st>>>(set->st_off.as<int>(), kcap, cnt.as<int>(),
                                               set->perm.as<int>(), inv.as<int>());
    HIPCHECK(hipGetLastError());
    HIPCHECK(set->nnb.reserve(sizeof(int) * N));
    HIPCHECK(set->lbo.reserve(sizeof(int) * N));
    HIPCHECK(st_nb.reserve(sizeof(int) * S));
    HIPCHECK(set->st_kmax.reserve(sizeof(int) * S));
    HIPCHECK(st_trip.reserve(sizeof(long long) * S));
    HIPCHECK(set->xbase.reserve(sizeof(int) * N));
    HIPCHECK(set->st_xsize.reserve(sizeof(int) * S));
    k_struct_tables<<<S, 256, 0, st>>>(set->st_off.as<int>(), set->perm.as<int>(), cnt.as<int>(),
                                        set->st_npad.as<int>(), set->nnb.as<int>(), set->lbo.as<int>(),
                                        st_nb.as<int>(), set->st_kmax.as<int>(), st_trip.as<long long>(),
                                        set->xbase.as<int>(), set->st_xsize.as<int>());
    HIPCHECK(hipGetLastError());
    std::vector<int> hnb(S);
    set->h_kmax.assign(S, 0);
    set->h_trip.assign(S, 0);
    HIPCHECK(hipMemcpyAsync(hnb.data(), st_nb.p, sizeof(int) * S, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipMemcpyAsync(set->h_kmax.data(), set->st_kmax.p, sizeof(int) * S, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipMemcpyAsync(set->h_trip.data(), st_trip.p, sizeof(long long) * S, hipMemcpyDeviceToHost, st));
    set->h_xsize.assign(S, 0);
    HIPCHECK(hipMemcpyAsync(set->h_xsize.data(), set->st_xsize.p, sizeof(int) * S, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));

    // per-structure launch tables
    set->h_boff.assign(S + 1, 0);
    set->h_slot.assign(S + 1, 0);
    set->kmax = 0;
    set->ntrip = 0;
    set->max_atoms = 0;
    set->n_batched = set->n_large = 0;
    for (int s = 0; s < S; ++s) {
        const int ns = set->h_off[s + 1] - set->h_off[s];
        set->h_boff[s + 1] = set->h_boff[s] + hnb[s];
        set->kmax = std::max(set->kmax, set->h_kmax[s]);
        set->ntrip += set->h_trip[s];
        set->max_atoms = std::max(set->max_atoms, ns);
        const bool large = set->h_large[s] != 0;
        const int npad = set->h_npad[s];
        // over the batching limit: one slot per block of the two-pass kernels
        const int nsl = large ? (ns + kLargeBlock - 1) / kLargeBlock : std::max(1, npad / 64);
        set->h_slot[s + 1] = set->h_slot[s] + nsl;
        if (large) ++set->n_large; else ++set->n_batched;
    }
    set->nb = set->h_boff[S];
    set->nslots = set->h_slot[S];
    HIPCHECK(set->st_boff.reserve(sizeof(int) * (S + 1)));
    HIPCHECK(set->st_slot.reserve(sizeof(int) * (S + 1)));
    HIPCHECK(hipMemcpyAsync(set->st_boff.p, set->h_boff.data(), sizeof(int) * (S + 1), hipMemcpyHostToDevice, st));
    HIPCHECK(hipMemcpyAsync(set->st_slot.p, set->h_slot.data(), sizeof(int) * (S + 1), hipMemcpyHostToDevice, st));

    const size_t KN = (size_t)kcap * N;
    HIPCHECK(set->gf.reserve(sizeof(float) * 7 * KN));
    HIPCHECK(set->gf_rlo.reserve(sizeof(float) * KN));
    HIPCHECK(set->gpk.reserve(sizeof(float4) * 2 * KN));
    HIPCHECK(set->gd.reserve(sizeof(double) * 7 * KN));
    HIPCHECK(set->gcs.reserve(sizeof(float) * kCosPairs * (size_t)N));
    HIPCHECK(set->rev.reserve(sizeof(int) * KN));
    HIPCHECK(set->revc.reserve(sizeof(int) * KN));
    HIPCHECK(set->jl.reserve(sizeof(int) * KN));
    HIPCHECK(set->nbr_j.reserve(sizeof(int) * KN));
    HIPCHECK(set->nbr_sh.reserve(sizeof(int) * KN));
    HIPCHECK(hipMemsetAsync(flags.p, 0, sizeof(int) * 4, st));
    k_geometry<<<grid_of((long long)KN, 256), 256, 0, st>>>(
        N, S, kcap, set->R1, set->R2, set->st_off.as<int>(), set->pos.as<double>(),
        meta.as<StructMeta>(), set->perm.as<int>(), inv.as<int>(), cnt.as<int>(), ent_j.as<int>(),
        ent_sh.as<int>(), set->lbo.as<int>(), set->xbase.as<int>(), set->st_npad.as<int>(),
        set->gf.as<float>(), set->gf_rlo.as<float>(), set->gpk.as<float4>(),
        set->gd.as<double>(), set->rev.as<int>(), set->revc.as<int>(), set->jl.as<int>(), set->nbr_j.as<int>(),
        set->nbr_sh.as<int>(), flags.as<int>());
    HIPCHECK(hipGetLastError());
    k_pair_cos<<<grid_of(N, 256), 256, 0, st>>>(N, kcap, set->gd.as<double>(), set->gcs.as<float>());
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(&hflags, flags.p, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    if (hflags & 8) {
        set_error("neighbour lists are not symmetric (reverse entry missing)");
        return MT_EINVAL;
    }
    return MT_OK;
}

int update_geometry(mt_set* set, const double* pos, hipStream_t st) {
    const int S = set->S, N = set->N, kcap = set->kcap;
    BuildScratch& B = set->build;
    const size_t KN = (size_t)kcap * N;
    if (pos != set->pos.p)
        HIPCHECK(hipMemcpyAsync(set->pos.p, pos, sizeof(double) * 3 * N, hipMemcpyDeviceToDevice, st));
    k_geometry<<<grid_of((long long)KN, 256), 256, 0, st>>>(
        N, S, kcap, set->R1, set->R2, set->st_off.as<int>(), set->pos.as<double>(),
        B.meta.as<StructMeta>(), set->perm.as<int>(), B.inv.as<int>(), B.cnt.as<int>(), B.ent_j.as<int>(),
        B.ent_sh.as<int>(), set->lbo.as<int>(), set->xbase.as<int>(), set->st_npad.as<int>(),
        set->gf.as<float>(), set->gf_rlo.as<float>(), set->gpk.as<float4>(),
        set->gd.as<double>(), set->rev.as<int>(), set->revc.as<int>(), set->jl.as<int>(), set->nbr_j.as<int>(),
        set->nbr_sh.as<int>(), B.flags.as<int>());
    HIPCHECK(hipGetLastError());
    k_pair_cos<<<grid_of(N, 256), 256, 0, st>>>(N, kcap, set->gd.as<double>(), set->gcs.as<float>());
    HIPCHECK(hipGetLastError());
    return MT_OK;
}

int attach_reference(mt_set* set, const double* e_ref, const double* w_ref, const double* f_ref,
                     hipStream_t st) {
    const int S = set->S, N = set->N;
    HIPCHECK(set->eref.reserve(sizeof(double) * S));
    HIPCHECK(set->wref.reserve(sizeof(double) * 6 * S));
    HIPCHECK(set->fref64.reserve(sizeof(double) * 3 * N));
    HIPCHECK(set->fref32.reserve(sizeof(float) * 3 * N));
    HIPCHECK(set->scalars.reserve(sizeof(double) * 8));
    HIPCHECK(hipMemcpyAsync(set->eref.p, e_ref, sizeof(double) * S, hipMemcpyDeviceToDevice, st));
    HIPCHECK(hipMemcpyAsync(set->wref.p, w_ref, sizeof(double) * 6 * S, hipMemcpyDeviceToDevice, st));
    k_permute_forces<<<grid_of(N, 256), 256, 0, st>>>(N, set->perm.as<int>(), f_ref,
                                                       set->fref64.as<double>(), set->fref32.as<float>());
    HIPCHECK(hipGetLastError());
    k_ref_norms<<<1, 256, 0, st>>>(S, N, e_ref, w_ref, f_ref, set->scalars.as<double>());
    HIPCHECK(hipGetLastError());
    double q[3];
    HIPCHECK(hipMemcpyAsync(q, set->scalars.p, sizeof(q), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    for (int c = 0; c < 3; ++c) {
        if (!(q[c] > 0.0) || !std::isfinite(q[c])) {
            static const char* nm[3] = {"energy", "virial", "force"};
            set_error(std::string("reference ") + nm[c] +
                      " data have zero (or non-finite) norm; the relative RMSE is undefined");
            set->has_ref = false;
            return MT_EINVAL;
        }
        set->Q[c] = q[c];
    }
    set->has_ref = true;
    return MT_OK;
}

int export_neighbors(const mt_set* set, int32_t* i, int32_t* j, int32_t* shift, hipStream_t st) {
    const size_t KN = (size_t)set->kcap * set->N;
    k_export<<<grid_of((long long)KN, 256), 256, 0, st>>>(
        set->N, set->kcap, set->perm.as<int>(), set->nnb.as<int>(), set->lbo.as<int>(),
        set->st_off.as<int>(), set->S, set->st_boff.as<int>(), set->nbr_j.as<int>(),
        set->nbr_sh.as<int>(), set->nb, i, j, shift);
    HIPCHECK(hipGetLastError());
    return MT_OK;
}

}  // namespace mt
