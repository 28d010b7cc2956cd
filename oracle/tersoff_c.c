/*
 * Plain C float64 reference of the Tersoff site energies, forces, virials and
 * fitness -- TEST INFRASTRUCTURE ONLY (used by the CPU tests and by the
 * benchmark's CPU baseline; the GPU library never links or calls it).
 *
 * It evaluates the paper's definitions directly, one atom at a time:
 *   U = sum_i U_i,  U_i = 1/2 sum_j f_C(r_ij) [f_R(r_ij) - b_ij f_A(r_ij)]   Sec. II.A Eqs. 1-3
 *   f_R = A e^{-lambda r},  f_A = B e^{-mu r}                                Sec. II.A Eqs. 4-5
 *   b_ij = (1 + zeta_ij^n)^{-1/(2n)} (1 when zeta_ij = 0)                     Sec. II.A Eq. 6
 *   zeta_ij = sum_{k != j} f_C(r_ik) g(cos theta_ijk)                         Sec. II.A Eq. 7
 *   g = beta (cos - h)^2 (minimal form, Sec. II.B Eq. 10) or Tersoff's
 *   g = gamma (1 + c^2/d^2 - c^2/(d^2 + (cos - h)^2))                       Sec. II.A Eq. 8
 *   f_C: 1 below R1, (1 + cos(pi (r - R1)/(R2 - R1)))/2 between, 0 above R2   Sec. II.A Eq. 9
 *   A, B, lambda, mu from D0, alpha, r0 and the slope S (2 in the minimal
 *   form)                                                                     Sec. II.B Eqs. 11-14
 * The forces and the virial are the exact derivatives of U, written out by the
 * chain rule (the paper cites their formulas); F_i = -dU/dr_i and
 * W = -dU/d(strain), so that W_mn = -sum over bonds of (dU_i/dd)_m d_n for the
 * bond vectors d = r_j + T - r_i.  The fitness is Sec. III.B:
 * Z = w_e Z_e + w_v Z_v + w_f Z_f with relative RMSEs of the per-atom energies,
 * the per-atom virials (xx yy zz yz zx xy) and the force components.
 *
 * Neighbour entries come from the caller (the oracle's brute-force periodic
 * enumeration): entries of atom i are ent_start[i] .. ent_start[i+1]-1, with
 * partner ent_j[e] and bond vector ent_d[3e..3e+2].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define TC_MAX_NBR 64
#define TC_PI 3.14159265358979323846

typedef struct {
    double A, B, lam, mu;         /* pair terms */
    double n;                     /* bond-order exponent */
    int full;                     /* Tersoff's angular function */
    double beta, h;               /* minimal: g = beta (cos - h)^2 */
    double gam, c2, d2;           /* Tersoff: gamma, c^2, d^2 (and h) */
} Params;

static void params_of(const double* x, int full, Params* p) {
    const double D0 = x[0], alpha = x[1], r0 = x[2];
    const double S = full ? x[3] : 2.0;
    p->A = D0 / (S - 1.0) * exp(alpha * r0 * sqrt(2.0 * S));
    p->B = D0 * S / (S - 1.0) * exp(alpha * r0 * sqrt(2.0 / S));
    p->lam = alpha * sqrt(2.0 * S);
    p->mu = alpha * sqrt(2.0 / S);
    p->full = full;
    if (full) {
        p->gam = x[4]; p->n = x[5]; p->c2 = x[6] * x[6]; p->d2 = x[7] * x[7]; p->h = x[8];
        p->beta = 0.0;
    } else {
        p->beta = x[3]; p->n = x[4]; p->h = x[5];
        p->gam = 0.0; p->c2 = 0.0; p->d2 = 1.0;
    }
}

/* g(cos) and dg/dcos */
static void angular(const Params* p, double cs, double* g, double* dg) {
    const double t = cs - p->h;
    if (p->full) {
        const double q = p->d2 + t * t;
        *g = p->gam * (1.0 + p->c2 / p->d2 - p->c2 / q);
        *dg = p->gam * p->c2 * 2.0 * t / (q * q);
    } else {
        *g = p->beta * t * t;
        *dg = 2.0 * p->beta * t;
    }
}

/* f_C and df_C/dr */
static void cutoff(double r, double R1, double R2, double* fc, double* dfc) {
    if (r <= R1) { *fc = 1.0; *dfc = 0.0; return; }
    if (r >= R2) { *fc = 0.0; *dfc = 0.0; return; }
    const double w = TC_PI / (R2 - R1);
    *fc = 0.5 * (1.0 + cos(w * (r - R1)));
    *dfc = -0.5 * w * sin(w * (r - R1));
}

/*
 * Site energy U_i of atom i and dU_i/dd for each of its bond vectors
 * (G[3m..3m+2] for entry s0 + m).  Returns -1 if the atom has more than
 * TC_MAX_NBR entries.
 */
static int site(const Params* p, double R1, double R2, const double* d, int M, double* U, double* G) {
    if (M > TC_MAX_NBR) return -1;
    double r[TC_MAX_NBR], u[TC_MAX_NBR][3], fc[TC_MAX_NBR], dfc[TC_MAX_NBR];
    double fR[TC_MAX_NBR], fA[TC_MAX_NBR], zeta[TC_MAX_NBR], b[TC_MAX_NBR], coef[TC_MAX_NBR];
    for (int m = 0; m < M; ++m) {
        const double* v = d + 3 * m;
        r[m] = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        for (int a = 0; a < 3; ++a) u[m][a] = v[a] / r[m];
        cutoff(r[m], R1, R2, &fc[m], &dfc[m]);
        fR[m] = p->A * exp(-p->lam * r[m]);
        fA[m] = p->B * exp(-p->mu * r[m]);
    }
    /* bond orders */
    for (int m = 0; m < M; ++m) {
        double z = 0.0;
        for (int k = 0; k < M; ++k) {
            if (k == m) continue;
            const double cs = u[m][0] * u[k][0] + u[m][1] * u[k][1] + u[m][2] * u[k][2];
            double g, dg;
            angular(p, cs, &g, &dg);
            z += fc[k] * g;
        }
        zeta[m] = z;
        if (z > 0.0) {
            const double zn = pow(z, p->n);
            b[m] = pow(1.0 + zn, -1.0 / (2.0 * p->n));
            /* coef = dU_i/dzeta_m = -1/2 f_C f_A db/dzeta, db/dzeta = -b zeta^n / (2 zeta (1 + zeta^n)) */
            coef[m] = 0.5 * fc[m] * fA[m] * b[m] * zn / (2.0 * z * (1.0 + zn));
        } else {
            b[m] = 1.0;
            coef[m] = 0.0;
        }
    }
    double Ui = 0.0;
    for (int m = 0; m < M; ++m) Ui += 0.5 * fc[m] * (fR[m] - b[m] * fA[m]);
    *U = Ui;
    /* bond gradients */
    for (int m = 0; m < M; ++m) {
        /* pair term along u_m */
        const double rad = 0.5 * (dfc[m] * (fR[m] - b[m] * fA[m]) +
                                  fc[m] * (-p->lam * fR[m] + b[m] * p->mu * fA[m]));
        double gv[3] = {rad * u[m][0], rad * u[m][1], rad * u[m][2]};
        for (int k = 0; k < M; ++k) {
            if (k == m) continue;
            const double cs = u[m][0] * u[k][0] + u[m][1] * u[k][1] + u[m][2] * u[k][2];
            double g, dg;
            angular(p, cs, &g, &dg);
            /* zeta_m through cos(theta_mk): d cos/d d_m = (u_k - cos u_m) / r_m */
            /* zeta_k through f_C(r_m) and cos(theta_km) */
            for (int a = 0; a < 3; ++a) {
                const double dcos = (u[k][a] - cs * u[m][a]) / r[m];
                gv[a] += coef[m] * fc[k] * dg * dcos;
                gv[a] += coef[k] * (dfc[m] * g * u[m][a] + fc[m] * dg * dcos);
            }
        }
        G[3 * m + 0] = gv[0];
        G[3 * m + 1] = gv[1];
        G[3 * m + 2] = gv[2];
    }
    return 0;
}

static const int V6[6][2] = {{0, 0}, {1, 1}, {2, 2}, {1, 2}, {2, 0}, {0, 1}};

/*
 * Energies E [S], forces F [N][3] and virials W [S][6] of one parameter set x
 * (6 values, or 9 for the Tersoff form).  Returns 0, or -1 for an atom with
 * more than TC_MAX_NBR neighbour entries.
 */
int tc_evaluate(int N, int S, const int64_t* ent_start, const int64_t* ent_j, const double* ent_d,
                const int64_t* atom_struct, const double* x, int full, double R1, double R2,
                double* E, double* F, double* W) {
    Params p;
    params_of(x, full, &p);
    memset(E, 0, sizeof(double) * (size_t)S);
    memset(F, 0, sizeof(double) * 3 * (size_t)N);
    memset(W, 0, sizeof(double) * 6 * (size_t)S);
    double G[3 * TC_MAX_NBR];
    for (int i = 0; i < N; ++i) {
        const int64_t s0 = ent_start[i];
        const int M = (int)(ent_start[i + 1] - s0);
        double U;
        if (site(&p, R1, R2, ent_d + 3 * s0, M, &U, G) != 0) return -1;
        const int64_t st = atom_struct[i];
        E[st] += U;
        for (int m = 0; m < M; ++m) {
            const int64_t j = ent_j[s0 + m];
            const double* dv = ent_d + 3 * (s0 + m);
            for (int a = 0; a < 3; ++a) {
                F[3 * i + a] += G[3 * m + a];       /* d = r_j - r_i: dU/dr_i = -G */
                F[3 * j + a] -= G[3 * m + a];
            }
            for (int k = 0; k < 6; ++k) W[6 * st + k] -= G[3 * m + V6[k][0]] * dv[V6[k][1]];
        }
    }
    return 0;
}

static double rel_rmse(double res, double norm) { return res > 0.0 ? sqrt(res / norm) : 0.0; }

/*
 * Z, Z_e, Z_v, Z_f [P][4] of P parameter sets X [P][nx] (nx = 6, or 9 with
 * full = 1) against per-atom reference energies eref [S], per-atom virials
 * wref [S][6] and forces fref [N][3], weights w [3].  Candidates are shared
 * out over `threads` OpenMP threads (0: the runtime's default); each
 * candidate's sums run in a fixed order.  Returns 0, or -1 as tc_evaluate,
 * or -2 if a work buffer cannot be allocated.
 */
int tc_fitness(int N, int S, const int64_t* ent_start, const int64_t* ent_j, const double* ent_d,
               const int64_t* atom_struct, int P, const double* X, int full, double R1, double R2,
               const double* eref, const double* wref, const double* fref, const double* w,
               double* Z, int threads) {
    const int nx = full ? 9 : 6;
    int64_t* sizes = (int64_t*)calloc((size_t)S, sizeof(int64_t));
    if (!sizes) return -2;
    for (int i = 0; i < N; ++i) sizes[atom_struct[i]]++;
    double Qe = 0.0, Qv = 0.0, Qf = 0.0;
    for (int s = 0; s < S; ++s) {
        Qe += eref[s] * eref[s];
        for (int k = 0; k < 6; ++k) Qv += wref[6 * s + k] * wref[6 * s + k];
    }
    for (int i = 0; i < 3 * N; ++i) Qf += fref[i] * fref[i];
    int status = 0;
#ifdef _OPENMP
    const int nt = threads > 0 ? threads : omp_get_max_threads();
#else
    (void)threads;
#endif
#pragma omp parallel num_threads(nt)
    {
        double* E = (double*)malloc(sizeof(double) * (size_t)S);
        double* F = (double*)malloc(sizeof(double) * 3 * (size_t)N);
        double* Wv = (double*)malloc(sizeof(double) * 6 * (size_t)S);
        const int ok = E && F && Wv;
#pragma omp for schedule(dynamic, 1)
        for (int c = 0; c < P; ++c) {
            if (!ok) {
#pragma omp atomic write
                status = -2;
                continue;
            }
            if (tc_evaluate(N, S, ent_start, ent_j, ent_d, atom_struct, X + (size_t)nx * c, full, R1, R2,
                            E, F, Wv) != 0) {
#pragma omp atomic write
                status = -1;
                continue;
            }
            double re = 0.0, rv = 0.0, rf = 0.0;
            for (int s = 0; s < S; ++s) {
                const double n = (double)sizes[s];
                const double de = E[s] / n - eref[s];
                re += de * de;
                for (int k = 0; k < 6; ++k) {
                    const double dw = Wv[6 * s + k] / n - wref[6 * s + k];
                    rv += dw * dw;
                }
            }
            for (int i = 0; i < 3 * N; ++i) {
                const double df = F[i] - fref[i];
                rf += df * df;
            }
            const double Ze = rel_rmse(re, Qe), Zv = rel_rmse(rv, Qv), Zf = rel_rmse(rf, Qf);
            Z[4 * c + 0] = w[0] * Ze + w[1] * Zv + w[2] * Zf;
            Z[4 * c + 1] = Ze;
            Z[4 * c + 2] = Zv;
            Z[4 * c + 3] = Zf;
        }
        free(E);
        free(F);
        free(Wv);
    }
    free(sizes);
    return status;
}

/* Threads the OpenMP runtime would use for tc_fitness with threads = 0. */
int tc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
