/*
 * mt_tersoff.h -- C ABI of the MI355X minimal-Tersoff fitting library.
 *
 * The library evaluates the minimal Tersoff potential of Fan et al.,
 * "A minimal Tersoff potential for diamond silicon with improved descriptions
 * of elastic and phonon transport properties" (arXiv:1909.11474), for every
 * candidate parameter set of a genetic-algorithm population and every training
 * structure, and returns energies, forces and virials (Sec. II) or the weighted
 * relative-RMSE fitness Z = w_e Z_e + w_v Z_v + w_f Z_f (Sec. III.B) and its
 * gradient with respect to the six parameters; the same for the
 * nine-parameter Tersoff form (the *_tf entry points).  One GPU kernel covers
 * all candidate x structure pairs of a call, as the GPU implementation of
 * Sec. III.C describes.  Position updates and velocity-Verlet kernels serve
 * the molecular dynamics the potential is built for (Sec. IV.C).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units: energies eV, lengths Angstrom, forces eV/A, velocities A/fs.
 * Parameters: x[p*6 + k], k = 0..5 = D0 (eV), alpha (1/A), r0 (A), beta, n, h
 *   (Sec. II.B; the Pauling slope S is fixed to 2, so A = D0 exp(2 alpha r0),
 *   B = 2 D0 exp(alpha r0), lambda = 2 alpha, mu = alpha).  x lives in device
 *   memory, float64, row-major [P][6].
 * Virial: W = -dE/d(strain), positive under compression; six components in
 *   the order xx, yy, zz, yz, zx, xy.  Per-atom virial W_i (9 components,
 *   row-major xx xy xz yx yy yz zx zy zz) is sum_j r_ij (x) dU_j/dr_ji with
 *   r_ij = r_j - r_i, and sums over atoms to W.
 * Memory: every pointer argument marked "device" is device memory owned by the
 *   caller (for instance a torch tensor's data_ptr()); the library never keeps
 *   a caller pointer beyond the call.  Arrays are contiguous and float64
 *   unless stated otherwise.
 * Streams: `stream` is a hipStream_t passed as void* (NULL = default stream).
 *   Evaluation calls are enqueued on it and return without synchronising;
 *   set creation, reference attachment, mt_set_update_positions,
 *   mt_set_list_skin and mt_profile_fitness_kernels synchronise it.
 * Errors: every call returns MT_OK (0) or a negative mt_status; mt_last_error()
 *   then gives a message for the calling thread.  Argument errors are detected
 *   before any work is enqueued.  A candidate whose parameters are outside the
 *   potential's domain (non-finite, D0 <= 0, alpha <= 0, n <= 0, beta < 0) is
 *   not a call error: its outputs are NaN and the other candidates are
 *   unaffected.
 * Threads: an mt_set may be used from one thread at a time.
 *
 * Tersoff form: tersoff_eval_tf, fitness_eval_tf and fitness_grad_tf take the nine-parameter
 * form of Sec. II.A (Eqs. 2-9 with Tersoff's angular function, Eq. 8) written
 * through Eqs. 11-14 with a free slope S:
 *   x[p*9 + k], k = 0..8 = D0 (eV), alpha (1/A), r0 (A), S, gamma, n, c, d, h;
 *   A = D0/(S-1) exp(alpha r0 sqrt(2S)), B = S D0/(S-1) exp(alpha r0 sqrt(2/S)),
 *   lambda = alpha sqrt(2S), mu = alpha sqrt(2/S),
 *   zeta_ij = sum_k f_C(r_ik) gamma (1 + c^2/d^2 - c^2/(d^2 + (cos theta_ijk - h)^2)).
 *   Device float64 [P][9].  Outside the domain: non-finite, D0 <= 0, alpha <= 0,
 *   S <= 1, gamma < 0, n <= 0 or d = 0 (NaN outputs for that candidate).
 */
#ifndef MT_TERSOFF_H
#define MT_TERSOFF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mt_set mt_set;   /* opaque: structures, neighbour lists, references */

enum mt_status {
    MT_OK = 0,
    MT_EINVAL = -1,          /* bad argument (NULL, size <= 0, R2 <= R1, ...)         */
    MT_ENOMEM = -2,          /* device allocation failed                            */
    MT_EHIP = -3,            /* a HIP runtime call failed                           */
    MT_ENBR_OVERFLOW = -4,   /* an atom has more neighbours than the capacity       */
    MT_ENOREF = -5,          /* fitness requested but no reference data attached    */
    MT_ESTATE = -6,          /* call not valid in the set's current state           */
    MT_ECOINCIDENT = -7      /* two atoms (or an atom and an image) coincide        */
};

enum mt_precision {
    MT_FP64 = 0,             /* all arithmetic in float64                            */
    MT_FP32_ACC64 = 1        /* per-pair/triplet arithmetic in float32; per-structure
                                energy, virial and fitness sums in float64           */
};

enum mt_schedule {
    MT_BATCHED = 0,          /* one launch covers all candidate x structure pairs
                                (replayed from a captured HIP graph)                 */
    MT_PLAIN = 1             /* one launch per (candidate, structure) pair           */
};

/* Largest coordination number handled by the batched kernels. */
#define MT_MAX_NBR 16
/* Largest structure handled by the batched kernels; bigger structures take the
 * two-pass large-system kernels. */
#define MT_MAX_BATCHED_ATOMS 512
/* Largest coordination number handled by fitness_grad (every set allows). */
#define MT_MAX_GRAD_NBR MT_MAX_NBR

/*
 * Build a structure set: copies the structures and finds, on the GPU with a
 * cell list, every neighbour entry (j, periodic image T) of every atom i with
 * 0 < |r_j + T - r_i| < R2.  The cutoff f_C of Sec. II.A vanishes at and
 * beyond R2, so these are exactly the interacting pairs; R1 and R2 are fixed by
 * hand in the paper (Sec. II.B: 2.8 and 3.2 A), not fitted, so the neighbour
 * lists and all pair geometry are built once here and reused by every call.
 * Cells may be triclinic and smaller than 2 R2 (several images of one atom,
 * or of the atom itself, can then be neighbours).
 *
 *   out          receives the new set (host pointer to a host pointer)
 *   n_struct     S >= 1
 *   atom_offset  host int64 [S+1]; atoms of structure s are
 *                atom_offset[s] .. atom_offset[s+1]-1; atom_offset[0] = 0 and
 *                every structure has at least one atom
 *   pos          device float64 [3][N_tot] Cartesian positions, SoA (x row,
 *                then y row, then z row); atoms need not be wrapped into the cell
 *   cell         device float64 [S][3][3]; rows are the lattice vectors a, b, c
 *   R1, R2       cutoff radii, 0 < R1 < R2
 *   max_nbr      neighbour capacity per atom, 1..MT_MAX_NBR
 * Returns MT_ENBR_OVERFLOW if any atom has more than max_nbr neighbours and
 * MT_ECOINCIDENT for coincident atoms; no set is created then.
 */
int mt_set_create(mt_set** out, int n_struct, const int64_t* atom_offset,
                  const double* pos, const double* cell, double R1, double R2,
                  int max_nbr, void* stream);

/*
 * Attach reference data for the fitness (Sec. III.B), copied into the set:
 *   e_ref  device [S]       reference energy per atom of each structure (eV/atom)
 *   w_ref  device [S][6]    reference virial per atom (eV/atom), xx yy zz yz zx xy
 *   f_ref  device [3][N_tot] reference forces (eV/A), SoA
 * Each of sum e_ref^2, sum w_ref^2 and sum |f_ref|^2 must be positive (they are
 * the denominators of the relative RMSEs); otherwise MT_EINVAL.
 */
int mt_set_attach_reference(mt_set* set, const double* e_ref, const double* w_ref,
                            const double* f_ref, void* stream);

/* Release the set and its device memory.  NULL is accepted. */
int mt_set_destroy(mt_set* set);

/*
 * Sizes of a set, written to host int64 stats[8]:
 *   0 n_struct, 1 n_atoms, 2 n_bonds (directed neighbour entries),
 *   3 n_triplets (ordered (j, k != j) pairs of entries sharing a centre atom),
 *   4 largest coordination, 5 largest structure (atoms),
 *   6 structures handled by the batched kernels, 7 by the large-system kernels.
 */
int mt_set_stats(const mt_set* set, int64_t* stats);

/*
 * New positions for the set's atoms (same structures, cells and atom counts),
 * for molecular dynamics: neighbour lists and bond geometry are rebuilt in the
 * set's buffers.  pos is device [3][N_tot] float64 in the caller's atom order.
 * Work lists and captured graphs are rebuilt on the next call, and attached
 * reference data is dropped (attach it again before fitness calls).
 * Synchronises the stream.  Errors as for mt_set_create; after a failed update
 * every later call on the set returns MT_ESTATE (destroy it).
 */
int mt_set_update_positions(mt_set* set, const double* pos, void* stream);

/*
 * Neighbour lists with a Verlet skin: rebuild the set's lists with every pair
 * closer than R2 + skin (A, >= 0; pairs beyond R2 carry f_C = 0 and add
 * nothing), so that mt_set_update_geometry can move atoms without a new
 * search until some atom has moved skin/2 since the last rebuild
 * (mt_set_update_positions).  mt_set_neighbors then lists the skin pairs too.
 * Synchronises the stream; errors as for mt_set_update_positions.
 */
int mt_set_list_skin(mt_set* set, double skin, void* stream);

/*
 * New positions with the neighbour lists of the last rebuild: bond geometry
 * only, asynchronous on `stream`, no host synchronisation.  Correct while no
 * atom has moved more than skin/2 since that rebuild (the caller checks, for
 * instance with mt_md_max_disp).  pos device [3][N_tot].
 */
int mt_set_update_geometry(mt_set* set, const double* pos, void* stream);

/*
 * Copy the neighbour entries out, in the caller's atom numbering, for checks:
 *   i, j    device int32 [n_bonds]  global atom indices (centre, neighbour)
 *   shift   device int32 [3][n_bonds] lattice-vector multiples n1 n2 n3 of the
 *           image: r_ij = r_j + n1 a + n2 b + n3 c - r_i
 * Entries are grouped by centre atom; the order inside a group is unspecified.
 */
int mt_set_neighbors(const mt_set* set, int32_t* i, int32_t* j, int32_t* shift, void* stream);

/*
 * Energies, forces and virials of P parameter sets on every structure
 * (Sec. II.A/II.B; forces F_i = -dE/dr_i and virial W = -dE/d(strain), i.e. the
 * exact derivatives of the site-energy sum, which the cited force and virial
 * formulas compute).  Any output may be NULL to skip it.
 *   x             device [P][6]
 *   energy        device [P][S]        total energy of each structure (eV)
 *   force         device [P][3][N_tot] forces (eV/A)
 *   virial        device [P][S][6]     total virial of each structure (eV)
 *   atom_virial   device [P][9][N_tot] per-atom virial (eV)
 *   vel           device [3][N_tot]    velocities (A/fs), needed for heat_current
 *   heat_current  device [P][3]        sum_i W_i v_i over all atoms (eV A/fs)
 */
int tersoff_eval(mt_set* set, const double* x, int P, int precision, int schedule,
                 double* energy, double* force, double* virial, double* atom_virial,
                 const double* vel, double* heat_current, void* stream);

/*
 * tersoff_eval for the nine-parameter Tersoff form (Sec. II.A, Eqs. 2-9, with
 * Eqs. 11-14 at a free slope S): x is device [P][9] as described at the top
 * of this file; every other argument, output and error as for tersoff_eval.
 */
int tersoff_eval_tf(mt_set* set, const double* x, int P, int precision, int schedule,
                    double* energy, double* force, double* virial, double* atom_virial,
                    const double* vel, double* heat_current, void* stream);

/*
 * Fitness of P parameter sets against the attached reference (Sec. III.B):
 *   Z_e = sqrt(sum_s (e_s - e*_s)^2 / sum_s e*_s^2), e_s = E_s / N_s,
 *   Z_v the same over the six virial-per-atom components of every structure,
 *   Z_f the same over all force components, Z = w_e Z_e + w_v Z_v + w_f Z_f.
 *   w   host float64 [3] = w_e, w_v, w_f
 *   Z   device [P][4] = Z, Z_e, Z_v, Z_f
 * MT_ENOREF without a reference.
 */
int fitness_eval(mt_set* set, const double* x, int P, const double* w, int precision,
                 int schedule, double* Z, void* stream);

/*
 * fitness_eval for the nine-parameter Tersoff form (the Sec. III.B fitness of
 * the Sec. II.A potential): x is device [P][9] as described at the top of this
 * file; w, Z, schedule, precision and errors as for fitness_eval.
 */
int fitness_eval_tf(mt_set* set, const double* x, int P, const double* w, int precision,
                    int schedule, double* Z, void* stream);

/*
 * Fitness and its gradient dZ/dx with respect to the six parameters (the
 * derivative of the Sec. III.B fitness, including the force and virial terms,
 * which need mixed second derivatives of the energy).  A term with Z_x = 0
 * contributes no gradient.  Every set fitness_eval accepts is handled:
 * structures over MT_MAX_BATCHED_ATOMS atoms (or too large for one block's LDS
 * with the adjoint's residual buffer) take a two-pass adjoint that stages bond
 * gradients and force residuals in device memory, held by the set.
 *   Z     device [P][4]
 *   dZdx  device [P][6]
 */
int fitness_grad(mt_set* set, const double* x, int P, const double* w, int precision,
                 double* Z, double* dZdx, void* stream);

/*
 * fitness_grad for the nine-parameter Tersoff form: x is device [P][9] as
 * described at the top of this file and dZdx is device [P][9], the derivative
 * with respect to D0, alpha, r0, S, gamma, n, c, d, h; limits and errors as for
 * fitness_grad.
 */
int fitness_grad_tf(mt_set* set, const double* x, int P, const double* w, int precision,
                    double* Z, double* dZdx, void* stream);

/*
 * Device bytes of the fixed partial-sum array that fitness_eval_noalloc uses
 * (32 MiB per GPU, held from the first such call until the process ends).
 */
#define MT_NOALLOC_SCRATCH_BYTES (32u << 20)

/*
 * fitness_eval for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid allocation): the
 * same batched kernels and result as fitness_eval (minimal form, batched
 * schedule), with the per-slot partial sums in a fixed device array of
 * MT_NOALLOC_SCRATCH_BYTES per GPU instead of the set's workspace.  It calls
 * no hipMalloc or hipFree and captures no graph: the kernels are launched
 * directly on `stream`.
 *   x, P, w, precision, Z  as for fitness_eval
 * The work list for this P, precision and launch shape must exist already: make
 * one fitness_eval call (or mt_autotune) with them first, else MT_ESTATE.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (each call overwrites every sum it reads, nothing has to start at
 * zero); calls that overlap on one GPU, from any thread or stream, race.
 * Errors: as for fitness_eval; MT_EINVAL when P x (partial-sum slots of the
 * set) x 64 bytes exceeds MT_NOALLOC_SCRATCH_BYTES, when the set has a
 * structure that takes the two-pass path (over MT_MAX_BATCHED_ATOMS atoms, or
 * too large for one block's LDS), or when the current device is not the set's.
 * fitness_terms does not read these sums (MT_ESTATE after this call).
 */
int fitness_eval_noalloc(mt_set* set, const double* x, int P, const double* w, int precision,
                         double* Z, void* stream);

/*
 * Per-structure terms behind the most recent fitness_eval, fitness_eval_tf,
 * fitness_grad or fitness_grad_tf call on this set: the predicted quantities
 * whose residuals the Sec. III.B fitness sums, for comparing predicted and
 * reference energies and virials structure by structure.  They are read from
 * the partial sums that call left in the set's workspace, so they are the
 * values its Z was computed from (float32 arithmetic with float64 sums for
 * MT_FP32_ACC64).
 *   x   device [P][6] or [P][9]: the parameter sets of that call; read only to
 *       give candidates outside the potential's domain NaN rows
 *   e   device [P][S]     E_s / N_s (eV/atom), or NULL
 *   w   device [P][S][6]  W_s / N_s (eV/atom), xx yy zz yz zx xy, or NULL
 *   rf  device [P][S]     sum over the structure's atoms of |F_i - F*_i|^2
 *                         (eV^2/A^2), or NULL
 * Enqueued on `stream`, which must be that call's stream or ordered after it.
 * Errors: MT_EINVAL for a NULL set or x, or P other than that call's;
 * MT_ESTATE when no fitness call has run since the set was created, or
 * tersoff_eval, mt_profile_fitness_kernels, mt_autotune, a position update or
 * a reference attachment has overwritten or outdated the partial sums since.
 */
int fitness_terms(mt_set* set, const double* x, int P, double* e, double* w, double* rf,
                  void* stream);

/*
 * Molecular-dynamics steps for the potential's application (Sec. IV.C:
 * equilibrium and homogeneous non-equilibrium MD of diamond Si).  Velocity
 * Verlet is kick(dt/2), drift(dt), mt_set_update_positions, tersoff_eval,
 * kick(dt/2).  Units: A, fs, u, eV; arrays device float64 SoA [3][N] in the
 * caller's atom order; all calls are asynchronous on `stream`.
 *
 * mt_md_kick: v_i += dt_half (F_i + F_ext,i - <F_ext>) / (m_i 103.642691),
 *   F_ext,i = W_i^T F_e (W_i the per-atom virial of tersoff_eval, [9][N]
 *   row-major), <F_ext> = W^T F_e / N with W the total virial [6] (xx yy zz
 *   yz zx xy; symmetric).  The external power sum_i F_ext,i . v_i equals
 *   F_e . J with the heat current J = sum_i W_i v_i of tersoff_eval, and the
 *   mean is removed so that the driving force adds no momentum.  fe (host [3],
 *   in 1/A), atom_virial and virial are all NULL for equilibrium MD, or
 *   all given.  inv_mass device [N] (1/u).
 * mt_md_drift: r_i += dt v_i.
 * mt_md_scale: v_i *= lambda (velocity-rescaling thermostats).
 * mt_md_kinetic: out (device [4]) = sum_i m_i |v_i|^2 (u A^2/fs^2) and the
 *   momentum sum_i m_i v_i, in a fixed summation order.
 * Errors: MT_EINVAL for N <= 0 or a NULL required pointer; MT_EHIP if a
 * launch fails.
 */
int mt_md_kick(int N, double* vel, const double* force, const double* atom_virial,
               const double* virial, const double* fe, const double* inv_mass, double dt_half,
               void* stream);
int mt_md_drift(int N, double* pos, const double* vel, double dt, void* stream);
int mt_md_scale(int N, double* vel, double lambda, void* stream);
int mt_md_kinetic(int N, const double* vel, const double* mass, double* out, void* stream);
/* out (device [1]) = max_i |r_i - ref_i|^2 (A^2), for the skin check. */
int mt_md_max_disp(int N, const double* pos, const double* ref, double* out, void* stream);

/*
 * Choose launch shapes (block size, candidate tile, schedule) for this set
 * and population size by timing the candidates on the GPU; the choice is kept
 * in the set and used by later calls with the same P and precision.  With
 * reference data attached it also chooses between replaying a captured graph
 * per fitness_eval call and launching the kernels directly, by the host-clock
 * rate of a burst of back-to-back calls.  When cache_path is not NULL every
 * timing is appended to that text file as a comment line ("# ...") and the
 * choice as a line "<set key> | block=B tile=T persistent=0|1 graph=0|1 ms=..";
 * a matching entry already there is used without timing (MT_EINVAL if its
 * shape is out of range: block a multiple of 64 up to 512, tile >= 0).  Calls
 * that overlap on one set race (the set's workspace is shared).
 */
int mt_autotune(mt_set* set, int P, int precision, const char* cache_path);

/*
 * Kernel timing for measurement.  While enabled, every launch of the batched
 * evaluation kernel (and of the adjoint kernel) is bracketed by HIP events on
 * the stream it is launched on, and calls run without graph replay.
 * mt_profile_read synchronises those events and returns, per kernel kind
 * (0 = batched evaluation, 1 = adjoint), the summed duration in milliseconds
 * and the number of launches since the last read, then resets the counters.
 *   ms        host double [2]
 *   launches  host int64 [2]
 */
int mt_profile_enable(mt_set* set, int enable);
int mt_profile_read(mt_set* set, double* ms, int64_t* launches);

/*
 * Back-to-back timing of the batched fitness kernels, for roofline figures:
 * the kernel launches that fitness_eval (nx = 6) or fitness_eval_tf (nx = 9)
 * makes for P candidates at this precision and launch shape (two-pass
 * structures and the finalize excluded) are issued reps times in a row on
 * the stream between one pair of HIP events, so the dispatch latency that an
 * event pair around each launch adds is paid once instead of per launch.
 *   x         device double [P][nx], as for fitness_eval / fitness_eval_tf
 *   ms        host double: average milliseconds per pass
 *   launches  host int64: kernel launches per pass
 * Overwrites the set's partial sums (not Z); synchronises the stream.
 * Errors: MT_EINVAL for a NULL pointer, nx not 6 or 9, P or reps <= 0;
 * MT_ENOREF without reference data; MT_EHIP if a HIP call fails.
 */
int mt_profile_fitness_kernels(mt_set* set, const double* x, int nx, int P, int precision, int reps,
                               double* ms, int64_t* launches, void* stream);

/*
 * The same back-to-back timing per kernel launch: each launch of the batched
 * fitness plan (one per coordination class and block size) is issued reps
 * times in a row between one event pair, so that the roofline of each kernel
 * can be taken on its own.
 *   x, nx, P, precision, reps  as for mt_profile_fitness_kernels
 *   max_launches        capacity of ms and coordination_class
 *   ms                  host double [max_launches]: average ms of each launch
 *   coordination_class  host int [max_launches]: largest coordination the
 *                       launch's kernel instance serves
 *   struct_launch       host int [S] or NULL: index of the launch evaluating
 *                       each structure, -1 for the two-pass path
 *   n_launches          host int: launches of the plan
 * Overwrites the set's partial sums; synchronises the stream.  Errors as for
 * mt_profile_fitness_kernels; MT_EINVAL also when the plan has more than
 * max_launches launches (n_launches is set).
 */
int mt_profile_fitness_launches(mt_set* set, const double* x, int nx, int P, int precision, int reps,
                                int max_launches, double* ms, int* coordination_class,
                                int* struct_launch, int* n_launches, void* stream);

/* Message for the calling thread's most recent error (never NULL). */
const char* mt_last_error(void);

/* Library version string. */
const char* mt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MT_TERSOFF_H */
