// Host-side state of a structure set and the launch entry points of each
// translation unit.
#pragma once

#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "mt_common.h"
#include "mt_tersoff.h"

namespace mt {

// Device buffer owned by the library.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    // Grow to at least `n` bytes (contents are not preserved).
    hipError_t reserve(size_t n) {
        if (n <= bytes && p) return hipSuccess;
        release();
        hipError_t e = hipMalloc(&p, n < 256 ? 256 : n);
        if (e == hipSuccess) bytes = n < 256 ? 256 : n;
        return e;
    }
    template <typename T> T* as() const { return static_cast<T*>(p); }
};

struct LaunchCfg {            // launch shape of the batched kernel
    int block = 0;            // threads per block, multiple of 64, >= largest padded structure
    int tile = 0;             // candidates per work item (0: derived from the block)
    int persistent = 0;       // 1: static LPT bins over a fixed grid; 0: one block per item
    int graph = 1;            // fitness_eval: 1 replays a captured graph, 0 launches directly
};

struct ClassPlan {            // work list of one launch: a coordination class at one block size
    int mc = 0;               // class: largest coordination the kernel instance serves
    int block = 0;            // threads per block of this launch
    DevBuf items;             // Item[n_items]
    DevBuf bin_off;           // int[n_bins + 1]
    std::vector<Item> h_items;
    int n_items = 0;
    int n_bins = 0;
    size_t lds = 0;           // dynamic LDS bytes
};

struct ItemPlan {             // uploaded work lists for one (P, launch shape, kernel family)
    std::vector<std::unique_ptr<ClassPlan>> cls;
    // structures of at most MT_MAX_BATCHED_ATOMS atoms whose single replica does
    // not fit the LDS of a block in this family: evaluated by the two-pass path
    std::vector<int> twopass;
};

// Kernel families: precision x (fitness, energy/force/virial, adjoint) for the
// minimal potential and (suffix F) for the nine-parameter Tersoff form.
enum Family {
    FAM_FIT32 = 0, FAM_EVAL32, FAM_FIT64, FAM_EVAL64, FAM_ADJ32, FAM_ADJ64,
    FAM_FIT32F, FAM_EVAL32F, FAM_FIT64F, FAM_EVAL64F, FAM_ADJ32F, FAM_ADJ64F, NFAM
};

struct GraphKey {             // what a captured fitness graph depends on
    const void* x = nullptr;
    void* Z = nullptr;
    int P = 0, precision = 0, block = 0, tile = 0, persistent = 0, form = 0;
    double w[3] = {0, 0, 0};
    bool operator==(const GraphKey& o) const {
        return x == o.x && Z == o.Z && P == o.P && precision == o.precision && form == o.form &&
               block == o.block &&
               tile == o.tile && persistent == o.persistent && w[0] == o.w[0] && w[1] == o.w[1] &&
               w[2] == o.w[2];
    }
};

// Temporaries of the neighbour search and table build, kept with the set so
// that position updates (molecular dynamics) reuse them instead of allocating.
struct BuildScratch {
    DevBuf meta, atom_bin, atom_wrap, bin_count, bin_start, bin_fill, bin_atoms, cnt, ent_j, ent_sh,
        inv, flags, st_nb, st_trip;
};

struct GraphEntry {
    GraphKey key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

}  // namespace mt

struct mt_set {
    int S = 0, N = 0, kcap = 0, kmax = 0, nb = 0, nslots = 0;
    long long ntrip = 0;
    int max_atoms = 0, n_batched = 0, n_large = 0;
    size_t lds_max = 65536;   // dynamic LDS bytes a block may use on the set's device
    double R1 = 0, R2 = 0;
    double skin = 0;          // neighbour lists hold pairs closer than R2 + skin
    int device = 0;

    // host copies of per-structure tables
    std::vector<int> h_off, h_boff, h_npad, h_kmax, h_slot, h_large, h_xsize;
    std::vector<long long> h_trip;           // ordered triplets per structure

    // device data (see mt_common.h for the layout)
    mt::DevBuf pos, cell;
    mt::DevBuf st_off, st_boff, st_npad, st_kmax, st_slot, st_xsize;
    mt::DevBuf perm, nnb, lbo, xbase, rev, revc, jl;
    mt::DevBuf nbr_j, nbr_sh;                // caller-numbering neighbour entries, [kcap][N]
    mt::DevBuf gf, gd;                       // float / double geometry, 8 resp. 7 arrays of [kcap][N]
    mt::DevBuf gf_rlo;                       // float low part of r, [kcap][N]
    mt::DevBuf gpk;                          // float geometry packed as 2 x float4, [2][kcap][N]
    mt::DevBuf gcs;                          // cos(theta) of bond pairs j < k < 6, [15][N] float

    // references (sorted order)
    bool has_ref = false;
    // false after a failed mt_set_update_positions: the tables are inconsistent
    bool usable = true;
    mt::DevBuf eref, wref, fref32, fref64;
    double Q[3] = {0, 0, 0};

    // parameter sets of the call being enqueued (device [P][6], or [P][9] for
    // the Tersoff form) and their form (0 minimal, 1 Tersoff form)
    const double* cur_x = nullptr;
    int cur_form = 0;
    // population size and form of the fitness partial sums the workspace holds
    // (after fitness_eval / fitness_grad; 0 once another call overwrote them)
    int fit_P = 0;
    int fit_form = 0;

    // workspaces
    mt::DevBuf partial;                      // [P][nslots][NV] double
    mt::DevBuf partial2;                     // gradient partials
    mt::DevBuf abuf;                         // two-pass adjoint: staged force residuals
    // fitness_grad: the fitness writes each batched atom's force residual
    // F - F* here ([P][3][N] in the call's arithmetic, sorted atom order) and
    // the adjoint reads it; grad_resid is set only for that fitness call
    mt::DevBuf resid;
    void* grad_resid = nullptr;
    mt::DevBuf zwork;                        // [P][4] scratch for fitness_grad
    mt::DevBuf gbuf;                         // large path bond gradients
    mt::DevBuf scalars;                      // small device scratch
    mt::BuildScratch build;                  // neighbour-search temporaries

    std::map<std::tuple<int, int, int, int, int>, std::unique_ptr<mt::ItemPlan>> plans;
    std::map<std::pair<int, int>, mt::LaunchCfg> tuned;     // (P, precision) -> cfg
    std::vector<mt::GraphEntry> graphs;      // most recently used first
    hipStream_t capture_stream = nullptr;

    // kernel timing (mt_profile_enable): event pairs per kernel kind
    bool profiling = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events[2];
    std::vector<hipEvent_t> event_pool;

    mt::SetDev dev() const;
    ~mt_set();
};

namespace mt {

// mt_set.hip
int build_set(mt_set* set, const int64_t* atom_offset, const double* pos, const double* cell,
              hipStream_t stream);
int attach_reference(mt_set* set, const double* e_ref, const double* w_ref, const double* f_ref,
                     hipStream_t stream);
int export_neighbors(const mt_set* set, int32_t* i, int32_t* j, int32_t* shift, hipStream_t stream);
// New positions with the neighbour lists of the last build (no host sync).
int update_geometry(mt_set* set, const double* pos, hipStream_t stream);

// mt_api.hip: destroy the set's captured fitness graphs (after any workspace
// they reference is reallocated)
void clear_graphs(mt_set* set);

// mt_eval.hip
int launch_batched(mt_set* set, const LaunchCfg& cfg, int P, int precision, int mode,
                   const double* vel, double* force, double* atom_virial, hipStream_t stream);
int launch_plain(mt_set* set, int P, int precision, int mode, const double* vel, double* force,
                 double* atom_virial, hipStream_t stream);
// Average time of reps back-to-back passes of the batched fitness kernels.
int time_batched_kernels(mt_set* set, const LaunchCfg& cfg, int P, int precision, int reps,
                         hipStream_t stream, double* ms, int64_t* launches);
// Each launch of the batched fitness plan timed alone (reps back to back).
int time_class_launches(mt_set* set, const LaunchCfg& cfg, int P, int precision, int reps,
                        hipStream_t stream, int max_launches, double* ms, int* mc, int* struct_launch,
                        int* n_launches);
int launch_large(mt_set* set, int P, int precision, int mode, const double* vel, double* force,
                 double* atom_virial, hipStream_t stream);
// Reserve the two-pass staging buffer for the set's large structures and the
// plan's two-pass structures (before graph capture: capture may not allocate).
int reserve_twopass(mt_set* set, const ItemPlan* plan, int P, int precision);
// partial: the per-slot partial sums to finalize (null: the set's workspace)
int launch_finalize_fit(mt_set* set, int P, const double* w, double* Z, hipStream_t stream,
                        const double* partial = nullptr);
int launch_finalize_eval(mt_set* set, int P, double* energy, double* virial, double* heat,
                         hipStream_t stream);
// Per-structure e_s, w_s and squared force residual from the fitness partial
// sums in the set's workspace (set->cur_x and cur_form select the candidates'
// domain check).
int launch_fitness_terms(mt_set* set, int P, double* e, double* w, double* rf, hipStream_t stream);
// The adjoint of the batched structures reads the force residuals the
// fitness call just before it wrote to set->resid (set->grad_resid).
int launch_adjoint(mt_set* set, const LaunchCfg& cfg, int P, int precision, const double* w,
                   const double* Z, hipStream_t stream);
int launch_finalize_grad(mt_set* set, int P, const double* Z, double* dZdx, hipStream_t stream);

// MODE_STAGE (two-pass path only): stage the bond gradients, no partial sums
// and no gather.
enum Mode { MODE_FIT = 0, MODE_EVAL = 1, MODE_STAGE = 2 };

ItemPlan* get_plan(mt_set* set, int P, const LaunchCfg& cfg, int family);
// The cached work list for these arguments, or null (never builds one).
ItemPlan* find_plan(mt_set* set, int P, const LaunchCfg& cfg, int family);
// The batched fitness launches of an existing plan, partial sums written to
// `partial` ([P][nslots][kNVFit]); no allocation, no profiling events.
int launch_plan_fit(mt_set* set, ItemPlan* plan, const LaunchCfg& cfg, int precision, double* partial,
                    hipStream_t stream);
// Batched kernel family of a call: precision x mode x parameter form.
int family_for(int precision, int mode, int form);
LaunchCfg default_cfg(const mt_set* set, int P, int precision);
int class_of(int family, int kmax);
const std::vector<int>& family_classes(int family);

// Start/stop events for one kernel launch when the set is profiling (kind 0
// batched, 1 adjoint); null events otherwise.  The launch records them around
// the dispatch itself (hipExtLaunchKernelGGL).
struct ProfScope {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ProfScope(mt_set* s, int kind);
};

}  // namespace mt
