// C ABI entry points (declared in include/mt_tersoff.h): argument checks, set
// lifecycle, dispatch to the batched / plain / large-structure kernels, HIP
// graph replay of the batched fitness path, and the launch-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "mt_host.h"
#include "mt_tersoff.h"

namespace mt {

static thread_local std::string g_last_error = "no error";

void set_error(const std::string& msg) { g_last_error = msg; }

int hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string("HIP error '") + hipGetErrorString(e) + "' in " + what;
    return e == hipErrorOutOfMemory ? MT_ENOMEM : MT_EHIP;
}

}  // namespace mt

using namespace mt;

#define HIPCHECK(call)                                   \
    do {                                                 \
        hipError_t _e = (call);                          \
        if (_e != hipSuccess) return hip_fail(_e, #call); \
    } while (0)

#define TRY(call)                 \
    do {                          \
        int _rc = (call);         \
        if (_rc != MT_OK) return _rc; \
    } while (0)

static int fail(int code, const std::string& msg) {
    set_error(msg);
    return code;
}

mt::SetDev mt_set::dev() const {
    SetDev d{};
    d.S = S; d.N = N; d.kcap = kcap; d.nb = nb; d.nslots = nslots;
    d.st_off = st_off.as<int>(); d.st_boff = st_boff.as<int>(); d.st_npad = st_npad.as<int>();
    d.st_kmax = st_kmax.as<int>(); d.st_slot = st_slot.as<int>(); d.st_xsize = st_xsize.as<int>();
    d.perm = perm.as<int>(); d.nnb = nnb.as<int>(); d.lbo = lbo.as<int>(); d.xbase = xbase.as<int>();
    d.rev = rev.as<int>(); d.revc = revc.as<int>(); d.jl = jl.as<int>();
    const size_t KN = (size_t)kcap * N;
    const float* f = gf.as<float>();
    const float4* pk = gpk.as<float4>();
    d.gf = GeomArrays<float>{f, f + KN, f + 2 * KN, f + 3 * KN, gf_rlo.as<float>(), f + 4 * KN,
                             f + 5 * KN, f + 6 * KN, pk, pk + KN};
    const double* g = gd.as<double>();
    d.gd = GeomArrays<double>{g, g + KN, g + 2 * KN, g + 3 * KN, nullptr, g + 4 * KN,
                              g + 5 * KN, g + 6 * KN, nullptr, nullptr};
    d.gcs = gcs.as<float>();
    d.fref32 = fref32.as<float>();
    d.fref64 = fref64.as<double>();
    return d;
}

void mt::clear_graphs(mt_set* set) {
    for (auto& g : set->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    set->graphs.clear();
}

mt_set::~mt_set() {
    clear_graphs(this);
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    for (auto& v : prof_events)
        for (auto& pr : v) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
}

namespace mt {

static hipEvent_t pool_event(mt_set* set) {
    if (!set->event_pool.empty()) {
        hipEvent_t e = set->event_pool.back();
        set->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

ProfScope::ProfScope(mt_set* set, int kind) {
    if (!set->profiling || kind < 0) return;
    e0 = pool_event(set);
    e1 = pool_event(set);
    if (!e0 || !e1) { e0 = e1 = nullptr; return; }
    set->prof_events[kind].push_back({e0, e1});
}

}  // namespace mt

// Reserve per-call workspaces; any reallocation invalidates captured graphs.
static int ensure_workspace(mt_set* set, int P, int nv) {
    const void* before = set->partial.p;
    HIPCHECK(set->partial.reserve(sizeof(double) * nv * (size_t)P * std::max(1, set->nslots)));
    if (before != set->partial.p) clear_graphs(set);
    return MT_OK;
}

static int check_common(mt_set* set, const double* x, int P, int precision) {
    if (!set) return fail(MT_EINVAL, "set is NULL");
    if (!set->usable) return fail(MT_ESTATE, "the set's last position update failed; destroy it");
    if (!x) return fail(MT_EINVAL, "x is NULL");
    if (P <= 0) return fail(MT_EINVAL, "P must be positive");
    if (precision != MT_FP64 && precision != MT_FP32_ACC64)
        return fail(MT_EINVAL, "precision must be MT_FP64 or MT_FP32_ACC64");
    if ((long long)P * std::max(1, set->nslots) * kNVEval > (1ll << 31))
        return fail(MT_EINVAL, "P too large for this set");
    return MT_OK;
}

static LaunchCfg cfg_for(mt_set* set, int P, int precision) {
    auto it = set->tuned.find({P, precision});
    if (it != set->tuned.end()) return it->second;
    return default_cfg(set, P, precision);
}

extern "C" {

const char* mt_last_error(void) { return g_last_error.c_str(); }

const char* mt_version(void) { return "mt_tersoff 0.1 (gfx950)"; }

int mt_set_create(mt_set** out, int n_struct, const int64_t* atom_offset, const double* pos,
                  const double* cell, double R1, double R2, int max_nbr, void* stream) {
    if (!out) return fail(MT_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_struct <= 0) return fail(MT_EINVAL, "n_struct must be positive");
    if (!atom_offset || !pos || !cell) return fail(MT_EINVAL, "atom_offset, pos and cell must not be NULL");
    if (!(R1 > 0.0) || !(R2 > R1) || !std::isfinite(R2))
        return fail(MT_EINVAL, "cutoffs must satisfy 0 < R1 < R2 < inf");
    if (max_nbr < 1 || max_nbr > MT_MAX_NBR)
        return fail(MT_EINVAL, "max_nbr must be in 1.." + std::to_string(MT_MAX_NBR));
    if (atom_offset[0] != 0) return fail(MT_EINVAL, "atom_offset[0] must be 0");
    for (int s = 0; s < n_struct; ++s)
        if (atom_offset[s + 1] <= atom_offset[s])
            return fail(MT_EINVAL, "structure " + std::to_string(s) + " has no atoms");
    const long long N = atom_offset[n_struct];
    if (N * (long long)max_nbr >= (1ll << 31)) return fail(MT_EINVAL, "too many atoms");
    auto set = new mt_set();
    set->S = n_struct;
    set->N = (int)N;
    set->kcap = max_nbr;
    set->R1 = R1;
    set->R2 = R2;
    (void)hipGetDevice(&set->device);
    int rc = build_set(set, atom_offset, pos, cell, (hipStream_t)stream);
    if (rc != MT_OK) {
        delete set;
        return rc;
    }
    *out = set;
    return MT_OK;
}

int mt_set_attach_reference(mt_set* set, const double* e_ref, const double* w_ref,
                            const double* f_ref, void* stream) {
    if (!set) return fail(MT_EINVAL, "set is NULL");
    if (!e_ref || !w_ref || !f_ref) return fail(MT_EINVAL, "reference pointers must not be NULL");
    if (!set->usable) return fail(MT_ESTATE, "the set's last position update failed; destroy it");
    clear_graphs(set);
    set->fit_P = 0;
    return attach_reference(set, e_ref, w_ref, f_ref, (hipStream_t)stream);
}

int mt_set_update_positions(mt_set* set, const double* pos, void* stream) {
    if (!set || !pos) return fail(MT_EINVAL, "set and pos must not be NULL");
    if (!set->usable) return fail(MT_ESTATE, "the set's last position update failed; destroy it");
    // everything derived from positions is rebuilt in the existing buffers;
    // work lists and captured graphs depend on the coordination layout, and the
    // stored reference forces on the atom order, so all three are dropped
    std::vector<int64_t> off(set->h_off.begin(), set->h_off.end());
    const auto layout = std::make_tuple(set->h_kmax, set->h_xsize, set->h_npad, set->h_large, set->nslots);
    set->has_ref = false;
    set->fit_P = 0;
    const int rc = build_set(set, off.data(), pos, set->cell.as<double>(), (hipStream_t)stream);
    if (rc != MT_OK) {
        set->usable = false;
        return rc;
    }
    // the work lists (and graphs of them) stay valid while every structure keeps
    // its coordination class, exchange-slot layout and padded size
    if (layout != std::make_tuple(set->h_kmax, set->h_xsize, set->h_npad, set->h_large, set->nslots)) {
        clear_graphs(set);
        set->plans.clear();
    }
    return MT_OK;
}

int mt_set_update_geometry(mt_set* set, const double* pos, void* stream) {
    if (!set || !pos) return fail(MT_EINVAL, "set and pos must not be NULL");
    if (!set->usable) return fail(MT_ESTATE, "the set's last position update failed; destroy it");
    return update_geometry(set, pos, (hipStream_t)stream);
}

int mt_set_list_skin(mt_set* set, double skin, void* stream) {
    if (!set) return fail(MT_EINVAL, "set is NULL");
    if (!set->usable) return fail(MT_ESTATE, "the set's last position update failed; destroy it");
    if (!(skin >= 0.0) || !std::isfinite(skin)) return fail(MT_EINVAL, "skin must be finite and >= 0");
    set->skin = skin;
    return mt_set_update_positions(set, set->pos.as<double>(), stream);
}

int mt_set_destroy(mt_set* set) {
    if (set) {
        (void)hipDeviceSynchronize();
        delete set;
    }
    return MT_OK;
}

int mt_set_stats(const mt_set* set, int64_t* stats) {
    if (!set || !stats) return fail(MT_EINVAL, "set and stats must not be NULL");
    stats[0] = set->S;
    stats[1] = set->N;
    stats[2] = set->nb;
    stats[3] = set->ntrip;
    stats[4] = set->kmax;
    stats[5] = set->max_atoms;
    stats[6] = set->n_batched;
    stats[7] = set->n_large;
    return MT_OK;
}

int mt_set_neighbors(const mt_set* set, int32_t* i, int32_t* j, int32_t* shift, void* stream) {
    if (!set || !i || !j || !shift) return fail(MT_EINVAL, "NULL argument");
    return export_neighbors(set, i, j, shift, (hipStream_t)stream);
}

}  // extern "C"

static int eval_impl(mt_set* set, const double* x, int form, int P, int precision, int schedule,
                     double* energy, double* force, double* virial, double* atom_virial,
                     const double* vel, double* heat_current, void* stream) {
    TRY(check_common(set, x, P, precision));
    if (schedule != MT_BATCHED && schedule != MT_PLAIN)
        return fail(MT_EINVAL, "schedule must be MT_BATCHED or MT_PLAIN");
    if (heat_current && !vel) return fail(MT_EINVAL, "heat_current needs vel");
    hipStream_t st = (hipStream_t)stream;
    TRY(ensure_workspace(set, P, kNVEval));
    set->fit_P = 0;
    set->cur_x = x;
    set->cur_form = form;
    if (schedule == MT_BATCHED) {
        const LaunchCfg cfg = cfg_for(set, P, precision);
        TRY(launch_batched(set, cfg, P, precision, MODE_EVAL, vel, force, atom_virial, st));
    } else {
        TRY(launch_plain(set, P, precision, MODE_EVAL, vel, force, atom_virial, st));
    }
    TRY(launch_large(set, P, precision, MODE_EVAL, vel, force, atom_virial, st));
    return launch_finalize_eval(set, P, energy, virial, heat_current, st);
}

static int fitness_sequence(mt_set* set, const double* x, int form, int P, const double* w,
                            int precision, int schedule, double* Z, hipStream_t st) {
    set->cur_x = x;
    set->cur_form = form;
    if (schedule == MT_BATCHED) {
        const LaunchCfg cfg = cfg_for(set, P, precision);
        TRY(launch_batched(set, cfg, P, precision, MODE_FIT, nullptr, nullptr, nullptr, st));
    } else {
        TRY(launch_plain(set, P, precision, MODE_FIT, nullptr, nullptr, nullptr, st));
    }
    TRY(launch_large(set, P, precision, MODE_FIT, nullptr, nullptr, nullptr, st));
    return launch_finalize_fit(set, P, w, Z, st);
}

static int check_fitness(mt_set* set, const double* x, int P, const double* w, int precision, double* Z) {
    TRY(check_common(set, x, P, precision));
    if (!w || !Z) return fail(MT_EINVAL, "w and Z must not be NULL");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(w[k])) return fail(MT_EINVAL, "weights must be finite");
    if (!set->has_ref) return fail(MT_ENOREF, "no reference data attached to the set");
    return MT_OK;
}

static int fitness_graph(mt_set* set, const double* x, int form, int P, const double* w,
                         int precision, int schedule, double* Z, hipStream_t st);

static int fitness_impl(mt_set* set, const double* x, int form, int P, const double* w,
                        int precision, int schedule, double* Z, void* stream) {
    TRY(check_fitness(set, x, P, w, precision, Z));
    if (schedule != MT_BATCHED && schedule != MT_PLAIN)
        return fail(MT_EINVAL, "schedule must be MT_BATCHED or MT_PLAIN");
    hipStream_t st = (hipStream_t)stream;
    TRY(ensure_workspace(set, P, kNVFit));
    set->fit_P = 0;
    const LaunchCfg cfg = cfg_for(set, P, precision);
    if (schedule == MT_PLAIN || set->profiling || !cfg.graph)
        TRY(fitness_sequence(set, x, form, P, w, precision, schedule, Z, st));
    else
        TRY(fitness_graph(set, x, form, P, w, precision, schedule, Z, st));
    set->fit_P = P;
    set->fit_form = form;
    return MT_OK;
}

// Batched fitness by replaying a captured graph of the batched kernel(s) and
// the finalize (captured on the first call with these arguments).
static int fitness_graph(mt_set* set, const double* x, int form, int P, const double* w,
                         int precision, int schedule, double* Z, hipStream_t st) {
    const LaunchCfg cfg = cfg_for(set, P, precision);

    GraphKey key;
    key.x = x; key.Z = Z; key.P = P; key.precision = precision; key.form = form;
    key.block = cfg.block; key.tile = cfg.tile; key.persistent = cfg.persistent;
    key.w[0] = w[0]; key.w[1] = w[1]; key.w[2] = w[2];
    size_t hit = set->graphs.size();
    for (size_t i = 0; i < set->graphs.size(); ++i)
        if (set->graphs[i].key == key) { hit = i; break; }
    if (hit == set->graphs.size()) {
        ItemPlan* plan = get_plan(set, P, cfg, family_for(precision, MODE_FIT, form));
        if (!plan) return fail(MT_EINVAL, "could not build the work list");
        TRY(reserve_twopass(set, plan, P, precision));     // allocate before capture
        if (!set->capture_stream) HIPCHECK(hipStreamCreateWithFlags(&set->capture_stream, hipStreamNonBlocking));
        GraphEntry ge;
        ge.key = key;
        HIPCHECK(hipStreamBeginCapture(set->capture_stream, hipStreamCaptureModeThreadLocal));
        int rc = fitness_sequence(set, x, form, P, w, precision, schedule, Z, set->capture_stream);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(set->capture_stream, &graph);
        if (rc != MT_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        ge.graph = graph;
        e = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return hip_fail(e, "hipGraphInstantiate");
        }
        if (set->graphs.size() >= 16) {
            GraphEntry& old = set->graphs.back();
            (void)hipGraphExecDestroy(old.exec);
            (void)hipGraphDestroy(old.graph);
            set->graphs.pop_back();
        }
        set->graphs.insert(set->graphs.begin(), ge);
        hit = 0;
    } else if (hit != 0) {
        std::swap(set->graphs[0], set->graphs[hit]);
        hit = 0;
    }
    HIPCHECK(hipGraphLaunch(set->graphs[0].exec, st));
    return MT_OK;
}

extern "C" {

int tersoff_eval(mt_set* set, const double* x, int P, int precision, int schedule, double* energy,
                 double* force, double* virial, double* atom_virial, const double* vel,
                 double* heat_current, void* stream) {
    return eval_impl(set, x, 0, P, precision, schedule, energy, force, virial, atom_virial, vel,
                     heat_current, stream);
}

int tersoff_eval_tf(mt_set* set, const double* x, int P, int precision, int schedule,
                    double* energy, double* force, double* virial, double* atom_virial,
                    const double* vel, double* heat_current, void* stream) {
    return eval_impl(set, x, 1, P, precision, schedule, energy, force, virial, atom_virial, vel,
                     heat_current, stream);
}

int fitness_eval(mt_set* set, const double* x, int P, const double* w, int precision, int schedule,
                 double* Z, void* stream) {
    return fitness_impl(set, x, 0, P, w, precision, schedule, Z, stream);
}

int fitness_eval_tf(mt_set* set, const double* x, int P, const double* w, int precision,
                    int schedule, double* Z, void* stream) {
    return fitness_impl(set, x, 1, P, w, precision, schedule, Z, stream);
}

}  // extern "C"

static int grad_impl(mt_set* set, const double* x, int form, int P, const double* w,
                     int precision, double* Z, double* dZdx, void* stream) {
    TRY(check_fitness(set, x, P, w, precision, Z));
    if (!dZdx) return fail(MT_EINVAL, "dZdx must not be NULL");
    hipStream_t st = (hipStream_t)stream;
    TRY(ensure_workspace(set, P, kNVFit));
    // force residuals of the batched atoms, written by the fitness and read by
    // the adjoint
    HIPCHECK(set->resid.reserve((precision == MT_FP64 ? sizeof(double) : sizeof(float)) * 3 * (size_t)P *
                                set->N));
    set->fit_P = 0;
    set->grad_resid = set->resid.p;
    const int frc = fitness_sequence(set, x, form, P, w, precision, MT_BATCHED, Z, st);
    set->grad_resid = nullptr;
    TRY(frc);
    set->fit_P = P;
    set->fit_form = form;
    const LaunchCfg cfg = cfg_for(set, P, precision);
    TRY(launch_adjoint(set, cfg, P, precision, w, Z, st));
    return launch_finalize_grad(set, P, Z, dZdx, st);
}

extern "C" {

int fitness_grad(mt_set* set, const double* x, int P, const double* w, int precision, double* Z,
                 double* dZdx, void* stream) {
    return grad_impl(set, x, 0, P, w, precision, Z, dZdx, stream);
}

int fitness_grad_tf(mt_set* set, const double* x, int P, const double* w, int precision,
                    double* Z, double* dZdx, void* stream) {
    return grad_impl(set, x, 1, P, w, precision, Z, dZdx, stream);
}

int fitness_terms(mt_set* set, const double* x, int P, double* e, double* w, double* rf,
                  void* stream) {
    if (!set) return fail(MT_EINVAL, "set is NULL");
    if (!x) return fail(MT_EINVAL, "x is NULL");
    if (P <= 0) return fail(MT_EINVAL, "P must be positive");
    if (set->fit_P == 0)
        return fail(MT_ESTATE, "no fitness partial sums: call fitness_eval or fitness_grad first");
    if (P != set->fit_P)
        return fail(MT_EINVAL, "P differs from the last fitness call's (" + std::to_string(set->fit_P) + ")");
    set->cur_x = x;
    set->cur_form = set->fit_form;
    return launch_fitness_terms(set, P, e, w, rf, (hipStream_t)stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free fitness: partial sums in a fixed device array.
// ---------------------------------------------------------------------------
// Each GPU the library runs on holds its own copy of this array until the
// process ends; its device address is taken once per device.
static __device__ __align__(256) double scratch[MT_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

int scratch_of_device(int dev, double** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(MT_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        // the array's host-side name is not a device address: ask for this
        // device's copy (the set's device is current here)
        HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return MT_OK;
}
}  // namespace

extern "C" {

int fitness_eval_noalloc(mt_set* set, const double* x, int P, const double* w, int precision,
                         double* Z, void* stream) {
    TRY(check_fitness(set, x, P, w, precision, Z));
    if (set->n_large > 0)
        return fail(MT_EINVAL, "fitness_eval_noalloc: the set has structures over " +
                                   std::to_string(MT_MAX_BATCHED_ATOMS) + " atoms (two-pass path)");
    const size_t need = sizeof(double) * kNVFit * (size_t)P * std::max(1, set->nslots);
    if (need > MT_NOALLOC_SCRATCH_BYTES)
        return fail(MT_EINVAL, "fitness_eval_noalloc: P x partial-sum slots needs " + std::to_string(need) +
                                   " bytes of scratch, more than " +
                                   std::to_string((long long)MT_NOALLOC_SCRATCH_BYTES));
    const LaunchCfg cfg = cfg_for(set, P, precision);
    ItemPlan* plan = find_plan(set, P, cfg, family_for(precision, MODE_FIT, 0));
    if (!plan)
        return fail(MT_ESTATE, "fitness_eval_noalloc: no work list for this P and precision yet "
                               "(make one fitness_eval call with them first)");
    if (!plan->twopass.empty())
        return fail(MT_EINVAL, "fitness_eval_noalloc: a structure needs the two-pass path");
    int dev = 0;
    HIPCHECK(hipGetDevice(&dev));
    if (dev != set->device) return fail(MT_EINVAL, "the set's device is not the current device");
    double* part = nullptr;
    TRY(scratch_of_device(dev, &part));
    hipStream_t st = (hipStream_t)stream;
    set->fit_P = 0;              // the set's own workspace does not hold these sums
    set->cur_x = x;
    set->cur_form = 0;
    TRY(launch_plan_fit(set, plan, cfg, precision, part, st));
    return launch_finalize_fit(set, P, w, Z, st, part);
}

int mt_profile_enable(mt_set* set, int enable) {
    if (!set) return fail(MT_EINVAL, "set is NULL");
    set->profiling = enable != 0;
    return MT_OK;
}

int mt_profile_fitness_kernels(mt_set* set, const double* x, int nx, int P, int precision, int reps,
                               double* ms, int64_t* launches, void* stream) {
    TRY(check_common(set, x, P, precision));
    if (nx != 6 && nx != 9) return fail(MT_EINVAL, "nx must be 6 (minimal) or 9 (Tersoff form)");
    if (reps <= 0) return fail(MT_EINVAL, "reps must be positive");
    if (!ms || !launches) return fail(MT_EINVAL, "ms and launches must not be NULL");
    if (!set->has_ref) return fail(MT_ENOREF, "no reference data attached to the set");
    TRY(ensure_workspace(set, P, kNVFit));
    set->fit_P = 0;
    set->cur_x = x;
    set->cur_form = nx == 9 ? 1 : 0;
    return time_batched_kernels(set, cfg_for(set, P, precision), P, precision, reps,
                                (hipStream_t)stream, ms, launches);
}

int mt_profile_fitness_launches(mt_set* set, const double* x, int nx, int P, int precision, int reps,
                                int max_launches, double* ms, int* coordination_class,
                                int* struct_launch, int* n_launches, void* stream) {
    TRY(check_common(set, x, P, precision));
    if (nx != 6 && nx != 9) return fail(MT_EINVAL, "nx must be 6 (minimal) or 9 (Tersoff form)");
    if (reps <= 0 || max_launches <= 0) return fail(MT_EINVAL, "reps and max_launches must be positive");
    if (!ms || !coordination_class || !n_launches) return fail(MT_EINVAL, "NULL output");
    if (!set->has_ref) return fail(MT_ENOREF, "no reference data attached to the set");
    TRY(ensure_workspace(set, P, kNVFit));
    set->fit_P = 0;
    set->cur_x = x;
    set->cur_form = nx == 9 ? 1 : 0;
    return time_class_launches(set, cfg_for(set, P, precision), P, precision, reps, (hipStream_t)stream,
                               max_launches, ms, coordination_class, struct_launch, n_launches);
}

int mt_profile_read(mt_set* set, double* ms, int64_t* launches) {
    if (!set || !ms || !launches) return fail(MT_EINVAL, "NULL argument");
    for (int k = 0; k < 2; ++k) {
        double tot = 0.0;
        for (auto& pr : set->prof_events[k]) {
            HIPCHECK(hipEventSynchronize(pr.second));
            float t = 0.f;
            HIPCHECK(hipEventElapsedTime(&t, pr.first, pr.second));
            tot += t;
            set->event_pool.push_back(pr.first);
            set->event_pool.push_back(pr.second);
        }
        ms[k] = tot;
        launches[k] = (int64_t)set->prof_events[k].size();
        set->prof_events[k].clear();
    }
    return MT_OK;
}

int mt_autotune(mt_set* set, int P, int precision, const char* cache_path) {
    if (!set) return fail(MT_EINVAL, "set is NULL");
    if (P <= 0) return fail(MT_EINVAL, "P must be positive");
    if (precision != MT_FP64 && precision != MT_FP32_ACC64)
        return fail(MT_EINVAL, "precision must be MT_FP64 or MT_FP32_ACC64");
    const int fam = precision == MT_FP64 ? FAM_FIT64 : FAM_FIT32;
    char key[200];
    snprintf(key, sizeof key, "N=%d S=%d nb=%d trip=%lld P=%d prec=%d", set->N, set->S, set->nb,
             set->ntrip, P, precision);
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            auto bar = line.find(" | ");
            if (bar == std::string::npos || line.substr(0, bar) != key) continue;
            LaunchCfg c;
            const int nread = sscanf(line.c_str() + bar + 3, "block=%d tile=%d persistent=%d graph=%d",
                                     &c.block, &c.tile, &c.persistent, &c.graph);
            // the batched kernels are compiled for at most 512 threads per
            // block, in whole wavefronts
            if (nread >= 3 && (c.block < 64 || c.block > 512 || c.block % 64 != 0 || c.tile < 0 ||
                               (c.persistent != 0 && c.persistent != 1) || (c.graph != 0 && c.graph != 1)))
                return fail(MT_EINVAL, "cache entry holds an invalid launch shape (block: a multiple of 64 "
                                       "up to 512; tile >= 0; persistent and graph 0 or 1)");
            if (nread >= 3 && get_plan(set, P, c, fam)) {
                set->tuned[{P, precision}] = c;
                clear_graphs(set);
                return MT_OK;
            }
        }
    }
    int maxpad = 8;
    for (int s = 0; s < set->S; ++s)
        if (!set->h_large[s]) maxpad = std::max(maxpad, set->h_npad[s]);
    std::vector<LaunchCfg> cands;
    for (int block : {64, 128, 256, 512}) {
        if (block < maxpad) continue;
        // powers of two plus tiles that let a whole generation fit in one
        // round of resident wavefronts for common population sizes
        for (int tile : {1, 2, 4, 8, 12, 16, 20, 24, 32, 40, 48, 64, 80, 128}) {
            if (tile > P && tile != 1) continue;
            for (int pers : {0, 1}) cands.push_back(LaunchCfg{block, tile, pers});
        }
    }
    if (cands.empty()) return fail(MT_EINVAL, "no batched structures to tune");
    // timing inputs: Table 2-like parameters for all candidates, zero references if none
    hipStream_t st;
    HIPCHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    DevBuf xb;
    HIPCHECK(xb.reserve(sizeof(double) * 6 * P));
    std::vector<double> hx(6 * (size_t)P);
    for (int c = 0; c < P; ++c) {
        const double base[6] = {3.21481, 1.43134, 2.23801, 0.282818, 0.602568, -0.641048};
        for (int k = 0; k < 6; ++k) hx[6 * c + k] = base[k] * (1.0 + 0.01 * ((c * 7 + k) % 5));
    }
    HIPCHECK(hipMemcpy(xb.p, hx.data(), sizeof(double) * hx.size(), hipMemcpyHostToDevice));
    if (!set->has_ref) {
        HIPCHECK(set->fref32.reserve(sizeof(float) * 3 * set->N));
        HIPCHECK(set->fref64.reserve(sizeof(double) * 3 * set->N));
        HIPCHECK(hipMemset(set->fref32.p, 0, sizeof(float) * 3 * set->N));
        HIPCHECK(hipMemset(set->fref64.p, 0, sizeof(double) * 3 * set->N));
    }
    int rc = ensure_workspace(set, P, kNVFit);
    if (rc) { (void)hipStreamDestroy(st); return rc; }
    set->fit_P = 0;
    set->cur_x = xb.as<double>();
    set->cur_form = 0;
    hipEvent_t e0, e1;
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    DevBuf zb;
    HIPCHECK(zb.reserve(sizeof(double) * 4 * (size_t)P));
    const double wt[3] = {1.0, 1.0, 1.0};
    float best = 1e30f;
    LaunchCfg bestc = cands[0];
    const bool have_ref = set->has_ref;
    auto saved = set->tuned.find({P, precision});
    const bool had = saved != set->tuned.end();
    const LaunchCfg prev = had ? saved->second : LaunchCfg{};
    for (const LaunchCfg& c : cands) {
        ItemPlan* plan = get_plan(set, P, c, fam);
        if (!plan) continue;
        size_t lds = 0;
        for (auto& cp : plan->cls) lds = std::max(lds, cp->lds);
        if (lds > 160 * 1024) continue;
        set->tuned[{P, precision}] = c;
        // one generation: batched kernel(s) and the finalize kernel
        auto gen = [&]() -> int {
            if (have_ref)
                return fitness_sequence(set, xb.as<double>(), 0, P, wt, precision, MT_BATCHED, zb.as<double>(), st);
            return launch_batched(set, c, P, precision, MODE_FIT, nullptr, nullptr, nullptr, st);
        };
        if (gen() != MT_OK) continue;
        float tmin = 1e30f;
        for (int r = 0; r < 3; ++r) {
            (void)hipEventRecord(e0, st);
            (void)gen();
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            tmin = std::min(tmin, ms);
        }
        if (tmin < best) { best = tmin; bestc = c; }
        if (cache_path) {
            std::ofstream logf(cache_path, std::ios::app);
            logf << "# " << key << " | block=" << c.block << " tile=" << c.tile << " persistent="
                 << c.persistent << " ms=" << tmin << "\n";
        }
    }
    // Graph replay or direct launches: what a caller sees is the rate of
    // back-to-back generations, host enqueue included, so time a burst of
    // calls from the host clock.
    if (have_ref) {
        float best_burst = 1e30f;
        int best_graph = 1;
        for (int g : {1, 0}) {
            LaunchCfg c = bestc;
            c.graph = g;
            set->tuned[{P, precision}] = c;
            clear_graphs(set);
            for (int r = 0; r < 3; ++r)
                (void)fitness_eval(set, xb.as<double>(), P, wt, precision, MT_BATCHED, zb.as<double>(), st);
            (void)hipStreamSynchronize(st);
            constexpr int kBurst = 50;
            const auto t0 = std::chrono::steady_clock::now();
            for (int r = 0; r < kBurst; ++r)
                (void)fitness_eval(set, xb.as<double>(), P, wt, precision, MT_BATCHED, zb.as<double>(), st);
            (void)hipStreamSynchronize(st);
            const float ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count() / kBurst;
            if (ms < best_burst) { best_burst = ms; best_graph = g; }
            if (cache_path) {
                std::ofstream logf(cache_path, std::ios::app);
                logf << "# " << key << " | block=" << c.block << " tile=" << c.tile << " persistent="
                     << c.persistent << " graph=" << g << " burst_ms=" << ms << "\n";
            }
        }
        bestc.graph = best_graph;
        clear_graphs(set);
    }
    if (had) set->tuned[{P, precision}] = prev; else set->tuned.erase({P, precision});
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return hip_fail(err, "autotune launches");
    set->tuned[{P, precision}] = bestc;
    clear_graphs(set);
    if (cache_path) {
        std::ofstream outf(cache_path, std::ios::app);
        outf << key << " | block=" << bestc.block << " tile=" << bestc.tile
             << " persistent=" << bestc.persistent << " graph=" << bestc.graph << " ms=" << best << "\n";
    }
    return MT_OK;
}

}  // extern "C"
