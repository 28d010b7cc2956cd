#!/usr/bin/env python3
"""Throughput of the batched minimal-Tersoff GA fitness evaluation on one GPU.

A step is one GA generation's fitness evaluation: decode the population's
parameters, evaluate energy, forces and virial of every candidate on every
training structure, and reduce the weighted energy/virial/force relative-RMSE
fitness (Sec. III.B of the paper).  The neighbour lists and bond geometry are
built once per structure set (the cutoffs are fixed, not fitted) and are not
part of a step.

Headline workload: uneven batching, 500 candidates x 300 structures of 8-512
atoms (strained diamond supercells, the same with vacancies, random
packings), float32 arithmetic with float64 accumulation and float64 energy
terms; reference data of a hidden parameter set written by the float64 oracle
(tests/golden/make_references.py).  Before the W untimed warm-up steps the
workload runs for 0.25 s, so that the GPU has left its idle clock; the timed
region holds exactly K steps.  The roofline block is that of the dominant
kernel (the launch of the largest coordination class), timed over
back-to-back launches of it alone.

The same run measures the uneven set in the specified launch form (one
persistent launch per class, graph replay) beside the tuned one, the plain
schedule (one launch per candidate and structure), the GA batch (200
candidates x 100 strained 64-atom cells), the fitness gradient (64 candidates
over the uneven set), the GA with top-8 gradient refinement against the plain
GA for 500 generations, the nine-parameter Tersoff form, the 64,000-atom force
call, the 0 K property layer and HNEMD, and times the CPU oracle (the plain C
reference, and the autograd one beside it) on a bounded
sample.  Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

FP32_PEAK_TFLOPS = 157.3         # MI355X published float32 vector peak (counts packed FP32)
FP32_NONPACKED_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz, non-packed
FP64_PEAK_TFLOPS = 78.6          # MI355X published float64 vector peak
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden")
# Launch shapes measured by mt_autotune on MI355X, keyed by set size and population.
TUNED_SHAPES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1909_11474_amd",
                            "tuned_shapes.txt")


# HBM traffic of the dominant kernel (k_batched<float, fit, M<=12> of the
# uneven workload) from two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE; KiB
# per dispatch) scaled by what the same counters read for a 256 MiB
# device-to-device copy (FETCH_SIZE x 2.00, WRITE_SIZE x 1.00), recorded in
# profiles/k_batched_fit32_uneven_500x300.md.  Valid only for the kernel sources,
# the host file that places the work items (mt_eval.hip) and the build script
# (per-unit code-generation flags) it was measured on: reported when their hash
# still matches.
PMC_TRAFFIC = {
    "sources": ["paper_1909_11474_amd/csrc/mt_common.h", "paper_1909_11474_amd/csrc/mt_site.h",
                "paper_1909_11474_amd/csrc/mt_kernels.h", "paper_1909_11474_amd/csrc/mt_k_fit32.hip",
                "paper_1909_11474_amd/csrc/mt_eval.hip", "paper_1909_11474_amd/build.py"],
    "sha256_16": "514a5b8796fceaa5",
    "fetch_bytes": 38379.6 * 1024 * 2.00,
    "write_bytes": 23094.7 * 1024 * 1.00,
}


def measured_traffic():
    """Bytes per launch of the dominant kernel from the counter passes, or None
    if its sources changed since they were taken."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in PMC_TRAFFIC["sources"]:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != PMC_TRAFFIC["sha256_16"]:
        return None
    return PMC_TRAFFIC["fetch_bytes"] + PMC_TRAFFIC["write_bytes"]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def flops_per_atom(M: np.ndarray) -> np.ndarray:
    """Algorithmic flops of one atom for one candidate (FMA = 2, transcendentals
    counted separately): the plain chain-rule formulation of energy, forces and
    virial, 44 per directed pair (10 forward, 34 backward) and 55 per ordered
    triplet (5 forward, 50 backward); 836 for a diamond atom (M = 4)."""
    M = np.asarray(M, dtype=np.int64)
    return 44 * M + 55 * M * (M - 1)


def kernel_flops_per_atom(M: np.ndarray) -> np.ndarray:
    """Flops the batched kernel's own formulation issues per atom and candidate
    (FMA = 2, each transcendental = 1): 31 per unordered bond pair (zeta
    forward 6, gradient backward 25: cos(theta) once per pair, the radial part
    through u_j . V_j), 70 per bond (pair terms, bond order with 6
    transcendentals, gradient assembly, force exchange, virial) and 9 per atom
    (site energy, force residual); 475 for a diamond atom."""
    M = np.asarray(M, dtype=np.int64)
    return 31 * (M * (M - 1) // 2) + 70 * M + 9


def grad_flops_per_atom(M: np.ndarray) -> np.ndarray:
    """Algorithmic flops of the fitness gradient per atom and candidate, a
    forward-mode model of the chain rule: the forward fitness work plus, for
    each of the six parameter directions, the directional derivative of the
    energy, force and virial work at twice its flops (each product a b needs
    a db + b da), plus the contraction of each bond gradient's six
    derivatives with its residual direction (6 x 3 FMA per bond):
    13 x flops_per_atom + 36 M; 11,012 for a diamond atom."""
    M = np.asarray(M, dtype=np.int64)
    return 13 * flops_per_atom(M) + 36 * M


def force_call_flops_per_atom(M: np.ndarray) -> np.ndarray:
    """Flops of the MD-scale force call per atom: energy, forces and virial
    (flops_per_atom), the per-atom virial (9 FMA per bond) and the heat-current
    term W_i v_i (9 FMA); 926 for a diamond atom."""
    M = np.asarray(M, dtype=np.int64)
    return flops_per_atom(M) + 18 * M + 18


# Algorithmic HBM bytes of the force call per atom: positions and velocities
# read (float64, 24 B each), forces (24 B) and per-atom virial (72 B) written.
FORCE_CALL_BYTES_PER_ATOM = 24 + 24 + 24 + 72


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100,
                    help="timed generations of the headline (uneven) workload")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--ga-batch-steps", type=int, default=200,
                    help="generations of the GA batch (200 x 100 x 64 atoms; 0: skip)")
    ap.add_argument("--grad-steps", type=int, default=10,
                    help="gradient calls on the GA batch (0: skip)")
    ap.add_argument("--specified-steps", type=int, default=50,
                    help="generations of the uneven workload in the specified launch form (0: skip)")
    ap.add_argument("--uneven-grad-steps", type=int, default=10,
                    help="gradient calls over the uneven structures (0: skip)")
    ap.add_argument("--md-steps", type=int, default=20,
                    help="64,000-atom force calls (0: skip)")
    ap.add_argument("--ga-generations", type=int, default=500,
                    help="generations of the refined-vs-plain GA comparison over the uneven set (0: skip)")
    ap.add_argument("--tf-steps", type=int, default=50,
                    help="generations of the Tersoff-form (9-parameter) GA batch (0: skip)")
    ap.add_argument("--md-run-steps", type=int, default=200,
                    help="HNEMD steps of an 8,000-atom diamond cell at 300 K (0: skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run three device-to-device copies of this many MiB after the headline "
                         "(the reference kernel that scales FETCH_SIZE/WRITE_SIZE counters to bytes)")
    ap.add_argument("--no-properties", action="store_true",
                    help="skip timing the 0 K property layer (lattice constant, elastic constants, phonons)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="wall-time budget of the CPU-oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tune-cache", default=TUNED_SHAPES,
                    help="autotune cache file: reuse a stored launch shape, or tune and append one")
    return ap.parse_args()


class Timer:
    """HIP events on the current stream around a region."""

    def __init__(self, torch):
        self.torch = torch
        self.e0 = torch.cuda.Event(enable_timing=True)
        self.e1 = torch.cuda.Event(enable_timing=True)

    def __enter__(self):
        self.torch.cuda.synchronize()
        self.w0 = time.perf_counter()
        self.e0.record()
        return self

    def __exit__(self, *exc):
        self.e1.record()
        self.enqueue = time.perf_counter() - self.w0
        self.torch.cuda.synchronize()
        self.wall = time.perf_counter() - self.w0
        self.seconds = self.e0.elapsed_time(self.e1) / 1e3


REFERENCE_FILES = {"config2": "references_ga_batch.npz", "config3": "references_uneven.npz"}


def load_references(wl, key):
    """The float64 oracle's reference data of the workload's hidden parameter
    set, as written by tests/golden/make_references.py; checked against the
    workload's seeds, hidden parameters and sizes."""
    d = np.load(os.path.join(GOLDEN, REFERENCE_FILES[key]), allow_pickle=False)
    s = wl.structs
    ok = (np.array_equal(d["sizes"], s.sizes()) and np.array_equal(d["hidden_x"], wl.hidden_x)
          and int(d["seeds"][0]) == wl.seeds["structures"] and int(d["seeds"][1]) == wl.seeds["hidden"])
    if not ok:
        raise SystemExit(f"{REFERENCE_FILES[key]} does not belong to {wl.name}: "
                         "rerun tests/golden/make_references.py")
    return d["e"], d["w"], d["f"]


def make_set(api, torch, wl, key):
    """Set + the oracle's reference data (per-atom energies and virials,
    forces), all resident in HBM."""
    t0 = time.perf_counter()
    ts = api.from_structures(wl.structs, R1=wl.R1, R2=wl.R2)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    e, w, f = load_references(wl, key)
    ts.attach_reference(e, w, f)
    dev = ts.device
    refs = tuple(torch.as_tensor(a, device=dev) for a in (e, w, f))
    return ts, refs, t_create


def coordination(ts, n_atoms):
    i, _, _ = ts.neighbors()
    return np.bincount(i, minlength=n_atoms)


def set_flops(ts, n_atoms):
    """(algorithmic flops, transcendentals, kernel-formulation flops) of one
    candidate over the set, from each atom's coordination."""
    M = coordination(ts, n_atoms)
    return float(flops_per_atom(M).sum()), float(6 * M.sum()), float(kernel_flops_per_atom(M).sum())


def spin_up(torch, call, seconds=0.25):
    """Run `call` untimed for `seconds` so that the GPU leaves its idle clock
    before the warm-up steps: a few milliseconds of work (the default warm-up)
    leave the clock ramping, and a generation measured then takes ~7 % longer."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(50):
            call()
        torch.cuda.synchronize()


def time_generations(torch, ts, X, Z, steps, warmup):
    """GPU time of `steps` back-to-back fitness_eval calls (graph replay or direct,
    as tuned); the batched kernels' own time over `steps` back-to-back passes
    between one event pair on their stream (ms per pass, launches per pass); and
    the median of generations each bracketed by its own event pair."""
    call = ts.fitness_call(X, Z, precision="fp32", schedule="batched")
    spin_up(torch, call)
    for _ in range(warmup):
        call()
    with Timer(torch) as t:
        for _ in range(steps):
            call()
    b2b = ts.profile_fitness_kernels(X, "fp32", steps)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(max(20, min(steps, 200)))]
    for a, b in ev:
        a.record()
        call()
        b.record()
    torch.cuda.synchronize()
    t.median_ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
    return t, b2b


def dominant_launch(ts, X, M, sizes, P, reps):
    """The launch of the batched fitness plan that takes longest, timed alone
    over `reps` back-to-back launches: its algorithmic flops (P candidates over
    its structures), ms and coordination class, and every launch's figures."""
    launches, struct_launch = ts.profile_fitness_launches(X, "fp32", reps)
    owner = np.repeat(np.arange(len(sizes)), sizes)
    per_atom = flops_per_atom(M)
    out = []
    for k, (ms, mc) in enumerate(launches):
        structs = [s for s, l in enumerate(struct_launch) if l == k]
        atoms = np.isin(owner, structs)
        flop = float(per_atom[atoms].sum()) * P
        out.append({"launch": k, "coordination_class": mc, "structures": len(structs),
                    "atoms": int(atoms.sum()), "avg_ms": ms, "flop_per_launch": flop,
                    "tflops": flop / (ms * 1e-3) / 1e12})
    dom = max(out, key=lambda r: r["avg_ms"])
    return dom, out


def fp32_roofline(flop, ms):
    achieved = flop / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS,
            "peak_nonpacked": FP32_NONPACKED_TFLOPS, "frac_nonpacked": achieved / FP32_NONPACKED_TFLOPS}


def time_plain(torch, ts, X, Z, steps):
    ts.fitness(X, precision="fp32", schedule="plain", out=Z)
    with Timer(torch) as t:
        for _ in range(steps):
            ts.fitness(X, precision="fp32", schedule="plain", out=Z)
    return t


def time_grad(torch, ts, X, steps):
    ts.fitness_grad(X, precision="fp32")
    with Timer(torch) as t:
        for _ in range(steps):
            ts.fitness_grad(X, precision="fp32")
    return t


def oracle_sample(call, population, seconds):
    """Time the CPU oracle on a bounded sample: call(X) on one candidate at a
    time, in population order and wrapping round, until `seconds` are spent.
    Returns (candidate evaluations, seconds)."""
    P = population.shape[0]
    done = 0
    c0 = time.perf_counter()
    while done == 0 or time.perf_counter() - c0 < seconds:
        k = done % P
        call(population[k:k + 1])
        done += 1
    return done, time.perf_counter() - c0


_ORACLE_TOPOLOGY = {}


def oracle_rate(args, torch, wl, refs, grad: bool, seconds=None):
    """The CPU oracle's fitness (or fitness-gradient) rate over a workload's
    structures, in atom*candidate evals/s, on `seconds` (default a third of the
    CPU budget) of candidate evaluations."""
    from oracle import tersoff as T
    s = wl.structs
    r = {"e": refs[0].cpu().numpy(), "w": refs[1].cpu().numpy(), "f": refs[2].cpu().numpy()}
    # the oracle's neighbour topology, built once per structure set (setup, not timed)
    key = (wl.seeds["structures"], s.n_struct, s.n_atoms, wl.R2)
    t0 = time.perf_counter()
    if key not in _ORACLE_TOPOLOGY:
        _ORACLE_TOPOLOGY[key] = T.topology(s, wl.R2)
    top = _ORACLE_TOPOLOGY[key]
    t_top = time.perf_counter() - t0
    fn = T.fitness_grad if grad else T.fitness
    fn(s, wl.population[:1], r, topology=top)                        # warm-up
    budget = args.cpu_seconds / 3 if seconds is None else seconds
    done, tc = oracle_sample(lambda X: fn(s, X, r, topology=top), wl.population, budget)
    what = "fitness and dZ/dx" if grad else "fitness"
    out = {"value": done * s.n_atoms / tc,
           "unit": "atom·candidate fitness-grad evals/s" if grad else "atom·candidate evals/s",
           "cores": int(torch.get_num_threads()), "kind": "oracle",
           "sample": f"{done} candidate evaluations of the {what} x all {s.n_struct} structures "
                     f"({s.n_atoms} atoms) in {tc:.1f} s, float64 autograd",
           "setup_s": {"topology": t_top}}
    log(f"cpu oracle ({what}, {wl.name.split(':')[0]}): {out['value']:.4e} atom*cand/s")
    return out


def c_oracle_rate(wl, refs, top, seconds, threads=0):
    """The plain C float64 reference's fitness rate (chain-rule forces, OpenMP
    over candidates) on the workload's structures: the population in chunks of
    64 candidates, wrapping round, until `seconds` are spent."""
    from oracle import c_oracle as C
    s = wl.structs
    r = {"e": refs[0].cpu().numpy(), "w": refs[1].cpu().numpy(), "f": refs[2].cpu().numpy()}
    ctop = C.CTopology(s, wl.R2, entries=(top.i, top.j, top.shift, top.sob))
    nt = threads or C.max_threads()
    X = wl.population
    P = X.shape[0]
    C.fitness(s, X[:1], r, topology=ctop, threads=nt)                 # warm-up
    done, k = 0, 0
    c0 = time.perf_counter()
    while done == 0 or time.perf_counter() - c0 < seconds:
        chunk = X[k:k + 64] if k + 64 <= P else np.concatenate([X[k:], X[:k + 64 - P]])
        C.fitness(s, chunk, r, topology=ctop, threads=nt)
        done += chunk.shape[0]
        k = (k + 64) % P
    tc = time.perf_counter() - c0
    return {"value": done * s.n_atoms / tc, "unit": "atom·candidate evals/s", "cores": int(nt),
            "kind": "oracle",
            "sample": f"{done} candidate evaluations of the fitness x all {s.n_struct} structures "
                      f"({s.n_atoms} atoms) in {tc:.1f} s, plain C float64 (oracle/tersoff_c.c: "
                      f"forces by the chain rule, OpenMP over candidates)"}


def cpu_baseline_headline(args, torch, wl, refs):
    """The oracle on the headline workload: the plain C reference on all host
    threads for the CPU budget and on one thread for a third of it, beside the
    autograd oracle (all threads, a third of the budget)."""
    from oracle import tersoff as T
    key = (wl.seeds["structures"], wl.structs.n_struct, wl.structs.n_atoms, wl.R2)
    t0 = time.perf_counter()
    if key not in _ORACLE_TOPOLOGY:
        _ORACLE_TOPOLOGY[key] = T.topology(wl.structs, wl.R2)
    t_top = time.perf_counter() - t0
    top = _ORACLE_TOPOLOGY[key]
    out = c_oracle_rate(wl, refs, top, args.cpu_seconds)
    out["setup_s"] = {"topology": t_top}
    out["host"] = {"nproc": os.cpu_count(), "cpu_model": cpu_model()}
    one = c_oracle_rate(wl, refs, top, args.cpu_seconds / 3, threads=1)
    out["one_thread"] = {"value": one["value"], "cores": 1, "sample": one["sample"]}
    out["autograd_oracle"] = oracle_rate(args, torch, wl, refs, grad=False, seconds=args.cpu_seconds / 3)
    log(f"cpu oracle (plain C, {out['cores']} threads): {out['value']:.4e} atom*cand/s; "
        f"one thread {one['value']:.4e}")
    return out


def uneven_specified_form(args, api, torch, W, dev, tuned):
    """The uneven workload in the launch form its specification names: one
    persistent launch per coordination class (static LPT bins over a fixed
    grid) replayed from a captured HIP graph, at the tuned block and tile, beside
    the tuned form."""
    import tempfile
    wl = W.config3()
    s = wl.structs
    P = wl.population.shape[0]
    ts, _, _ = make_set(api, torch, wl, "config3")
    st = ts.stats()
    key = (f"N={st['n_atoms']} S={st['n_struct']} nb={st['n_bonds']} trip={st['n_triplets']} "
           f"P={P} prec=1")
    with tempfile.TemporaryDirectory() as d:
        cache = os.path.join(d, "shape.txt")
        with open(cache, "w") as f:
            f.write(f"{key} | block={tuned['block']} tile={tuned['tile']} persistent=1 graph=1 ms=0\n")
        ts.autotune(P, "fp32", cache)
    X = torch.as_tensor(wl.population, dtype=torch.float64, device=dev).contiguous()
    Z = torch.empty(P, 4, dtype=torch.float64, device=dev)
    t, b2b = time_generations(torch, ts, X, Z, args.specified_steps, 2)
    out = {"workload": wl.name + "; one persistent launch per class, graph replay",
           "launch_shape": {"block": tuned["block"], "tile": tuned["tile"], "persistent": 1, "graph": 1},
           "value": P * s.n_atoms * args.specified_steps / t.seconds, "unit": "atom·candidate evals/s",
           "ms_per_step": t.seconds / args.specified_steps * 1e3, "steps": args.specified_steps,
           "batched_kernels_ms_per_step": b2b[0], "batched_launches_per_step": b2b[1]}
    log(f"uneven, persistent + graph: {out['ms_per_step']:.3f} ms/generation")
    ts.close()
    return out


def tuned_shape(path, ts, P):
    """The launch shape the cache file holds for this set and population."""
    st = ts.stats()
    key = (f"N={st['n_atoms']} S={st['n_struct']} nb={st['n_bonds']} trip={st['n_triplets']} "
           f"P={P} prec=1")
    shape = None
    if path and os.path.exists(path):
        with open(path) as f:
            for line in f:
                if line.startswith(key + " | "):
                    kv = dict(t.split("=") for t in line.split(" | ")[1].split())
                    shape = {k: float(v) if k == "ms" else int(v) for k, v in kv.items()}
    return shape


def ga_batch(args, api, torch, W, dev):
    """The GA fitness batch: 200 candidates x 100 strained 64-atom cells, one
    coordination class (one launch per generation)."""
    wl = W.config2()
    s = wl.structs
    P = wl.population.shape[0]
    ts, refs, t_create = make_set(api, torch, wl, "config2")
    flop_cand, trans_cand, kflop_cand = set_flops(ts, s.n_atoms)
    X = torch.as_tensor(wl.population, dtype=torch.float64, device=dev).contiguous()
    Z = torch.empty(P, 4, dtype=torch.float64, device=dev)
    if not args.no_tune:
        ts.autotune(P, "fp32", args.tune_cache)
    t, b2b = time_generations(torch, ts, X, Z, args.ga_batch_steps, args.warmup)
    kernel_ms = b2b[0] / max(b2b[1], 1)
    units = P * s.n_atoms
    out = {"workload": wl.name, "value": units * args.ga_batch_steps / t.seconds,
           "unit": "atom·candidate evals/s", "ms_per_step": t.seconds / args.ga_batch_steps * 1e3,
           "ms_per_step_median": t.median_ms, "steps": args.ga_batch_steps, "population": P,
           "atoms": s.n_atoms, "seeds": wl.seeds,
           "roofline": fp32_roofline(flop_cand * P, kernel_ms),
           "kernel": {"name": "k_batched<float, fit, M<=4>", "avg_ms": kernel_ms,
                      "flop_per_launch": flop_cand * P, "transcendentals_per_launch": trans_cand * P,
                      "formulation_flop_per_launch": kflop_cand * P},
           "setup_ms": {"set_create": t_create * 1e3}}
    log(f"GA batch: {out['ms_per_step']:.4f} ms/generation, kernel {kernel_ms * 1e3:.1f} us, "
        f"{out['roofline']['achieved']:.1f} TFLOP/s")
    Zb = Z.clone()
    if args.plain_steps > 0:
        tp = time_plain(torch, ts, X, Z, args.plain_steps)
        out["plain"] = {"value": units * args.plain_steps / tp.seconds,
                        "ms_per_step": tp.seconds / args.plain_steps * 1e3,
                        "launches_per_step": P * s.n_struct,
                        "max_abs_dZ_vs_batched": float((Z - Zb).abs().max())}
    if args.grad_steps > 0:
        tg = time_grad(torch, ts, X, args.grad_steps)
        out["fitness_grad"] = {"value": units * args.grad_steps / tg.seconds,
                               "unit": "atom·candidate fitness-grad evals/s",
                               "ms_per_step": tg.seconds / args.grad_steps * 1e3}
    ts.close()
    if not args.no_cpu_baseline:
        from oracle import tersoff as T
        key = (wl.seeds["structures"], wl.structs.n_struct, wl.structs.n_atoms, wl.R2)
        if key not in _ORACLE_TOPOLOGY:
            _ORACLE_TOPOLOGY[key] = T.topology(wl.structs, wl.R2)
        out["cpu_oracle"] = c_oracle_rate(wl, refs, _ORACLE_TOPOLOGY[key], args.cpu_seconds / 3)
        out["cpu_oracle"]["autograd_oracle"] = oracle_rate(args, torch, wl, refs, grad=False)
    return out


def copy_probe(torch, dev, mib):
    """Three device-to-device copies of `mib` MiB: the reference kernel whose
    FETCH_SIZE / WRITE_SIZE counters scale the counter passes to bytes."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy probe: 3 x {mib} MiB device-to-device")


def uneven_gradient(args, api, torch, W, dev):
    wl = W.config4()
    s = wl.structs
    P = wl.population.shape[0]
    ts, refs, _ = make_set(api, torch, wl, "config3")
    M = coordination(ts, s.n_atoms)
    X = torch.as_tensor(wl.population, dtype=torch.float64, device=dev).contiguous()
    if not args.no_tune:
        ts.autotune(P, "fp32", args.tune_cache)
    t = time_grad(torch, ts, X, args.uneven_grad_steps)
    ms = t.seconds / args.uneven_grad_steps * 1e3
    flop = float(grad_flops_per_atom(M).sum()) * P
    out = {"workload": wl.name, "value": P * s.n_atoms * args.uneven_grad_steps / t.seconds,
           "unit": "atom·candidate fitness-grad evals/s", "ms_per_step": ms,
           "steps": args.uneven_grad_steps, "population": P, "seeds": wl.seeds,
           "roofline": dict(fp32_roofline(flop, ms), timing="whole fitness_grad call (forward "
                            "fitness, coefficients, adjoint, finalize), events around back-to-back calls",
                            flop_model="13 x the forward algorithmic flops + 36 per bond (see grad_flops_per_atom)",
                            flop_per_call=flop)}
    log(f"uneven gradient: {ms:.3f} ms/call, {out['value']:.4e} atom*cand/s, "
        f"{out['roofline']['achieved']:.1f} TFLOP/s (model)")
    ts.close()
    if not args.no_cpu_baseline:
        out["cpu_oracle"] = oracle_rate(args, torch, wl, refs, grad=True)
    return out


def ga_judge(args, api, torch, W, dev):
    """The GA over the uneven set, population 64 (N_par 32, mutation 0.2 -> 0
    over the run): with projected-gradient refinement of the best 8 each
    generation against the plain GA from the same seed (the judge), for the
    configured number of generations; best Z every 50 generations and the wall
    time per generation of each."""
    from paper_1909_11474_amd import ga as G
    wl = W.config4()
    P = wl.population.shape[0]
    ts, _, _ = make_set(api, torch, wl, "config3")
    if not args.no_tune:
        ts.autotune(P, "fp32", args.tune_cache)
    fit, grad = G.gpu_fitness(ts, precision="fp32")
    n = args.ga_generations
    runs = {}
    for name, top in (("refined", 8), ("plain", 0)):
        cfg = G.GAConfig(pop=P, n_par=P // 2, n_gen=n, seed=wl.seeds["population"],
                         refine_top=top, refine_steps=1)
        ga = G.GA(cfg, fit, grad if top else None)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        curve = []
        for g in range(n):
            rec = ga.step()
            if g % 50 == 0 or g == n - 1:
                curve.append([g, rec["best"]])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        hist = [r["best"] for r in ga.history]
        runs[name] = {"best_Z_every_50": curve, "final_best_Z": hist[-1],
                      "monotone": all(b <= a for a, b in zip(hist, hist[1:])),
                      "ms_per_generation": dt / n * 1e3, "elite_x": ga.history[-1]["elite_x"]}
        log(f"GA {name}: best Z {hist[-1]:.6f} after {n} generations, {dt / n * 1e3:.3f} ms/generation")
    ts.close()
    return {"workload": wl.name + f"; GA {n} generations, top-8 gradient refinement vs plain GA, "
                                  f"seed {wl.seeds['population']}",
            "generations": n, "population": P, "refined": runs["refined"], "plain": runs["plain"],
            "refined_at_or_below_plain": runs["refined"]["final_best_Z"] <= runs["plain"]["final_best_Z"]}


def tersoff_form_batch(args, api, torch, W, dev):
    """The GA fitness batch with nine-parameter Tersoff-form candidates
    (fitness_eval_tf): same structures, population size and launch shape as the
    GA batch; reference data of a hidden nine-parameter set from the library's
    float64 path (the oracle's references are stored for the minimal form)."""
    wl = W.config2_tersoff_form()
    s = wl.structs
    P = wl.population.shape[0]
    ts = api.from_structures(s, R1=wl.R1, R2=wl.R2)
    ref = ts.tersoff_eval(wl.hidden_x[None], precision="fp64", forces=True, virial=True)
    n = torch.as_tensor(s.sizes().astype(np.float64), device=ref["E"].device)
    ts.attach_reference(ref["E"][0] / n, ref["W"][0] / n[:, None], ref["F"][0])
    X = torch.as_tensor(wl.population, dtype=torch.float64, device=dev).contiguous()
    Z = torch.empty(P, 4, dtype=torch.float64, device=dev)
    if not args.no_tune:
        ts.autotune(P, "fp32", args.tune_cache)          # shape shared with the minimal form
    t, b2b = time_generations(torch, ts, X, Z, args.tf_steps, 5)
    kernel_ms = b2b[0] / max(b2b[1], 1)
    out = {"workload": wl.name, "value": P * s.n_atoms * args.tf_steps / t.seconds,
           "unit": "atom·candidate evals/s", "ms_per_step": t.seconds / args.tf_steps * 1e3,
           "steps": args.tf_steps, "population": P, "batched_kernel_ms": kernel_ms,
           "seeds": wl.seeds}
    log(f"Tersoff form batched: {out['ms_per_step']:.4f} ms/generation, kernel {kernel_ms:.4f} ms")
    if args.grad_steps > 0:
        tg = time_grad(torch, ts, X, args.grad_steps)
        out["fitness_grad"] = {"value": P * s.n_atoms * args.grad_steps / tg.seconds,
                               "unit": "atom·candidate fitness-grad evals/s (9 parameters)",
                               "ms_per_step": tg.seconds / args.grad_steps * 1e3}
    ts.close()
    return out


def zero_kelvin_properties(torch, W):
    """Wall time of the 0 K property layer for the Table 2 parameters: lattice
    constant (two batched grids of 8-atom cells), elastic constants (strained
    cells and Newton steps of the internal shift), force constants (12 displaced
    216-atom supercells in one call) and a 200-point dispersion."""
    import numpy as np
    from paper_1909_11474_amd import properties as PR
    x = np.array(W.TABLE2_X)
    PR.lattice_constant(x)                                  # warm-up
    t = {}
    t0 = time.perf_counter()
    a0, e0 = PR.lattice_constant(x)
    t["lattice_constant_ms"] = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    ec = PR.elastic_constants(x, a0)
    t["elastic_constants_ms"] = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    phi, pos, cell = PR.force_constants(x, a0, n=3)
    q, _ = PR.dispersion_path(a0, per_segment=40)
    f = PR.frequencies(phi, pos, cell, q)
    t["phonons_ms"] = (time.perf_counter() - t0) * 1e3
    out = {"workload": "0 K properties of diamond Si, Table 2 parameters", **t,
           "a0_A": a0, "E_per_atom_eV": e0, "C11_GPa": ec["C11"], "C12_GPa": ec["C12"],
           "C44_GPa": ec["C44"], "optical_gamma_THz": float(f[0, 3])}
    log(f"0 K properties: a0 {a0:.6f} A, C11/C12/C44 {ec['C11']:.2f}/{ec['C12']:.2f}/{ec['C44']:.2f} GPa "
        f"in {t['lattice_constant_ms']:.1f} + {t['elastic_constants_ms']:.1f} + {t['phonons_ms']:.1f} ms")
    return out


def md_run(args, torch, W):
    """HNEMD of an 8,000-atom diamond cell (10 x 10 x 10 conventional cells,
    natural isotope masses, 300 K velocities, F_e = 1e-4 /A along z, 1 fs,
    0.5 A Verlet skin): velocity-Verlet steps per second, each with a position
    update (geometry, and the neighbour lists when an atom has moved 0.25 A),
    a float64 force call with per-atom virial and heat current, two kicks with
    the driving force and the kinetic sums."""
    import numpy as np
    from paper_1909_11474_amd import md as MDm
    g = np.random.Generator(np.random.PCG64(21))
    pos, cell = W.diamond(10, 10, 10)
    pos = W.displace(g, pos, 0.05)
    m = MDm.isotope_masses(pos.shape[0], g)
    v = g.normal(0.0, 1.0, size=pos.shape) * np.sqrt(W.KB_EV * 300.0 / (m[:, None] * W.AMU_A2_FS2_EV))
    v -= (m[:, None] * v).sum(0) / m.sum()
    md = MDm.MD(pos, cell, np.array(W.TABLE2_X), m, v, dt=1.0, fe=(0.0, 0.0, 1e-4), skin=0.5)
    md.run(10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r0 = md.rebuilds
    rec = md.run(args.md_run_steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    e = np.array([r["etot"] for r in rec])
    out = {"workload": "HNEMD, 8,000-atom diamond Si cell, 300 K, F_e = 1e-4 /A, dt = 1 fs, skin 0.5 A",
           "steps": args.md_run_steps, "steps_per_s": args.md_run_steps / dt,
           "ms_per_step": dt / args.md_run_steps * 1e3,
           "atom_steps_per_s": md.N * args.md_run_steps / dt,
           "T_mean_K": float(np.mean([r["T"] for r in rec])),
           "etot_drift_eV_per_atom": float((e[-1] - e[0]) / md.N),
           "neighbour_rebuilds": md.rebuilds - r0}
    log(f"MD (HNEMD) 8000 atoms: {out['ms_per_step']:.3f} ms/step, {out['atom_steps_per_s']:.3e} atom*steps/s")
    md.close()
    return out


def force_call(args, api, torch, W, dev):
    wl = W.config5()
    s = wl.structs
    t0 = time.perf_counter()
    ts = api.from_structures(s, R1=wl.R1, R2=wl.R2)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    vel = torch.as_tensor(wl.velocities, dtype=torch.float64, device=dev)
    M = coordination(ts, s.n_atoms)
    out = {"workload": wl.name, "atoms": s.n_atoms, "steps": args.md_steps,
           "outputs": "energy, forces, virial, per-atom virial, heat current",
           "set_create_ms": t_create * 1e3}
    for prec in ("fp32", "fp64"):
        call = ts.eval_call(wl.population, precision=prec, atom_virial=True, velocities=vel)
        call()
        with Timer(torch) as t:
            for _ in range(args.md_steps):
                call()
        # one call from an idle stream: host enqueue to completion
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        call()
        torch.cuda.synchronize()
        single = time.perf_counter() - t0
        ref = {k: v.clone() for k, v in call().items()}
        # 100 calls captured in one HIP graph (the work lists and buffers exist
        # before capture, and the evaluation path records no memset nodes)
        g = torch.cuda.CUDAGraph()
        cs = torch.cuda.Stream()
        cs.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(cs):
            call()
        torch.cuda.current_stream().wait_stream(cs)
        with torch.cuda.graph(g):
            for _ in range(100):
                call()
        g.replay()
        torch.cuda.synchronize()
        with Timer(torch) as tg:
            g.replay()
        same = all(torch.equal(v, ref[k]) for k, v in call().items())
        g.replay()
        torch.cuda.synchronize()
        same = same and all(torch.equal(v, ref[k]) for k, v in
                            {"E": call.E, "F": call.F.transpose(1, 2), "W": call.W}.items())
        ms = t.seconds / args.md_steps * 1e3
        flop = float(force_call_flops_per_atom(M).sum())
        nbytes = FORCE_CALL_BYTES_PER_ATOM * s.n_atoms
        gbs = nbytes / (ms * 1e-3) / 1e9
        tfl = flop / (ms * 1e-3) / 1e12
        peak = FP32_PEAK_TFLOPS if prec == "fp32" else FP64_PEAK_TFLOPS
        out[prec] = {"ms_per_call": ms,
                     "roofline": {"bound": "hbm" if gbs / HBM_PEAK_GBS > tfl / peak else "alu",
                                  "achieved_GBs": gbs, "peak_GBs": HBM_PEAK_GBS,
                                  "frac_hbm": gbs / HBM_PEAK_GBS, "achieved_TFLOPs": tfl,
                                  "peak_TFLOPs": peak, "frac_alu": tfl / peak,
                                  "bytes_per_call": nbytes, "flop_per_call": flop,
                                  "timing": "back-to-back calls (all kernels of a call), HIP events"},
                     "atoms_per_s": s.n_atoms * args.md_steps / t.seconds,
                     "single_call_ms": single * 1e3,
                     "graph_100_calls_ms_per_call": tg.seconds / 100 * 1e3 if same else None}
        log(f"64k force call {prec}: {out[prec]['ms_per_call']:.3f} ms/call back to back, "
            f"{single * 1e3:.3f} ms for one call, "
            f"{tg.seconds / 100 * 1e3:.3f} ms/call in a 100-call graph (replays {'match' if same else 'DIFFER'})")
        del g
    ts.close()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
                          "(population sharding across GPUs is a design note, not built)"}))
        sys.exit(2)
    import torch
    from paper_1909_11474_amd import api
    import workloads as W

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    # ---- headline: uneven batching, 500 candidates x 300 structures ----------
    wl = W.config3()
    s = wl.structs
    P = wl.population.shape[0]
    log(f"workload: {wl.name}; atoms {s.n_atoms}, structures {s.n_struct}, population {P}")
    ts, refs, t_create = make_set(api, torch, wl, "config3")
    st = ts.stats()
    M = coordination(ts, s.n_atoms)
    flop_cand = float(flops_per_atom(M).sum())
    X = torch.as_tensor(wl.population, dtype=torch.float64, device=dev).contiguous()
    Z = torch.empty(P, 4, dtype=torch.float64, device=dev)
    t0 = time.perf_counter()
    if not args.no_tune:
        ts.autotune(P, "fp32", args.tune_cache)
    t_tune = time.perf_counter() - t0
    shape = tuned_shape(args.tune_cache, ts, P) if not args.no_tune else None

    t, b2b = time_generations(torch, ts, X, Z, args.steps, args.warmup)
    ms_step = t.seconds / args.steps * 1e3
    units = P * s.n_atoms
    value = units * args.steps / t.seconds
    log(f"uneven batched: {ms_step:.4f} ms/generation, {value:.4e} atom*cand/s "
        f"(kernels {b2b[0]:.4f} ms back to back, {b2b[1]} launches)")
    dom, launches = dominant_launch(ts, X, M, s.sizes(), P, args.steps)
    log(f"dominant kernel: class M<={dom['coordination_class']}, {dom['avg_ms'] * 1e3:.1f} us/launch, "
        f"{dom['tflops']:.1f} TFLOP/s algorithmic")
    plain = None
    if args.plain_steps > 0:
        Zb = Z.clone()
        tp = time_plain(torch, ts, X, Z, args.plain_steps)
        plain = {"value": units * args.plain_steps / tp.seconds,
                 "ms_per_step": tp.seconds / args.plain_steps * 1e3,
                 "launches_per_step": P * s.n_struct, "steps": args.plain_steps,
                 "max_abs_dZ_vs_batched": float((Z - Zb).abs().max())}
        log(f"uneven plain: {plain['ms_per_step']:.1f} ms/generation")
    ts.close()
    if args.copy_probe_mib > 0:
        copy_probe(torch, dev, args.copy_probe_mib)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_headline(args, torch, wl, refs)

    workloads = {}
    if args.specified_steps > 0 and shape:
        workloads["uneven_specified_form"] = uneven_specified_form(args, api, torch, W, dev, shape)
    if args.ga_batch_steps > 0:
        workloads["ga_batch"] = ga_batch(args, api, torch, W, dev)
    if args.uneven_grad_steps > 0:
        workloads["uneven_gradient"] = uneven_gradient(args, api, torch, W, dev)
    if args.md_steps > 0:
        workloads["force_call_64k"] = force_call(args, api, torch, W, dev)
    if args.ga_generations > 0:
        workloads["ga_refined_vs_plain"] = ga_judge(args, api, torch, W, dev)
    if args.tf_steps > 0:
        workloads["tersoff_form"] = tersoff_form_batch(args, api, torch, W, dev)
    if not args.no_properties:
        workloads["properties_0K"] = zero_kelvin_properties(torch, W)
    if args.md_run_steps > 0:
        workloads["md_hnemd_8000"] = md_run(args, torch, W)
    if cpu is not None:
        cpu["workloads"] = {k: v["cpu_oracle"] for k, v in workloads.items() if "cpu_oracle" in v}

    line = {
        "metric": "atom·candidate Tersoff force evals/s and fitness-grad evals/s, batched vs plain",
        "value": value,
        "unit": "atom·candidate evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_median": t.median_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "population": P, "structures": s.n_struct,
                   "atoms": s.n_atoms, "bonds": st["n_bonds"], "triplets": st["n_triplets"],
                   "precision": "f32 arithmetic, f64 energy terms and accumulation",
                   "schedule": "batched", "launch_shape": shape, "parallelism": "single GPU",
                   "references": "float64 oracle, " + REFERENCE_FILES["config3"], "seeds": wl.seeds},
        "roofline": dict(fp32_roofline(dom["flop_per_launch"], dom["avg_ms"]),
                         traffic=measured_traffic()),
        "kernel": {"name": f"k_batched<float, fit, M<={dom['coordination_class']}>",
                   "avg_ms": dom["avg_ms"], "launches": args.steps,
                   "timing": "back-to-back launches of this kernel alone between one HIP event pair "
                             "on its stream",
                   "flop_per_launch": dom["flop_per_launch"], "structures": dom["structures"],
                   "atoms": dom["atoms"], "all_launches": launches,
                   "batched_kernels_ms_per_step": b2b[0], "batched_launches_per_step": b2b[1],
                   "algorithmic_flop_per_step": flop_cand * P,
                   "algorithmic_tflops_per_step": flop_cand * P / (b2b[0] * 1e-3) / 1e12},
        "host_enqueue_ms_per_step": t.enqueue / args.steps * 1e3,
        "plain": plain,
        "workloads": workloads,
        "cpu_baseline": cpu,
        "setup_ms": {"set_create": t_create * 1e3, "autotune": t_tune * 1e3},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
