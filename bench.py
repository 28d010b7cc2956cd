#!/usr/bin/env python3
"""Throughput of the batched minimal-Tersoff GA fitness evaluation on one GPU.

A step is one GA generation's fitness evaluation: decode the population's
parameters, evaluate energy, forces and virial of every candidate on every
training structure, and reduce the weighted energy/virial/force relative-RMSE
fitness (Sec. III.B of the paper).  The neighbour lists and bond geometry are
built once per structure set (the cutoffs are fixed, not fitted) and are not
part of a step.

Before the W untimed warm-up steps the fitness workloads (headline, uneven,
Tersoff form) run for 0.25 s, so that the GPU has left its idle clock; the
timed region then holds exactly K steps.

Headline workload: 200 candidates x 100 strained 64-atom diamond Si cells,
float32 arithmetic with float64 accumulation; reference data from a hidden
parameter set evaluated by the library's float64 path.  The same run also
measures the plain schedule (one launch per candidate and structure), the
fitness gradient, uneven batching (500 candidates x 300 structures of 8-512
atoms), the gradient over those structures (64 candidates), GA generations
with gradient refinement over them, the GA batch with nine-parameter
Tersoff-form candidates and the 64,000-atom force call, and times
the CPU oracle on a bounded sample.  Prints
one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

FP32_VALU_PEAK_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz, non-packed
PACKED_FP32_PEAK_TFLOPS = 157.3  # the vendor's float32 vector figure, which counts packed FP32 (unused here)
# Launch shapes measured by mt_autotune on MI355X, keyed by set size and population.
TUNED_SHAPES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1909_11474_amd",
                            "tuned_shapes.txt")


# HBM traffic of the dominant kernel from two rocprofv3 --pmc passes (FETCH_SIZE,
# WRITE_SIZE; KiB per dispatch) scaled by what the same counters read for a
# 256 MiB device-to-device copy (FETCH_SIZE x 2.00, WRITE_SIZE x 1.00), recorded
# in profiles/k_batched_fit32_ga_batch_traffic.md.  Valid only for the kernel
# sources and the host file that places the work items (mt_eval.hip) it was
# measured on: reported when their hash still matches.
PMC_TRAFFIC = {
    "sources": ["paper_1909_11474_amd/csrc/mt_common.h", "paper_1909_11474_amd/csrc/mt_site.h",
                "paper_1909_11474_amd/csrc/mt_kernels.h", "paper_1909_11474_amd/csrc/mt_k_fit32.hip",
                "paper_1909_11474_amd/csrc/mt_eval.hip"],
    "sha256_16": "7f930986759f6a97",
    "fetch_bytes": 1969.3 * 1024 * 2.00,
    "write_bytes": 4250.0 * 1024 * 1.00,
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


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--grad-steps", type=int, default=10)
    ap.add_argument("--uneven-steps", type=int, default=10,
                    help="generations of the uneven-batching workload (0: skip)")
    ap.add_argument("--uneven-grad-steps", type=int, default=5,
                    help="gradient calls over the uneven structures (0: skip)")
    ap.add_argument("--md-steps", type=int, default=20,
                    help="64,000-atom force calls (0: skip)")
    ap.add_argument("--ga-generations", type=int, default=10,
                    help="GA generations with gradient refinement over the uneven set (0: skip)")
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


def make_set(api, torch, wl):
    """Set + float64 reference data of the hidden parameter set (per-atom energies
    and virials, forces), all resident in HBM."""
    t0 = time.perf_counter()
    ts = api.from_structures(wl.structs, R1=wl.R1, R2=wl.R2)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    ref = ts.tersoff_eval(wl.hidden_x[None], precision="fp64", forces=True, virial=True)
    n = torch.as_tensor(wl.structs.sizes().astype(np.float64), device=ref["E"].device)
    refs = (ref["E"][0] / n, ref["W"][0] / n[:, None], ref["F"][0])
    ts.attach_reference(*refs)
    return ts, refs, t_create


def set_flops(ts, n_atoms):
    """(algorithmic flops, transcendentals, kernel-formulation flops) of one
    candidate over the set, from each atom's coordination."""
    i, _, _ = ts.neighbors()
    M = np.bincount(i, minlength=n_atoms)
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
    as tuned); then the batched kernels' own time, two ways: an event pair
    around each launch (prof: summed ms, launches; each pair adds the dispatch
    and completion latency) and `steps` back-to-back passes of the kernels
    alone between one event pair on their stream (b2b: ms per pass, launches
    per pass)."""
    call = ts.fitness_call(X, Z, precision="fp32", schedule="batched")
    spin_up(torch, call)
    for _ in range(warmup):
        call()
    with Timer(torch) as t:
        for _ in range(steps):
            call()
    ts.profile(True)
    ts.profile_read()
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    prof = ts.profile_read()["batched"]
    ts.profile(False)
    b2b = ts.profile_fitness_kernels(X, "fp32", steps)
    # per-generation times (an event pair around each call), for the median
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(max(20, min(steps, 200)))]
    for a, b in ev:
        a.record()
        call()
        b.record()
    torch.cuda.synchronize()
    t.median_ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
    return t, prof, b2b


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


def oracle_rate(args, torch, wl, refs, grad: bool):
    """The CPU oracle's fitness (or fitness-gradient) rate over a workload's
    structures, in atom*candidate evals/s, on a third of the CPU budget."""
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
    done, tc = oracle_sample(lambda X: fn(s, X, r, topology=top), wl.population, args.cpu_seconds / 3)
    what = "fitness and dZ/dx" if grad else "fitness"
    out = {"value": done * s.n_atoms / tc,
           "unit": "atom·candidate fitness-grad evals/s" if grad else "atom·candidate evals/s",
           "cores": int(torch.get_num_threads()), "kind": "oracle",
           "sample": f"{done} candidate evaluations of the {what} x all {s.n_struct} structures "
                     f"({s.n_atoms} atoms) in {tc:.1f} s, float64 autograd",
           "setup_s": {"topology": t_top}}
    log(f"cpu oracle ({what}, {wl.name.split(':')[0]}): {out['value']:.4e} atom*cand/s")
    return out


def uneven_batching(args, api, torch, W, dev):
    wl = W.config3()
    s = wl.structs
    P = wl.population.shape[0]
    log(f"workload: {wl.name}; atoms {s.n_atoms}, population {P}")
    ts, refs, t_create = make_set(api, torch, wl)
    st = ts.stats()
    flop_cand, _, _ = set_flops(ts, s.n_atoms)
    X = torch.as_tensor(wl.population, dtype=torch.float64, device=dev).contiguous()
    Z = torch.empty(P, 4, dtype=torch.float64, device=dev)
    t0 = time.perf_counter()
    if not args.no_tune:
        ts.autotune(P, "fp32", args.tune_cache)
    t_tune = time.perf_counter() - t0
    t, prof, b2b = time_generations(torch, ts, X, Z, args.uneven_steps, 2)
    units = P * s.n_atoms
    kernel_ms = b2b[0]
    out = {"workload": wl.name, "value": units * args.uneven_steps / t.seconds,
           "unit": "atom·candidate evals/s", "ms_per_step": t.seconds / args.uneven_steps * 1e3,
           "steps": args.uneven_steps, "atoms": s.n_atoms, "structures": s.n_struct,
           "bonds": st["n_bonds"], "triplets": st["n_triplets"], "population": P,
           "batched_kernels_ms_per_step": kernel_ms,
           "batched_launches_per_step": b2b[1],
           "batched_kernels_ms_per_step_event_pair_per_launch": prof[0] / args.uneven_steps,
           "algorithmic_tflops": flop_cand * P / (kernel_ms * 1e-3) / 1e12,
           "setup_ms": {"set_create": t_create * 1e3, "autotune": t_tune * 1e3},
           "seeds": wl.seeds}
    log(f"uneven batched: {out['ms_per_step']:.3f} ms/generation, {out['value']:.4e} atom*cand/s, "
        f"kernels {kernel_ms:.3f} ms ({out['algorithmic_tflops']:.2f} TFLOP/s)")
    if args.plain_steps > 0:
        tp = time_plain(torch, ts, X, Z, args.plain_steps)
        out["plain"] = {"value": units * args.plain_steps / tp.seconds,
                        "ms_per_step": tp.seconds / args.plain_steps * 1e3,
                        "launches_per_step": P * s.n_struct}
        log(f"uneven plain: {out['plain']['ms_per_step']:.1f} ms/generation")
    ts.close()
    if not args.no_cpu_baseline:
        out["cpu_oracle"] = oracle_rate(args, torch, wl, refs, grad=False)
    return out


def uneven_gradient(args, api, torch, W, dev):
    wl = W.config4()
    s = wl.structs
    P = wl.population.shape[0]
    ts, refs, _ = make_set(api, torch, wl)
    X = torch.as_tensor(wl.population, dtype=torch.float64, device=dev).contiguous()
    if not args.no_tune:
        ts.autotune(P, "fp32", args.tune_cache)
    t = time_grad(torch, ts, X, args.uneven_grad_steps)
    out = {"workload": wl.name, "value": P * s.n_atoms * args.uneven_grad_steps / t.seconds,
           "unit": "atom·candidate fitness-grad evals/s",
           "ms_per_step": t.seconds / args.uneven_grad_steps * 1e3,
           "steps": args.uneven_grad_steps, "population": P, "seeds": wl.seeds}
    log(f"uneven gradient: {out['ms_per_step']:.3f} ms/call, {out['value']:.4e} atom*cand/s")
    ts.close()
    if not args.no_cpu_baseline:
        out["cpu_oracle"] = oracle_rate(args, torch, wl, refs, grad=True)
    return out


def ga_generations(args, api, torch, W, dev):
    """The host GA (Sec. III.B) on the GPU fitness over the uneven structures,
    population 64, with projected-gradient refinement of the best 8 each
    generation: wall time per generation (fitness, sort, refinement with its
    gradient and trial fitness, selection, crossover, mutation)."""
    from paper_1909_11474_amd import ga as G
    wl = W.config4()
    P = wl.population.shape[0]
    ts, _, _ = make_set(api, torch, wl)
    if not args.no_tune:
        ts.autotune(P, "fp32", args.tune_cache)
    fit, grad = G.gpu_fitness(ts, precision="fp32")
    cfg = G.GAConfig(pop=P, n_par=P // 2, n_gen=500, seed=wl.seeds["population"],
                     refine_top=8, refine_steps=1)
    ga = G.GA(cfg, fit, grad)
    ga.step()                                              # warm-up: plans for P and 8
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.ga_generations):
        rec = ga.step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.ga_generations
    out = {"workload": wl.name + "; GA with top-8 gradient refinement",
           "ms_per_generation": dt * 1e3, "generations": args.ga_generations,
           "best_Z": rec["best"], "population": P}
    log(f"GA generation with refinement: {dt * 1e3:.3f} ms")
    ts.close()
    return out


def tersoff_form_batch(args, api, torch, W, dev):
    """The GA fitness batch with nine-parameter Tersoff-form candidates
    (fitness_eval_tf): same structures, population size and launch shape as the
    headline workload."""
    wl = W.config2_tersoff_form()
    s = wl.structs
    P = wl.population.shape[0]
    ts, _, _ = make_set(api, torch, wl)
    X = torch.as_tensor(wl.population, dtype=torch.float64, device=dev).contiguous()
    Z = torch.empty(P, 4, dtype=torch.float64, device=dev)
    if not args.no_tune:
        ts.autotune(P, "fp32", args.tune_cache)          # shape shared with the minimal form
    t, prof, b2b = time_generations(torch, ts, X, Z, args.tf_steps, 5)
    kernel_ms = b2b[0] / max(b2b[1], 1)
    out = {"workload": wl.name, "value": P * s.n_atoms * args.tf_steps / t.seconds,
           "unit": "atom·candidate evals/s", "ms_per_step": t.seconds / args.tf_steps * 1e3,
           "steps": args.tf_steps, "population": P, "batched_kernel_ms": kernel_ms,
           "seeds": wl.seeds}
    log(f"Tersoff form batched: {out['ms_per_step']:.4f} ms/generation, {out['value']:.4e} "
        f"atom*cand/s, kernel {kernel_ms:.4f} ms")
    if args.grad_steps > 0:
        tg = time_grad(torch, ts, X, args.grad_steps)
        out["fitness_grad"] = {"value": P * s.n_atoms * args.grad_steps / tg.seconds,
                               "unit": "atom·candidate fitness-grad evals/s (9 parameters)",
                               "ms_per_step": tg.seconds / args.grad_steps * 1e3}
        log(f"Tersoff form fitness_grad: {out['fitness_grad']['ms_per_step']:.3f} ms/generation")
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
        out[prec] = {"ms_per_call": t.seconds / args.md_steps * 1e3,
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

    wl = W.config2()
    s = wl.structs
    P = wl.population.shape[0]
    log(f"workload: {wl.name}; atoms {s.n_atoms}, structures {s.n_struct}, population {P}")
    ts, (e_ref, w_ref, f_ref), t_create = make_set(api, torch, wl)
    st = ts.stats()
    log("set:", st, f"created in {t_create * 1e3:.1f} ms")
    flop_cand, trans_cand, kflop_cand = set_flops(ts, s.n_atoms)
    flop_launch = flop_cand * P

    X = torch.as_tensor(wl.population, dtype=torch.float64, device=dev).contiguous()
    Z = torch.empty(P, 4, dtype=torch.float64, device=dev)
    t0 = time.perf_counter()
    if not args.no_tune:
        ts.autotune(P, "fp32", args.tune_cache)
    t_tune = time.perf_counter() - t0

    # ---- timed region: K generations; then the kernel alone -----------------
    t, prof, b2b = time_generations(torch, ts, X, Z, args.steps, args.warmup)
    ms_step = t.seconds / args.steps * 1e3
    units = P * s.n_atoms
    value = units * args.steps / t.seconds
    log(f"batched: {ms_step:.4f} ms/generation, {value:.4e} atom*cand/s "
        f"(wall {t.wall * 1e3:.3f} ms, host enqueue {t.enqueue * 1e3:.3f} ms for {args.steps} generations)")
    kernel_ms = b2b[0] / max(b2b[1], 1)         # one launch per pass: every structure has M <= 4
    pair_ms = prof[0] / max(prof[1], 1)
    achieved = flop_launch / (kernel_ms * 1e-3) / 1e12
    kernel_tflops = kflop_cand * P / (kernel_ms * 1e-3) / 1e12
    log(f"batched kernel: {kernel_ms:.4f} ms/launch over {args.steps} back-to-back launches "
        f"({pair_ms:.4f} ms with an event pair around each), "
        f"{achieved:.2f} TFLOP/s algorithmic, {kernel_tflops:.2f} TFLOP/s in the kernel's formulation")
    Zb = Z.clone()

    plain = None
    if args.plain_steps > 0:
        tp = time_plain(torch, ts, X, Z, args.plain_steps)
        plain = {"value": units * args.plain_steps / tp.seconds,
                 "ms_per_step": tp.seconds / args.plain_steps * 1e3,
                 "launches_per_step": P * s.n_struct, "steps": args.plain_steps,
                 "max_abs_dZ_vs_batched": float((Z - Zb).abs().max())}
        log(f"plain: {plain['ms_per_step']:.2f} ms/generation, {plain['value']:.4e} atom*cand/s")

    grad = None
    if args.grad_steps > 0:
        tg = time_grad(torch, ts, X, args.grad_steps)
        grad = {"value": units * args.grad_steps / tg.seconds,
                "unit": "atom·candidate fitness-grad evals/s",
                "ms_per_step": tg.seconds / args.grad_steps * 1e3, "steps": args.grad_steps}
        log(f"fitness_grad: {grad['ms_per_step']:.3f} ms/generation, {grad['value']:.4e} atom*cand/s")

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: 3 x {args.copy_probe_mib} MiB device-to-device")
        del src, dst

    # ---- CPU oracle on a bounded sample --------------------------------------
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import tersoff as T
        refs = {"e": e_ref.cpu().numpy(), "w": w_ref.cpu().numpy(), "f": f_ref.cpu().numpy()}
        top = T.topology(s, wl.R2)
        T.fitness(s, wl.population[:1], refs, topology=top)           # warm-up
        def sample(seconds):
            return oracle_sample(lambda X: T.fitness(s, X, refs, topology=top), wl.population, seconds)

        done, tc = sample(args.cpu_seconds)
        cpu = {"value": done * s.n_atoms / tc, "unit": "atom·candidate evals/s",
               "cores": int(torch.get_num_threads()), "kind": "oracle",
               "sample": f"{done} candidate evaluations (population of {P}, in order, wrapping) x "
                         f"all {s.n_struct} structures = {done * s.n_atoms} atom*candidate evals "
                         f"in {tc:.1f} s, float64 autograd",
               "host": {"nproc": os.cpu_count(), "cpu_model": cpu_model()}}
        log(f"cpu oracle: {cpu['value']:.4e} atom*cand/s on {cpu['cores']} threads")
        # the same oracle on one thread (a third of the budget)
        threads = torch.get_num_threads()
        torch.set_num_threads(1)
        try:
            done1, tc1 = sample(args.cpu_seconds / 3)
        finally:
            torch.set_num_threads(threads)
        cpu["one_thread"] = {"value": done1 * s.n_atoms / tc1, "cores": 1,
                             "sample": f"{done1} candidate evaluations in {tc1:.1f} s"}
        log(f"cpu oracle, one thread: {cpu['one_thread']['value']:.4e} atom*cand/s")
    ts.close()

    workloads = {}
    if args.uneven_steps > 0:
        workloads["uneven_batching"] = uneven_batching(args, api, torch, W, dev)
    if args.uneven_grad_steps > 0:
        workloads["uneven_gradient"] = uneven_gradient(args, api, torch, W, dev)
    if cpu is not None:
        # the oracle on the uneven structures too (fitness, and fitness with its gradient)
        cpu["workloads"] = {k: v["cpu_oracle"] for k, v in workloads.items() if "cpu_oracle" in v}
    if args.md_steps > 0:
        workloads["force_call_64k"] = force_call(args, api, torch, W, dev)
    if args.ga_generations > 0:
        workloads["ga_refined"] = ga_generations(args, api, torch, W, dev)
    if args.tf_steps > 0:
        workloads["tersoff_form"] = tersoff_form_batch(args, api, torch, W, dev)
    if not args.no_properties:
        workloads["properties_0K"] = zero_kelvin_properties(torch, W)
    if args.md_run_steps > 0:
        workloads["md_hnemd_8000"] = md_run(args, torch, W)

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
                   "precision": "f32 arithmetic, f64 accumulation", "schedule": "batched",
                   "parallelism": "single GPU", "seeds": wl.seeds},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VALU_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_VALU_PEAK_TFLOPS,
                     "traffic": measured_traffic()},
        "kernel": {"name": "k_batched<float, fit, M<=4>", "avg_ms": kernel_ms, "launches": args.steps,
                   "timing": "back-to-back launches between one HIP event pair on the kernel's stream",
                   "avg_ms_event_pair_per_launch": pair_ms,
                   "flop_per_launch": flop_launch, "transcendentals_per_launch": trans_cand * P,
                   "formulation_flop_per_launch": kflop_cand * P,
                   "formulation_tflops": kernel_tflops,
                   "formulation_frac": kernel_tflops / FP32_VALU_PEAK_TFLOPS,
                   "packed_fp32_peak": PACKED_FP32_PEAK_TFLOPS,
                   "frac_of_packed_fp32_peak": achieved / PACKED_FP32_PEAK_TFLOPS},
        "host_enqueue_ms_per_step": t.enqueue / args.steps * 1e3,
        "plain": plain,
        "fitness_grad": grad,
        "workloads": workloads,
        "cpu_baseline": cpu,
        "setup_ms": {"set_create": t_create * 1e3, "autotune": t_tune * 1e3},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
