"""Real-coded genetic algorithm driving the GPU fitness (paper Sec. III.B).

Each chromosome holds six genes in [0, 1]; gene k maps linearly onto the k-th
potential parameter between two limits.  One generation: evaluate Z for the
whole population (one batched GPU call), sort ascending (NaN last, ties by
index), keep the best individual unaltered, keep the best N_par as parents,
refill the population with children of uniform crossover between two distinct
random parents, then mutate every gene of every non-elite individual with
probability p_m(g) = p_m0 (1 - g / N_gen) to a fresh uniform draw.  The paper
uses N_pop = 200, N_par = 100, N_gen = 1000 and a mutation rate falling
linearly from 0.2 to zero.  The paper does not print the parameter limits, the
crossover operator, which individuals mutate or the tie rule; the choices here
are listed with the library's design notes.

Optional gradient refinement: after sorting, the best `refine_top` individuals
take projected gradient steps in gene space (dZ/dgene = dZ/dx (hi - lo), clipped
to [0, 1]); a step is kept only if it lowers Z, so the best Z never increases.
"""
from __future__ import annotations

import json
import time
from dataclasses import asdict, dataclass, field
from typing import Callable, Optional, Sequence

import numpy as np

# Parameter limits [D0 (eV), alpha (1/A), r0 (A), beta, n, h]; they contain the
# optimised values of Table 2 and keep every parameter of order unity.
DEFAULT_LO = (2.0, 1.0, 2.0, 0.1, 0.5, -1.0)
DEFAULT_HI = (5.0, 2.0, 2.6, 1.0, 1.5, 0.0)
# Limits for the nine-parameter Tersoff form [D0, alpha, r0, S, gamma, n, c, d, h]
# (fitness_eval_tf): the minimal box for the shared parameters, S in [1.5, 3],
# gamma in [0.05, 1], c and d in [0.5, 3].
TERSOFF_FORM_LO = (2.0, 1.0, 2.0, 1.5, 0.05, 0.5, 0.5, 0.5, -1.0)
TERSOFF_FORM_HI = (5.0, 2.0, 2.6, 3.0, 1.0, 1.5, 3.0, 3.0, 0.0)


@dataclass
class GAConfig:
    pop: int = 200
    n_par: int = 100
    n_gen: int = 1000
    mutation0: float = 0.2
    seed: int = 0
    lo: Sequence[float] = DEFAULT_LO
    hi: Sequence[float] = DEFAULT_HI
    refine_top: int = 0
    refine_steps: int = 1
    refine_step0: float = 0.02
    log_every: int = 1


def decode(genes: np.ndarray, lo: Sequence[float], hi: Sequence[float]) -> np.ndarray:
    """Genotype [P, n] in [0, 1] -> phenotype x = lo + g (hi - lo), n = len(lo)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return lo + np.asarray(genes, dtype=np.float64) * (hi - lo)


def sort_order(z: np.ndarray) -> np.ndarray:
    """Stable ascending order with NaN treated as +inf (ties keep index order)."""
    key = np.where(np.isnan(z), np.inf, z)
    return np.argsort(key, kind="stable")


class GA:
    """fitness(x [P,n] float64) -> Z [P]; grad(x [P,n]) -> (Z [P], dZ/dx [P,n]) for refinement;
    n = len(cfg.lo) genes (6 for the minimal potential, 9 for the Tersoff form)."""

    def __init__(self, cfg: GAConfig, fitness: Callable[[np.ndarray], np.ndarray],
                 grad: Optional[Callable[[np.ndarray], tuple]] = None):
        if not 1 <= cfg.n_par <= cfg.pop:
            raise ValueError("need 1 <= n_par <= pop")
        if cfg.n_par < 2 and cfg.pop > cfg.n_par:
            raise ValueError("crossover needs at least two parents")
        if cfg.refine_top and grad is None:
            raise ValueError("gradient refinement needs a gradient function")
        if len(cfg.lo) != len(cfg.hi):
            raise ValueError("lo and hi must have the same length")
        self.nx = len(cfg.lo)
        self.cfg = cfg
        self.fitness = fitness
        self.grad = grad
        self.rng = np.random.Generator(np.random.PCG64(cfg.seed))
        self.genes = self.rng.uniform(0.0, 1.0, size=(cfg.pop, self.nx))
        self.z = np.full(cfg.pop, np.nan)
        self.generation = 0
        self.step_size = np.full(cfg.pop, cfg.refine_step0)
        self.history = []

    # -- one generation ---------------------------------------------------------
    def evaluate(self) -> np.ndarray:
        z = np.asarray(self.fitness(decode(self.genes, self.cfg.lo, self.cfg.hi)), dtype=np.float64)
        if z.shape != (self.cfg.pop,):
            raise ValueError(f"fitness must return [{self.cfg.pop}], got {z.shape}")
        return z

    def refine(self):
        """Projected gradient steps for the best individuals (genes sorted)."""
        k = min(self.cfg.refine_top, self.cfg.pop)
        span = np.asarray(self.cfg.hi) - np.asarray(self.cfg.lo)
        for _ in range(self.cfg.refine_steps):
            g = self.genes[:k]
            z0, dzdx = self.grad(decode(g, self.cfg.lo, self.cfg.hi))
            z0 = np.asarray(z0, dtype=np.float64)
            dg = np.asarray(dzdx, dtype=np.float64) * span
            norm = np.linalg.norm(dg, axis=1, keepdims=True)
            norm[norm == 0] = 1.0
            trial = np.clip(g - self.step_size[:k, None] * dg / norm, 0.0, 1.0)
            zt = np.asarray(self.fitness_subset(trial), dtype=np.float64)
            ok = np.isfinite(zt) & (zt < z0)
            self.genes[:k][ok] = trial[ok]
            self.z[:k][ok] = zt[ok]
            self.step_size[:k] = np.where(ok, self.step_size[:k] * 1.5, self.step_size[:k] * 0.5)
        order = sort_order(self.z)
        self.genes = self.genes[order]
        self.z = self.z[order]
        self.step_size = self.step_size[order]

    def fitness_subset(self, genes: np.ndarray) -> np.ndarray:
        return self.fitness(decode(genes, self.cfg.lo, self.cfg.hi))

    def step(self) -> dict:
        cfg = self.cfg
        t0 = time.perf_counter()
        self.z = self.evaluate()
        order = sort_order(self.z)
        self.genes = self.genes[order]
        self.z = self.z[order]
        self.step_size = self.step_size[order]
        if cfg.refine_top:
            self.refine()
        record = {"generation": self.generation, "best": float(self.z[0]),
                  "median": float(np.median(np.where(np.isnan(self.z), np.inf, self.z))),
                  "elite_x": decode(self.genes[:1], cfg.lo, cfg.hi)[0].tolist()}
        # selection and crossover: children fill slots n_par .. pop-1
        n_child = cfg.pop - cfg.n_par
        if n_child > 0:
            pa = self.rng.integers(0, cfg.n_par, size=n_child)
            pb = self.rng.integers(0, cfg.n_par - 1, size=n_child)
            pb = pb + (pb >= pa)                            # a distinct second parent
            mask = self.rng.uniform(size=(n_child, self.nx)) < 0.5
            self.genes[cfg.n_par:] = np.where(mask, self.genes[pa], self.genes[pb])
            self.step_size[cfg.n_par:] = cfg.refine_step0
        # mutation of every non-elite individual
        pm = cfg.mutation0 * (1.0 - self.generation / cfg.n_gen)
        mut = self.rng.uniform(size=(cfg.pop - 1, self.nx)) < pm
        fresh = self.rng.uniform(size=(cfg.pop - 1, self.nx))
        self.genes[1:] = np.where(mut, fresh, self.genes[1:])
        self.generation += 1
        record["seconds"] = time.perf_counter() - t0
        self.history.append(record)
        return record

    def run(self, n_gen: Optional[int] = None, callback=None) -> dict:
        n = self.cfg.n_gen - self.generation if n_gen is None else n_gen
        rec = {}
        for _ in range(n):
            rec = self.step()
            if callback is not None:
                callback(rec)
        return rec

    def best(self):
        """(Z, x) of the current elite (after the last evaluation)."""
        return float(self.z[0]), decode(self.genes[:1], self.cfg.lo, self.cfg.hi)[0]

    # -- checkpoint / resume ------------------------------------------------------
    def state_dict(self) -> dict:
        return {"cfg": asdict(self.cfg), "genes": self.genes.copy(), "z": self.z.copy(),
                "generation": self.generation, "step_size": self.step_size.copy(),
                "rng": json.dumps(self.rng.bit_generator.state)}

    def load_state_dict(self, st: dict):
        self.genes = np.array(st["genes"], dtype=np.float64)
        self.z = np.array(st["z"], dtype=np.float64)
        self.generation = int(st["generation"])
        self.step_size = np.array(st["step_size"], dtype=np.float64)
        self.rng.bit_generator.state = json.loads(str(st["rng"]))

    def save(self, path: str):
        st = self.state_dict()
        np.savez(path, genes=st["genes"], z=st["z"], generation=st["generation"],
                 step_size=st["step_size"], rng=np.array(st["rng"]), cfg=np.array(json.dumps(st["cfg"])))

    def load(self, path: str):
        d = np.load(path, allow_pickle=False)
        self.load_state_dict({"genes": d["genes"], "z": d["z"], "generation": int(d["generation"]),
                              "step_size": d["step_size"], "rng": str(d["rng"])})


def gpu_fitness(tset, weights=(1.0, 1.0, 1.0), precision: str = "fp32"):
    """Fitness and gradient callables for GA backed by a TersoffSet."""
    import torch

    def fit(x: np.ndarray) -> np.ndarray:
        return tset.fitness(x, weights, precision)[:, 0].cpu().numpy()

    def grad(x: np.ndarray):
        Z, G = tset.fitness_grad(x, weights, precision)
        torch.cuda.current_stream().synchronize()
        return Z[:, 0].cpu().numpy(), G.cpu().numpy()

    return fit, grad
