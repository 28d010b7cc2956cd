"""Seeded synthetic inputs for the minimal-Tersoff fitting workloads.

This module builds the structures, populations and velocities that stand in
for the paper's DFT training set (Sec. III.A: strained diamond cells and 64-atom
periodic force cells).  It holds geometry and random draws only -- no potential
arithmetic -- so that both the CPU oracle and the GPU library can be fed the
same inputs without sharing any of the method's code.

Every generator takes an explicit seed and uses numpy's PCG64 bit generator.

Workloads (sizes follow the paper's training data shapes):

* ``config1``  one 64-atom diamond cell (2x2x2 conventional, a = 5.43 A),
  Gaussian displacements sigma = 0.05 A, one parameter set drawn inside the
  parameter box.
* ``config2``  100 strained 64-atom diamond cells (strain U(+-2 %), sigma =
  0.1 A) and a population of 200 parameter sets; the GA fitness batch.
* ``config3``  300 structures of 8-512 atoms: strained diamond supercells,
  the same with 1-4 vacancies, and random sequential packings at
  2.33 g/cm^3 with a 2.1 A minimum separation; population 500.
* ``config4``  config3's structures with a population of 64 (gradient runs).
* ``config5``  one 64,000-atom diamond cell (20^3 conventional cells) with
  thermal displacements sigma = 0.08 A and 300 K Maxwell-Boltzmann velocities.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# Table 2 of the paper: optimised minimal-Tersoff parameters
# [D0 (eV), alpha (1/A), r0 (A), beta, n, h] and the hand-chosen cutoffs.
TABLE2_X = (3.21481, 1.43134, 2.23801, 0.282818, 0.602568, -0.641048)
TABLE2_R1 = 2.8
TABLE2_R2 = 3.2

# Parameter box used for random draws.  The paper maps each gene in [0, 1]
# linearly onto two limits per parameter but does not print them (Sec. III.B);
# these limits contain Table 2 and keep every parameter of order unity.
PARAM_LO = (2.0, 1.0, 2.0, 0.1, 0.5, -1.0)
PARAM_HI = (5.0, 2.0, 2.6, 1.0, 1.5, 0.0)
# Nine-parameter Tersoff form [D0, alpha, r0, S, gamma, n, c, d, h]: a box of
# order-unity values around the minimal potential's (S = 2 inside it).
FULL_LO = (2.0, 1.0, 2.0, 1.5, 0.05, 0.5, 0.5, 0.5, -1.0)
FULL_HI = (5.0, 2.0, 2.6, 3.0, 1.0, 1.5, 3.0, 3.0, 0.0)

A_SI = 5.43                     # diamond Si lattice constant used for the cells (A)
RHO_SI = 0.04996                # 2.33 g/cm^3 in atoms / A^3
M_SI_AMU = 28.0855              # Si atomic mass (u)
KB_EV = 8.617333262e-5          # Boltzmann constant (eV/K)
AMU_A2_FS2_EV = 103.642691      # 1 u * A^2 / fs^2 expressed in eV

_DIAMOND_BASIS = np.array(
    [[0.00, 0.00, 0.00], [0.00, 0.50, 0.50], [0.50, 0.00, 0.50], [0.50, 0.50, 0.00],
     [0.25, 0.25, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75], [0.75, 0.75, 0.25]])


@dataclass
class StructureSet:
    """A batch of periodic structures.

    pos     [N_tot, 3] float64 Cartesian positions (A), structures concatenated
    cell    [S, 3, 3]  float64, rows are the lattice vectors a, b, c (A)
    offset  [S + 1]    int64, atoms of structure s are offset[s]:offset[s+1]
    """
    pos: np.ndarray
    cell: np.ndarray
    offset: np.ndarray
    kinds: List[str] = field(default_factory=list)

    @property
    def n_struct(self) -> int:
        return int(self.cell.shape[0])

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])

    def sizes(self) -> np.ndarray:
        return np.diff(self.offset)

    def structure(self, s: int):
        a, b = int(self.offset[s]), int(self.offset[s + 1])
        return self.pos[a:b], self.cell[s]

    def subset(self, idx) -> "StructureSet":
        idx = list(idx)
        pos = [self.pos[self.offset[s]:self.offset[s + 1]] for s in idx]
        return make_set([(p, self.cell[s]) for p, s in zip(pos, idx)],
                        [self.kinds[s] for s in idx] if self.kinds else None)


def make_set(structs, kinds: Optional[List[str]] = None) -> StructureSet:
    """Concatenate a list of (pos [N,3], cell [3,3]) into a StructureSet."""
    sizes = [int(p.shape[0]) for p, _ in structs]
    offset = np.zeros(len(structs) + 1, dtype=np.int64)
    offset[1:] = np.cumsum(sizes)
    pos = np.concatenate([np.asarray(p, dtype=np.float64) for p, _ in structs], axis=0)
    cell = np.stack([np.asarray(c, dtype=np.float64) for _, c in structs], axis=0)
    return StructureSet(pos=pos, cell=cell, offset=offset, kinds=list(kinds or []))


def diamond(nx: int, ny: int, nz: int, a: float = A_SI):
    """Perfect diamond lattice of nx*ny*nz conventional cubic cells (8 atoms each)."""
    grid = np.array([[i, j, k] for i in range(nx) for j in range(ny) for k in range(nz)],
                    dtype=np.float64)
    frac = (grid[:, None, :] + _DIAMOND_BASIS[None, :, :]).reshape(-1, 3)
    pos = frac * a
    cell = np.diag([nx * a, ny * a, nz * a]).astype(np.float64)
    return pos, cell


def random_strain(rng: np.random.Generator, max_eps: float = 0.02) -> np.ndarray:
    """Deformation gradient I + eps, eps symmetric: one isotropic diagonal draw
    and three independent shear draws, all uniform in [-max_eps, max_eps]."""
    iso = rng.uniform(-max_eps, max_eps)
    exy, eyz, ezx = rng.uniform(-max_eps, max_eps, size=3)
    eps = np.array([[iso, exy, ezx], [exy, iso, eyz], [ezx, eyz, iso]])
    return np.eye(3) + eps


def deform(pos: np.ndarray, cell: np.ndarray, F: np.ndarray):
    """Apply the homogeneous deformation F to positions and cell rows."""
    return pos @ F.T, cell @ F.T


def displace(rng: np.random.Generator, pos: np.ndarray, sigma: float) -> np.ndarray:
    return pos + rng.normal(0.0, sigma, size=pos.shape)


def draw_params_full(rng: np.random.Generator, count: int) -> np.ndarray:
    """Nine-parameter Tersoff sets drawn uniformly inside their box, [count, 9]."""
    u = rng.uniform(0.0, 1.0, size=(count, 9))
    lo = np.asarray(FULL_LO)
    hi = np.asarray(FULL_HI)
    return lo + u * (hi - lo)


def minimal_as_full(x: np.ndarray, d: float, c: float) -> np.ndarray:
    """The nine-parameter set whose g^T approaches beta (cos - h)^2 as d and
    c / d^2 grow (Sec. II.B): S = 2, gamma = beta d^4 / c^2."""
    D0, alpha, r0, beta, n, h = x
    return np.array([D0, alpha, r0, 2.0, beta * d ** 4 / c ** 2, n, c, d, h])


def draw_params(rng: np.random.Generator, count: int) -> np.ndarray:
    """Parameter sets drawn uniformly inside the parameter box, [count, 6]."""
    u = rng.uniform(0.0, 1.0, size=(count, 6))
    lo = np.asarray(PARAM_LO)
    hi = np.asarray(PARAM_HI)
    return lo + u * (hi - lo)


def random_packing(rng: np.random.Generator, n: int, rho: float = RHO_SI,
                   dmin: float = 2.1, max_tries: int = 200000):
    """Random sequential addition of n points in a periodic cube of density rho,
    every pair (minimum image) at least dmin apart."""
    L = (n / rho) ** (1.0 / 3.0)
    pts = np.empty((0, 3))
    tries = 0
    while pts.shape[0] < n:
        batch = rng.uniform(0.0, L, size=(64, 3))
        for p in batch:
            tries += 1
            if tries > max_tries:
                raise RuntimeError("random packing did not converge")
            if pts.shape[0]:
                d = pts - p
                d -= L * np.round(d / L)
                if np.min(np.einsum("ij,ij->i", d, d)) < dmin * dmin:
                    continue
            pts = np.vstack([pts, p])
            if pts.shape[0] == n:
                break
    return pts, np.diag([L, L, L]).astype(np.float64)


# ----------------------------------------------------------------------------
# Workload configurations
# ----------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    structs: StructureSet
    population: np.ndarray                 # [P, 6] (minimal) or [P, 9] (Tersoff form) parameter sets
    hidden_x: Optional[np.ndarray] = None  # parameters the reference data come from
    velocities: Optional[np.ndarray] = None
    R1: float = TABLE2_R1
    R2: float = TABLE2_R2
    seeds: dict = field(default_factory=dict)


def config1(disp_seed: int = 1, param_seed: int = 2) -> Workload:
    rng = np.random.Generator(np.random.PCG64(disp_seed))
    pos, cell = diamond(2, 2, 2)
    pos = displace(rng, pos, 0.05)
    x = draw_params(np.random.Generator(np.random.PCG64(param_seed)), 1)
    return Workload("config1: one 64-atom diamond Si cell, sigma 0.05 A, one parameter set",
                    make_set([(pos, cell)], ["diamond"]), x,
                    seeds={"displacements": disp_seed, "params": param_seed})


def strained_diamond_cells(seed: int, count: int, reps=(2, 2, 2), sigma: float = 0.1):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        pos, cell = diamond(*reps)
        pos, cell = deform(pos, cell, random_strain(rng))
        out.append((displace(rng, pos, sigma), cell))
    return out


def config2(struct_seed: int = 3, hidden_seed: int = 4, pop_seed: int = 5,
            n_struct: int = 100, pop: int = 200) -> Workload:
    structs = make_set(strained_diamond_cells(struct_seed, n_struct), ["diamond"] * n_struct)
    hidden = draw_params(np.random.Generator(np.random.PCG64(hidden_seed)), 1)[0]
    x = draw_params(np.random.Generator(np.random.PCG64(pop_seed)), pop)
    return Workload(f"config2: GA fitness batch, {pop} candidates x {n_struct} strained "
                    "64-atom diamond cells", structs, x, hidden_x=hidden,
                    seeds={"structures": struct_seed, "hidden": hidden_seed, "population": pop_seed})


def config2_tersoff_form(struct_seed: int = 3, hidden_seed: int = 11, pop_seed: int = 12,
                         n_struct: int = 100, pop: int = 200) -> Workload:
    """config 2's structures with nine-parameter Tersoff-form candidates and a
    hidden nine-parameter set (Sec. II.A Eq. 8 with a free slope S)."""
    structs = make_set(strained_diamond_cells(struct_seed, n_struct), ["diamond"] * n_struct)
    hidden = draw_params_full(np.random.Generator(np.random.PCG64(hidden_seed)), 1)[0]
    x = draw_params_full(np.random.Generator(np.random.PCG64(pop_seed)), pop)
    return Workload(f"config2-tf: GA fitness batch, Tersoff form (9 parameters), {pop} candidates "
                    f"x {n_struct} strained 64-atom diamond cells", structs, x, hidden_x=hidden,
                    seeds={"structures": struct_seed, "hidden": hidden_seed, "population": pop_seed})


def uneven_structures(seed: int = 6, n_each: int = 100) -> StructureSet:
    """Strained diamond supercells (8-512 atoms), the same with 1-4 vacancies,
    and random sequential packings of 8-512 atoms."""
    rng = np.random.Generator(np.random.PCG64(seed))
    structs, kinds = [], []
    for _ in range(n_each):
        reps = rng.integers(1, 5, size=3)
        pos, cell = diamond(*reps)
        pos, cell = deform(pos, cell, random_strain(rng))
        structs.append((displace(rng, pos, 0.1), cell))
        kinds.append("diamond")
    for _ in range(n_each):
        while True:
            reps = rng.integers(1, 5, size=3)
            if int(np.prod(reps)) >= 2:
                break
        pos, cell = diamond(*reps)
        nvac = int(rng.integers(1, 5))
        keep = np.sort(rng.permutation(pos.shape[0])[nvac:])
        pos = pos[keep]
        pos, cell = deform(pos, cell, random_strain(rng))
        structs.append((displace(rng, pos, 0.1), cell))
        kinds.append("vacancy")
    for _ in range(n_each):
        n = int(rng.integers(8, 513))
        structs.append(random_packing(rng, n))
        kinds.append("packing")
    return make_set(structs, kinds)


def config3(struct_seed: int = 6, hidden_seed: int = 4, pop_seed: int = 7,
            pop: int = 500, n_each: int = 100) -> Workload:
    structs = uneven_structures(struct_seed, n_each)
    hidden = draw_params(np.random.Generator(np.random.PCG64(hidden_seed)), 1)[0]
    x = draw_params(np.random.Generator(np.random.PCG64(pop_seed)), pop)
    return Workload(f"config3: uneven batching, {pop} candidates x {structs.n_struct} "
                    "structures of 8-512 atoms", structs, x, hidden_x=hidden,
                    seeds={"structures": struct_seed, "hidden": hidden_seed, "population": pop_seed})


def config4(struct_seed: int = 6, hidden_seed: int = 4, pop_seed: int = 8,
            pop: int = 64, n_each: int = 100) -> Workload:
    w = config3(struct_seed, hidden_seed, pop_seed, pop, n_each)
    w.name = (f"config4: fitness gradient, {pop} candidates x {w.structs.n_struct} "
              "structures of 8-512 atoms")
    return w


def maxwell_boltzmann(rng: np.random.Generator, n: int, temperature: float,
                      mass_amu: float = M_SI_AMU) -> np.ndarray:
    """Velocities (A/fs) from the Maxwell-Boltzmann distribution, zero total momentum."""
    sigma = np.sqrt(KB_EV * temperature / (mass_amu * AMU_A2_FS2_EV))
    v = rng.normal(0.0, sigma, size=(n, 3))
    return v - v.mean(axis=0, keepdims=True)


def config5(disp_seed: int = 9, vel_seed: int = 10, reps: int = 20) -> Workload:
    rng = np.random.Generator(np.random.PCG64(disp_seed))
    pos, cell = diamond(reps, reps, reps)
    pos = displace(rng, pos, 0.08)
    vel = maxwell_boltzmann(np.random.Generator(np.random.PCG64(vel_seed)), pos.shape[0], 300.0)
    x = np.asarray([TABLE2_X], dtype=np.float64)
    return Workload(f"config5: one {pos.shape[0]}-atom diamond Si cell ({reps}^3 conventional), "
                    "sigma 0.08 A, 300 K velocities", make_set([(pos, cell)], ["diamond"]), x,
                    velocities=vel, seeds={"displacements": disp_seed, "velocities": vel_seed})
