"""0 K properties of diamond silicon from the oracle potential (test
infrastructure only: imported by tests/ and nothing in the product path).

* Lattice constant and cohesive energy: minimum of the energy per atom of
  perfect diamond over the lattice constant (Sec. III.C prints -4.63 eV/atom
  and 5.434 A for the Table 2 parameters).
* Elastic constants C11, C12, C44 from stress-strain relations at zero
  temperature (Table 3): central differences of the stress sigma = -W / V over
  small homogeneous strains of the conventional cell; C44 with the internal
  coordinates relaxed (the two fcc sublattices shift against each other under
  shear), and the unrelaxed C44^0 as well.
* Harmonic phonons by the finite-displacement method (Fig. 4): force constants
  Phi_ab(0k, lk') = -dF_{lk',b}/du_{0k,a} by central differences of the forces
  in a periodic supercell, the dynamical matrix
  D_{ka,k'b}(q) = sum_l Phi_ab(0k, lk') exp(i q . (R_l + tau_k' - tau_k)) / m,
  and the frequencies sqrt(eig D) / (2 pi).

Each step calls oracle.tersoff.evaluate (float64 autograd) on explicit
structures; the only shortcuts are a bounded 1-D minimisation and scipy's
root finder for the internal relaxation.
"""
from __future__ import annotations

import math

import numpy as np

from . import tersoff as T

EV_A3_TO_GPA = 160.21766208          # 1 eV / A^3 in GPa
M_SI_AMU = 28.0855                   # silicon atomic mass (u)
# sqrt(eV / (A^2 u)) / (2 pi) in THz, from the CODATA 2018 elementary charge and
# atomic mass constant
THZ_PER_SQRT_EV_A2_AMU = math.sqrt(1.602176634e-19 / (1e-20 * 1.66053906660e-27)) / (2 * math.pi) / 1e12

_FCC = np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]])


def diamond_cell(a: float, n: int = 1):
    """Conventional diamond cell (8 atoms) repeated n x n x n; positions [8 n^3, 3]
    ordered cell by cell, sublattice A (fcc) then B (fcc + a/4 (1,1,1)) in each."""
    base = np.vstack([_FCC, _FCC + 0.25])
    pos = []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                pos.append((base + [i, j, k]) * a)
    return np.vstack(pos), np.eye(3) * a * n


def energy_per_atom(x, a: float, R1: float = 2.8, R2: float = 3.2) -> float:
    pos, cell = diamond_cell(a)
    return float(T.evaluate(pos, cell, x, R1, R2)["E"][0]) / pos.shape[0]


def lattice_constant(x, R1: float = 2.8, R2: float = 3.2, bounds=(5.0, 5.9)):
    """(a0, E per atom at a0): bounded minimisation of the energy per atom of the
    8-atom cell (Sec. III.C)."""
    from scipy.optimize import minimize_scalar
    res = minimize_scalar(lambda a: energy_per_atom(x, a, R1, R2), bounds=bounds,
                          method="bounded", options={"xatol": 1e-10})
    return float(res.x), float(res.fun)


def stress_gpa(pos, cell, x, R1=2.8, R2=3.2):
    """Stress tensor sigma = -W / V in GPa (tension positive) and the evaluation."""
    out = T.evaluate(pos, cell, x, R1, R2)
    Wt = np.zeros((3, 3))
    for (m, n), v in zip(T.VIRIAL6, out["W6"][0]):
        Wt[m, n] = Wt[n, m] = v
    return -Wt / abs(np.linalg.det(cell)) * EV_A3_TO_GPA, out


def relax_positions(pos, cell, x, R1=2.8, R2=3.2, xtol=1e-14):
    """Internal coordinates at fixed cell: the zero of the oracle's forces on
    atoms 1.., atom 0 held fixed (removes the rigid translation; the force on
    atom 0 then vanishes by the sum rule), by MINPACK's hybrid Powell method.
    Solving F = 0 rather than minimising E reaches the forces' round-off level;
    a minimiser stalls where energy differences fall below the energy's
    round-off (about 1e-7 eV/A here)."""
    from scipy.optimize import root

    def forces(flat):
        p = np.vstack([pos[:1], flat.reshape(-1, 3)])
        return T.evaluate(p, cell, x, R1, R2)["F"][1:].ravel()

    res = root(forces, pos[1:].ravel(), method="hybr", options={"xtol": xtol})
    return np.vstack([pos[:1], res.x.reshape(-1, 3)])


def elastic_constants(x, a0: float, R1=2.8, R2=3.2, strain=1e-4, shear=1e-3) -> dict:
    """C11, C12, C44 (relaxed), C44^0 (unrelaxed) in GPa at lattice constant a0
    (Table 3): sigma_xx and sigma_yy under eps_xx = +-strain; sigma_yz under the
    symmetric shear eps_yz = eps_zy = +-shear / 2 (engineering shear +-shear)."""
    pos0, cell0 = diamond_cell(a0)
    s = []
    for sign in (+1, -1):
        F = np.eye(3)
        F[0, 0] += sign * strain
        s.append(stress_gpa(pos0 @ F.T, cell0 @ F.T, x, R1, R2)[0])
    C11 = (s[0][0, 0] - s[1][0, 0]) / (2 * strain)
    C12 = (s[0][1, 1] - s[1][1, 1]) / (2 * strain)
    s44, s44u = [], []
    for sign in (+1, -1):
        F = np.eye(3)
        F[1, 2] = F[2, 1] = sign * shear / 2
        cell = cell0 @ F.T
        s44u.append(stress_gpa(pos0 @ F.T, cell, x, R1, R2)[0][1, 2])
        pos = relax_positions(pos0 @ F.T, cell, x, R1, R2)
        s44.append(stress_gpa(pos, cell, x, R1, R2)[0][1, 2])
    return {"C11": C11, "C12": C12, "C44": (s44[0] - s44[1]) / (2 * shear),
            "C44_unrelaxed": (s44u[0] - s44u[1]) / (2 * shear)}


def force_constants(x, a0: float, n: int = 3, h: float = 1e-3, R1=2.8, R2=3.2):
    """Phi[k, a, j, b] = -dF_{j,b}/du_{k,a} (eV/A^2) for the two basis atoms
    k = 0 (A) and 1 (B) of the first conventional cell of an n x n x n supercell,
    by central differences of the forces (displacement h in A); with the
    supercell positions [N, 3] and cell."""
    pos, cell = diamond_cell(a0, n)
    basis = (0, 4)                               # first A atom and first B atom
    phi = np.zeros((2, 3, pos.shape[0], 3))
    for k, atom in enumerate(basis):
        for a in range(3):
            f = []
            for sign in (+1, -1):
                p = pos.copy()
                p[atom, a] += sign * h
                f.append(T.evaluate(p, cell, x, R1, R2)["F"])
            phi[k, a] = -(f[0] - f[1]) / (2 * h)
    return phi, pos, cell


def dynamical_matrix(phi, pos, cell, q, mass: float = M_SI_AMU):
    """6 x 6 dynamical matrix at wavevector q (1/A, Cartesian) from supercell force
    constants; each pair takes its minimum-image separation (the force
    constants vanish well inside half the supercell)."""
    n_at = pos.shape[0]
    sub = np.array([0 if (i % 8) < 4 else 1 for i in range(n_at)])   # sublattice per atom
    tau = np.array([pos[0], pos[4]])
    L = np.diag(cell)
    D = np.zeros((6, 6), dtype=complex)
    for k in range(2):
        for j in range(n_at):
            kp = sub[j]
            d = pos[j] - tau[k]
            d = d - L * np.round(d / L)                # minimum image, cubic cell
            ph = np.exp(1j * np.dot(q, d))
            for a in range(3):
                for b in range(3):
                    D[3 * k + a, 3 * kp + b] += phi[k, a, j, b] * ph
    return D / mass


def frequencies_thz(phi, pos, cell, q, mass: float = M_SI_AMU):
    """Six phonon frequencies at q (THz), ascending; imaginary modes negative."""
    D = dynamical_matrix(phi, pos, cell, q, mass)
    D = 0.5 * (D + D.conj().T)
    w2 = np.linalg.eigvalsh(D)
    return np.sign(w2) * np.sqrt(np.abs(w2)) * THZ_PER_SQRT_EV_A2_AMU


def sound_velocity(C_gpa: float, a0: float, mass: float = M_SI_AMU) -> float:
    """sqrt(C / rho) in km/s for the 8-atom cell of lattice constant a0."""
    rho = 8 * mass * 1.66053906660e-27 / (a0 * 1e-10) ** 3        # kg/m^3
    return math.sqrt(C_gpa * 1e9 / rho) / 1e3
