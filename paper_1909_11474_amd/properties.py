"""0 K properties of diamond silicon on the GPU evaluation path.

Every energy, virial and force comes from one batched ``tersoff_eval`` call
(float64) over a set of structures built for the purpose: lattice constants,
strains and displaced supercells are batched as the structures of a set, so
each stage is a single launch sequence.  The host only builds the geometries
and does the small linear algebra (a cubic interpolation, a 3 x 3 Newton step,
6 x 6 Hermitian eigenproblems).

* Lattice constant: the zero of the hydrostatic virial tr W (tr W = -dE/d ln a
  of the cell), bracketed on a coarse grid of lattice constants, then on a fine
  grid inside the bracket, then inverse cubic interpolation (Sec. III.C).
* Elastic constants (Table 3, stress-strain at 0 K): sigma = -W / V under
  +-eps_xx (C11, C12) and +-eps_yz (C44).  The relaxed C44 lets the two fcc
  sublattices shift rigidly against each other (the only internal coordinate
  a homogeneous strain of diamond has), found by Newton steps on the total
  force of one sublattice with a finite-difference Hessian.
* Phonons (Fig. 4): force constants by central differences of the forces for
  displacements of the two basis atoms in an n x n x n conventional supercell,
  the dynamical matrix by a phase-weighted sum over minimum-image separations,
  frequencies from its eigenvalues.

x may be a minimal [6] or Tersoff-form [9] parameter vector.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np

EV_A3_TO_GPA = 160.21766208          # eV / A^3 in GPa
SI_MASS_AMU = 28.0855
# sqrt(eV / (A^2 u)) / (2 pi), in THz
THZ = math.sqrt(1.602176634e-19 / 1.66053906660e-27) * 1e10 / (2.0 * math.pi) / 1e12
VIRIAL_PAIRS = ((0, 0), (1, 1), (2, 2), (1, 2), (2, 0), (0, 1))   # xx yy zz yz zx xy


def conventional_cell(a: float, n: int = 1):
    """Diamond: n^3 conventional cells of 8 atoms; atom 8c + s, s < 4 on the fcc
    sublattice A, s >= 4 on B = A + a/4 (1, 1, 1)."""
    fcc = np.array([[0, 0, 0], [0, 2, 2], [2, 0, 2], [2, 2, 0]], dtype=np.float64) / 4.0
    basis = np.concatenate([fcc, fcc + 0.25])
    grid = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1)
    pos = (grid.reshape(-1, 1, 3) + basis[None]).reshape(-1, 3) * a
    return pos, np.eye(3) * (a * n)


def evaluate(structs: Sequence, x, R1: float = 2.8, R2: float = 3.2, forces: bool = False):
    """One float64 tersoff_eval over the structures [(pos, cell), ...]: energies [S],
    virial tensors [S, 3, 3] and, if asked, forces (a list of [N_s, 3])."""
    from . import api
    pos = np.concatenate([p for p, _ in structs])
    cell = np.stack([c for _, c in structs])
    off = np.concatenate([[0], np.cumsum([p.shape[0] for p, _ in structs])])
    ts = api.TersoffSet(pos, cell, off, R1, R2)
    try:
        out = ts.tersoff_eval(np.asarray(x, dtype=np.float64)[None], precision="fp64",
                              forces=forces, virial=True)
        E = out["E"][0].cpu().numpy()
        W6 = out["W"][0].cpu().numpy()
        F = out["F"][0].cpu().numpy() if forces else None
    finally:
        ts.close()
    W = np.zeros((len(structs), 3, 3))
    for k, (m, n) in enumerate(VIRIAL_PAIRS):
        W[:, m, n] = W[:, n, m] = W6[:, k]
    res = {"E": E, "W": W}
    if forces:
        res["F"] = [F[off[s]:off[s + 1]] for s in range(len(structs))]
    return res


def lattice_constant(x, R1: float = 2.8, R2: float = 3.2, bounds=(5.0, 5.9),
                     n_coarse: int = 91, n_fine: int = 64):
    """(a0, energy per atom at a0) of diamond: tr W(a) = 0."""
    def trace_w(grid):
        res = evaluate([conventional_cell(a) for a in grid], x, R1, R2)
        return np.trace(res["W"], axis1=1, axis2=2)

    def bracket(grid, w):
        # tr W > 0 under compression (a < a0), < 0 under tension
        k = np.nonzero((w[:-1] > 0) & (w[1:] <= 0))[0]
        if k.size == 0:
            raise ValueError(f"no zero of the hydrostatic virial in [{grid[0]}, {grid[-1]}] A")
        return int(k[0])

    grid = np.linspace(bounds[0], bounds[1], n_coarse)
    k = bracket(grid, trace_w(grid))
    fine = np.linspace(grid[k], grid[k + 1], n_fine)
    w = trace_w(fine)
    j = bracket(fine, w)
    lo = min(max(j - 1, 0), n_fine - 4)
    sel = slice(lo, lo + 4)
    a0 = float(np.polyval(np.polyfit(w[sel], fine[sel], 3), 0.0))   # inverse interpolation
    res = evaluate([conventional_cell(a0)], x, R1, R2)
    return a0, float(res["E"][0]) / 8.0


def _stress(W, cell):
    return -W / abs(np.linalg.det(cell)) * EV_A3_TO_GPA


def _strained(a0, F):
    pos, cell = conventional_cell(a0)
    return pos @ F.T, cell @ F.T


def elastic_constants(x, a0: float, R1: float = 2.8, R2: float = 3.2, strain: float = 1e-4,
                      shear: float = 1e-3, h: float = 1e-4, max_newton: int = 8) -> dict:
    """C11, C12, C44 (relaxed) and C44_unrelaxed in GPa at lattice constant a0, and
    the relaxed sublattice shift per unit engineering shear (A)."""
    Fs = []
    for sign in (+1, -1):
        F = np.eye(3)
        F[0, 0] += sign * strain
        Fs.append(F)
    for sign in (+1, -1):
        F = np.eye(3)
        F[1, 2] = F[2, 1] = sign * shear / 2
        Fs.append(F)
    base = [_strained(a0, F) for F in Fs]
    res = evaluate(base, x, R1, R2)
    sig = [_stress(W, c) for W, (_, c) in zip(res["W"], base)]
    C11 = (sig[0][0, 0] - sig[1][0, 0]) / (2 * strain)
    C12 = (sig[0][1, 1] - sig[1][1, 1]) / (2 * strain)
    C44u = (sig[2][1, 2] - sig[3][1, 2]) / (2 * shear)

    # relaxed shear: Newton on the shift s of sublattice B for both signs at once
    Bmask = np.zeros(8, dtype=bool)
    Bmask[4:] = True
    s = [np.zeros(3), np.zeros(3)]
    sheared = base[2:]
    shifts = [np.zeros(3)] + [sgn * h * e for e in np.eye(3) for sgn in (+1, -1)]
    for _ in range(max_newton):
        structs = []
        for (pos, cell), sk in zip(sheared, s):
            for d in shifts:
                p = pos.copy()
                p[Bmask] += sk + d
                structs.append((p, cell))
        res = evaluate(structs, x, R1, R2, forces=True)
        fB = np.array([f[Bmask].sum(axis=0) for f in res["F"]]).reshape(2, 7, 3)
        done = True
        for k in range(2):
            g = fB[k, 0]                                   # -dE/ds
            H = np.empty((3, 3))
            for b in range(3):
                H[:, b] = -(fB[k, 1 + 2 * b] - fB[k, 2 + 2 * b]) / (2 * h)
            step = np.linalg.solve(H, g)
            if np.abs(step).max() > 1e-13:
                done = False
            s[k] = s[k] + step
        if done:
            break
    relaxed = []
    for (pos, cell), sk in zip(sheared, s):
        p = pos.copy()
        p[Bmask] += sk
        relaxed.append((p, cell))
    res = evaluate(relaxed, x, R1, R2)
    sr = [_stress(W, c) for W, (_, c) in zip(res["W"], relaxed)]
    C44 = (sr[0][1, 2] - sr[1][1, 2]) / (2 * shear)
    return {"C11": float(C11), "C12": float(C12), "C44": float(C44), "C44_unrelaxed": float(C44u),
            "shift_per_shear": (s[0] - s[1]) / (2 * shear)}


def force_constants(x, a0: float, n: int = 3, h: float = 1e-3, R1: float = 2.8, R2: float = 3.2):
    """(phi [2, 3, N, 3] = -dF_j/du_k in eV/A^2 for basis atoms k = A (atom 0) and
    B (atom 4), supercell positions [N, 3], cell [3, 3]); the 12 displaced
    supercells form one set."""
    pos, cell = conventional_cell(a0, n)
    structs = []
    for atom in (0, 4):
        for a in range(3):
            for sign in (+1, -1):
                p = pos.copy()
                p[atom, a] += sign * h
                structs.append((p, cell))
    F = evaluate(structs, x, R1, R2, forces=True)["F"]
    phi = np.array([-(F[2 * i] - F[2 * i + 1]) / (2 * h) for i in range(6)])
    return phi.reshape(2, 3, pos.shape[0], 3), pos, cell


def dynamical_matrices(phi, pos, cell, qs, mass: float = SI_MASS_AMU):
    """D(q) [Q, 6, 6] (eV / (A^2 u)); sublattice of atom j is (j mod 8) >= 4."""
    qs = np.atleast_2d(np.asarray(qs, dtype=np.float64))
    L = np.diag(cell)
    sub = (np.arange(pos.shape[0]) % 8) >= 4
    D = np.zeros((qs.shape[0], 6, 6), dtype=np.complex128)
    for k, centre in enumerate((0, 4)):
        d = pos - pos[centre]
        d -= L * np.round(d / L)                             # minimum image (cubic supercell)
        ph = np.exp(1j * (qs @ d.T))                         # [Q, N]
        for kp in (0, 1):
            m = sub == bool(kp)
            # sum_j phi[k, a, j, b] e^{i q . d_j} over the atoms of sublattice kp
            D[:, 3 * k:3 * k + 3, 3 * kp:3 * kp + 3] = np.einsum(
                "qj,ajb->qab", ph[:, m], phi[k][:, m, :])
    return D / mass


def frequencies(phi, pos, cell, qs, mass: float = SI_MASS_AMU):
    """Phonon frequencies [Q, 6] in THz, ascending (imaginary modes negative)."""
    D = dynamical_matrices(phi, pos, cell, qs, mass)
    D = 0.5 * (D + np.conj(np.swapaxes(D, 1, 2)))
    w2 = np.linalg.eigvalsh(D)
    return np.sign(w2) * np.sqrt(np.abs(w2)) * THZ


def dispersion_path(a0: float, points=("G", "X", "W", "K", "G", "L"), per_segment: int = 40):
    """Wavevectors along a path through the fcc high-symmetry points (1/A) and the
    cumulative path length; G, X, W, K, L in units of 2 pi / a."""
    sym = {"G": (0, 0, 0), "X": (1, 0, 0), "W": (1, 0.5, 0), "K": (0.75, 0.75, 0),
           "L": (0.5, 0.5, 0.5)}
    qs = []
    for p0, p1 in zip(points[:-1], points[1:]):
        t = np.linspace(0.0, 1.0, per_segment, endpoint=(p1 == points[-1]))
        qs.append(np.asarray(sym[p0]) + t[:, None] * (np.asarray(sym[p1]) - np.asarray(sym[p0])))
    q = np.concatenate(qs) * 2 * np.pi / a0
    dist = np.concatenate([[0.0], np.cumsum(np.linalg.norm(np.diff(q, axis=0), axis=1))])
    return q, dist
