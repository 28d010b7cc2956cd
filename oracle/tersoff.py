"""Minimal Tersoff potential in plain float64 PyTorch (oracle; test infrastructure only).

Each function follows the paper's definitions directly; derivatives are taken
by autograd, so no hand-derived force, virial or gradient formula appears here.

Definitions used (paper Sec. II):
  U = sum_i U_i,  U_i = 1/2 sum_{j != i} U_ij                         (Sec. II.A, Eqs. 1-2)
  U_ij = f_C(r_ij) [f_R(r_ij) - b_ij f_A(r_ij)]                        (Sec. II.A, Eq. 3)
  f_R = A exp(-lambda r),  f_A = B exp(-mu r)                         (Sec. II.A, Eqs. 4-5)
  b_ij = (1 + zeta_ij^n)^(-1/(2n)),  b_ij = 1 when zeta_ij = 0         (Sec. II.A, Eq. 6)
  zeta_ij = sum_{k != i,j} f_C(r_ik) g(theta_ijk)                      (Sec. II.A, Eq. 7)
  g = beta (cos theta - h)^2                                            (Sec. II.B, Eq. 10)
  f_C: 1 for r <= R1, (1 + cos(pi (r-R1)/(R2-R1)))/2 between, 0 for r >= R2  (Sec. II.A, Eq. 9)
  A = D0/(S-1) exp(alpha r0 sqrt(2S)),  B = D0 S/(S-1) exp(alpha r0 sqrt(2/S)),
  lambda = alpha sqrt(2S),  mu = alpha sqrt(2/S),  with S fixed to 2      (Sec. II.B, Eqs. 11-14)

Parameter vectors: the minimal potential x = [D0, alpha, r0, beta, n, h]; the
Tersoff form with its original angular function
  g^T = gamma (1 + c^2/d^2 - c^2/(d^2 + (cos theta - h)^2))             (Sec. II.A, Eq. 8)
and a free slope S, x = [D0, alpha, r0, S, gamma, n, c, d, h] (the paper's nine
parameters A, B, lambda, mu, gamma, n, c, d, h with A, B, lambda, mu written
through D0, alpha, r0, S as in Eqs. 11-14).

Readings where the paper is silent (listed with the design notes of the
library): a neighbour entry is an (atom, periodic image) pair and "k != i, j"
excludes only the entry j itself; the virial is W = -dE/d(strain) (positive under
compression), reported per atom inside the fitness; the energy in the fitness
is per atom.  Forces and virial are the exact derivatives of U, which is what
the cited force and virial formulas compute.
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import numpy as np
import torch

from .neighbors import neighbor_list, neighbor_list_set, perpendicular_widths

DT = torch.float64
S_SLOPE = 2.0            # Pauling slope fixed to 2 in the minimal potential (Sec. II.B)

VIRIAL6 = ((0, 0), (1, 1), (2, 2), (1, 2), (2, 0), (0, 1))   # xx yy zz yz zx xy


def is_full(x) -> bool:
    """True for the nine-parameter Tersoff form, False for the minimal one."""
    return len(x) == 9


def derived_params(x: torch.Tensor):
    """(A, B, lambda, mu) from x (Sec. II.B, Eqs. 11-14); S = 2 for the minimal
    potential, x[3] for the nine-parameter form."""
    D0, alpha, r0 = x[0], x[1], x[2]
    S = x[3] if is_full(x) else torch.as_tensor(S_SLOPE, dtype=DT)
    A = D0 / (S - 1.0) * torch.exp(alpha * r0 * torch.sqrt(2.0 * S))
    B = D0 * S / (S - 1.0) * torch.exp(alpha * r0 * torch.sqrt(2.0 / S))
    lam = alpha * torch.sqrt(2.0 * S)
    mu = alpha * torch.sqrt(2.0 / S)
    return A, B, lam, mu


def angular(cos: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """g(theta): beta (cos - h)^2 (Sec. II.B, Eq. 10) or Tersoff's g^T (Sec. II.A, Eq. 8)."""
    if is_full(x):
        gamma, c, d, h = x[4], x[6], x[7], x[8]
        return gamma * (1.0 + c * c / (d * d) - c * c / (d * d + (cos - h) ** 2))
    beta, h = x[3], x[5]
    return beta * (cos - h) ** 2


def bond_order_exponent(x: torch.Tensor) -> torch.Tensor:
    """n of b = (1 + zeta^n)^(-1/(2n))."""
    return x[5] if is_full(x) else x[4]


def cutoff(r: torch.Tensor, R1: float, R2: float) -> torch.Tensor:
    """Cosine cutoff f_C (Sec. II.A, Eq. 9), closed at R1 and R2 as printed."""
    mid = 0.5 * (1.0 + torch.cos(math.pi * (r - R1) / (R2 - R1)))
    one = torch.ones_like(r)
    zero = torch.zeros_like(r)
    return torch.where(r <= R1, one, torch.where(r >= R2, zero, mid))


def triplets(center: np.ndarray, n_atoms: int):
    """All ordered pairs (p, q), p != q, of neighbour entries sharing a centre atom.

    ``center`` must be sorted ascending (entries grouped by centre atom)."""
    nb = center.shape[0]
    if nb == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    counts = np.bincount(center, minlength=n_atoms)
    start = np.concatenate([[0], np.cumsum(counts)])[:-1]
    m = counts[center]
    p = np.repeat(np.arange(nb), m)
    local = np.arange(p.shape[0]) - np.repeat(np.cumsum(m) - m, m)
    q = start[center[p]] + local
    keep = q != p
    return p[keep], q[keep]


def site_energies(d: torch.Tensor, center: np.ndarray, p: np.ndarray, q: np.ndarray,
                  n_atoms: int, x: torch.Tensor, R1: float, R2: float) -> torch.Tensor:
    """U_i for every atom, given the bond vectors d[e] = r_j + T - r_i of each
    neighbour entry e = (i, j, T) and the ordered entry pairs (p, q) with a common
    centre (Sec. II.A Eqs. 1-9, Sec. II.B Eq. 10)."""
    n = bond_order_exponent(x)
    A, B, lam, mu = derived_params(x)
    r = torch.sqrt((d * d).sum(dim=1))
    fc = cutoff(r, R1, R2)
    fR = A * torch.exp(-lam * r)
    fA = B * torch.exp(-mu * r)
    pt = torch.as_tensor(p)
    qt = torch.as_tensor(q)
    cos = (d[pt] * d[qt]).sum(dim=1) / (r[pt] * r[qt])
    g = angular(cos, x)
    zeta = torch.zeros_like(r).index_add(0, pt, fc[qt] * g)
    positive = zeta > 0
    zsafe = torch.where(positive, zeta, torch.ones_like(zeta))
    b = torch.where(positive, (1.0 + zsafe ** n) ** (-1.0 / (2.0 * n)), torch.ones_like(zeta))
    Uij = fc * (fR - b * fA)
    ct = torch.as_tensor(center)
    return torch.zeros(n_atoms, dtype=d.dtype).index_add(0, ct, 0.5 * Uij)


def _as_x(x) -> torch.Tensor:
    return torch.as_tensor(np.asarray(x, dtype=np.float64)).to(DT)


class _Topology:
    """Neighbour entries and triplets of a StructureSet (candidate independent)."""

    def __init__(self, structs, R2: float):
        self.structs = structs
        self.i, self.j, self.shift, self.sob = neighbor_list_set(structs, R2)
        self.N = structs.n_atoms
        self.S = structs.n_struct
        self.p, self.q = triplets(self.i, self.N)
        self.atom_struct = np.repeat(np.arange(self.S), structs.sizes())
        self.sizes = torch.as_tensor(structs.sizes().astype(np.float64))

    def reverse(self) -> np.ndarray:
        key = {(int(a), int(b), int(s0), int(s1), int(s2)): e for e, (a, b, (s0, s1, s2))
               in enumerate(zip(self.i, self.j, self.shift))}
        return np.array([key[(int(b), int(a), -int(s0), -int(s1), -int(s2))]
                         for a, b, (s0, s1, s2) in zip(self.i, self.j, self.shift)], dtype=np.int64)

    def bond_vectors(self, pos: torch.Tensor, eps: Optional[torch.Tensor] = None):
        cell = torch.as_tensor(self.structs.cell)
        T = torch.einsum("ek,ekl->el", torch.as_tensor(self.shift).to(DT), cell[self.sob])
        d = pos[self.j] + T - pos[self.i]
        if eps is not None:
            Fd = torch.eye(3, dtype=DT)[None] + eps[self.sob]
            d = torch.einsum("emn,en->em", Fd, d)
        return d


def _forward(top: _Topology, x: torch.Tensor, R1: float, R2: float, create_graph: bool):
    pos = torch.as_tensor(top.structs.pos).clone().requires_grad_(True)
    eps = torch.zeros(top.S, 3, 3, dtype=DT, requires_grad=True)
    d = top.bond_vectors(pos, eps)
    U = site_energies(d, top.i, top.p, top.q, top.N, x, R1, R2)
    E = torch.zeros(top.S, dtype=DT).index_add(0, torch.as_tensor(top.atom_struct), U)
    gpos, geps = torch.autograd.grad(E.sum(), (pos, eps), create_graph=create_graph)
    F = -gpos                                   # F_i = -dE/dr_i
    Wfull = -geps                               # W_mn = -dE/d eps_mn
    W6 = torch.stack([Wfull[:, a, b] for a, b in VIRIAL6], dim=1)
    return E, F, W6, U


def evaluate_set(structs, x, R1: float, R2: float, atom_virial: bool = False,
                 velocities: Optional[np.ndarray] = None, topology: Optional["_Topology"] = None):
    """Energy [S], forces [N,3], virial [S,6] (xx yy zz yz zx xy), site energies [N];
    optionally per-atom virial [N,3,3] and heat current [3].  All eV / A units.
    ``topology`` (from ``topology(structs, R2)``) reuses the neighbour entries
    of earlier calls on the same structures."""
    top = topology or _Topology(structs, R2)
    xt = _as_x(x)
    E, F, W6, U = _forward(top, xt, R1, R2, create_graph=False)
    out = {"E": E.detach().numpy(), "F": F.detach().numpy(), "W6": W6.detach().numpy(),
           "U": U.detach().numpy(), "n_bonds": int(top.i.shape[0]),
           "n_triplets": int(top.p.shape[0])}
    if atom_virial or velocities is not None:
        Wi = per_atom_virial(top, xt, R1, R2)
        out["Wi"] = Wi
        if velocities is not None:
            out["J"] = np.einsum("imn,in->m", Wi, np.asarray(velocities, dtype=np.float64))
    return out


def per_atom_virial(top: _Topology, x: torch.Tensor, R1: float, R2: float) -> np.ndarray:
    """W_i[m, n] = sum_j d_ij[m] * dU_j/dd_ji[n] (the per-atom virial of the cited
    force/virial formulas; sums to the total virial).  Each U_j depends only on the
    bond vectors leaving j, so dE/dd_e = dU_centre(e)/dd_e."""
    pos = torch.as_tensor(top.structs.pos)
    d = top.bond_vectors(pos).detach().clone().requires_grad_(True)
    U = site_energies(d, top.i, top.p, top.q, top.N, x, R1, R2)
    G = torch.autograd.grad(U.sum(), d)[0].numpy()
    rev = top.reverse()
    dn = d.detach().numpy()
    Wi = np.zeros((top.N, 3, 3))
    np.add.at(Wi, top.i, np.einsum("em,en->emn", dn, G[rev]))
    return Wi


def evaluate(pos, cell, x, R1: float, R2: float, **kw):
    """Single-structure convenience wrapper of ``evaluate_set``."""
    from workloads import make_set
    return evaluate_set(make_set([(pos, cell)]), x, R1, R2, **kw)


def _relative_rmse(residual_sq: torch.Tensor, norm_sq: torch.Tensor) -> torch.Tensor:
    """sqrt(R / Q) with its derivative taken as 0 where R = 0 (Sec. III.B)."""
    pos = residual_sq > 0
    safe = torch.where(pos, residual_sq, torch.ones_like(residual_sq))
    return torch.where(pos, torch.sqrt(safe / norm_sq), torch.zeros_like(residual_sq))


def _fitness_terms(top: _Topology, x: torch.Tensor, refs, weights, R1, R2, create_graph):
    e_ref = torch.as_tensor(np.asarray(refs["e"], dtype=np.float64))
    w_ref = torch.as_tensor(np.asarray(refs["w"], dtype=np.float64))
    f_ref = torch.as_tensor(np.asarray(refs["f"], dtype=np.float64))
    E, F, W6, _ = _forward(top, x, R1, R2, create_graph=create_graph)
    e = E / top.sizes
    w = W6 / top.sizes[:, None]
    Ze = _relative_rmse(((e - e_ref) ** 2).sum(), (e_ref ** 2).sum())
    Zv = _relative_rmse(((w - w_ref) ** 2).sum(), (w_ref ** 2).sum())
    Zf = _relative_rmse(((F - f_ref) ** 2).sum(), (f_ref ** 2).sum())
    we, wv, wf = (float(v) for v in weights)
    Z = we * Ze + wv * Zv + wf * Zf
    return torch.stack([Z, Ze, Zv, Zf])


def fitness(structs, X, refs, weights=(1.0, 1.0, 1.0), R1: float = 2.8, R2: float = 3.2,
            topology: Optional[_Topology] = None) -> np.ndarray:
    """Z, Z_e, Z_v, Z_f (Sec. III.B) for each parameter set in X [P,6] -> [P,4].

    refs: {"e": [S] eV/atom, "w": [S,6] eV/atom (xx yy zz yz zx xy), "f": [N,3] eV/A}."""
    top = topology or _Topology(structs, R2)
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    out = np.zeros((X.shape[0], 4))
    for c in range(X.shape[0]):
        out[c] = _fitness_terms(top, _as_x(X[c]), refs, weights, R1, R2, False).detach().numpy()
    return out


def fitness_grad(structs, X, refs, weights=(1.0, 1.0, 1.0), R1: float = 2.8, R2: float = 3.2,
                 topology: Optional[_Topology] = None):
    """(Z [P,4], dZ/dx [P,6]); the derivative of Z with respect to the phenotype x."""
    top = topology or _Topology(structs, R2)
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    Z = np.zeros((X.shape[0], 4))
    G = np.zeros((X.shape[0], X.shape[1]))
    for c in range(X.shape[0]):
        xt = _as_x(X[c]).clone().requires_grad_(True)
        terms = _fitness_terms(top, xt, refs, weights, R1, R2, True)
        (g,) = torch.autograd.grad(terms[0], xt)
        Z[c] = terms.detach().numpy()
        G[c] = g.numpy()
    return Z, G


def reference_data(structs, x, R1: float = 2.8, R2: float = 3.2):
    """Per-atom energies, per-atom virials and forces of parameter set x, in the
    layout the fitness uses: {"e": [S], "w": [S,6], "f": [N,3]}."""
    out = evaluate_set(structs, x, R1, R2)
    sizes = structs.sizes().astype(np.float64)
    return {"e": out["E"] / sizes, "w": out["W6"] / sizes[:, None], "f": out["F"]}


def topology(structs, R2: float) -> _Topology:
    return _Topology(structs, R2)


# ----------------------------------------------------------------------------
# Sampled per-atom quantities in large periodic cells
# ----------------------------------------------------------------------------

def local_forces(pos: np.ndarray, cell: np.ndarray, x, atoms: Sequence[int], R1: float,
                 R2: float):
    """Force, site energy and per-atom virial of selected atoms of a large cell.

    F_m = -dE/dr_m involves only U_m and the U_j of m's neighbours, and those
    depend only on atoms within 2 R2 of m.  Each sampled atom is therefore
    evaluated on the cluster of atoms (minimum image, valid because every
    perpendicular cell width exceeds 4 R2 + 2) within 2 R2 + 1 A of it."""
    pos = np.asarray(pos, dtype=np.float64)
    cell = np.asarray(cell, dtype=np.float64)
    if np.min(perpendicular_widths(cell)) <= 4.0 * R2 + 2.0:
        raise ValueError("cell too small for the cluster evaluation; use evaluate_set")
    inv = np.linalg.inv(cell)
    xt = _as_x(x)
    rc = 2.0 * R2 + 1.0
    F = np.zeros((len(atoms), 3))
    U = np.zeros(len(atoms))
    Wi = np.zeros((len(atoms), 3, 3))
    for k, m in enumerate(atoms):
        ds = (pos - pos[m]) @ inv
        ds -= np.round(ds)
        rel = ds @ cell
        sel = np.nonzero(np.einsum("ij,ij->i", rel, rel) < rc * rc)[0]
        sel = np.concatenate([[m], sel[sel != m]])
        local = rel[sel]                          # cluster coordinates, atom m at origin
        n = local.shape[0]
        # Non-periodic neighbour entries inside the cluster, by brute force.
        dd = local[None, :, :] - local[:, None, :]
        r2 = np.einsum("ijk,ijk->ij", dd, dd)
        ii, jj = np.nonzero((r2 < R2 * R2) & ~np.eye(n, dtype=bool))
        nbr_m = set(jj[ii == 0].tolist())
        centres = np.array(sorted({0} | nbr_m))
        keep = np.isin(ii, centres)
        ii, jj = ii[keep], jj[keep]
        order = np.lexsort((jj, ii))
        ii, jj = ii[order], jj[order]
        p, q = triplets(ii, n)
        lpos = torch.as_tensor(local).clone().requires_grad_(True)
        d = lpos[jj] - lpos[ii]
        Us = site_energies(d, ii, p, q, n, xt, R1, R2)
        Eloc = Us[torch.as_tensor(centres)].sum()
        (g,) = torch.autograd.grad(Eloc, lpos)
        F[k] = -g[0].numpy()
        U[k] = float(Us[0].detach())
        # per-atom virial of m: sum_j d_mj (x) dU_j/dd_jm
        dleaf = d.detach().clone().requires_grad_(True)
        Us2 = site_energies(dleaf, ii, p, q, n, xt, R1, R2)
        (G,) = torch.autograd.grad(Us2.sum(), dleaf)
        for e in np.nonzero(ii == 0)[0]:
            j = jj[e]
            rev = np.nonzero((ii == j) & (jj == 0))[0]
            assert rev.shape[0] == 1
            Wi[k] += np.outer(dleaf[e].detach().numpy(), G[rev[0]].numpy())
    return {"F": F, "U": U, "Wi": Wi}


# ----------------------------------------------------------------------------
# Closed form for the perfect diamond lattice
# ----------------------------------------------------------------------------

def diamond_closed_form(x, a: float, R1: float = 2.8, R2: float = 3.2) -> float:
    """Energy per atom of perfect diamond with lattice constant a.

    Every atom has four neighbours at r = sqrt(3) a / 4 (second shell at
    a/sqrt(2) = 3.84 A > R2 for a near 5.43), and each bond sees the other three
    at cos(theta) = -1/3, so zeta = 3 f_C(r) beta (-1/3 - h)^2 and
    U_i = 4 * 1/2 * f_C(r) [f_R - b f_A].  With S = 2 the pair part is the Morse
    form D0 [exp(-2 alpha (r - r0)) - 2 b exp(-alpha (r - r0))]."""
    D0, alpha, r0, beta, n, h = (float(v) for v in x)
    r = math.sqrt(3.0) * a / 4.0
    if a / math.sqrt(2.0) < R2:
        raise ValueError("second neighbour shell inside the cutoff")
    if r <= R1:
        fc = 1.0
    elif r >= R2:
        fc = 0.0
    else:
        fc = 0.5 * (1.0 + math.cos(math.pi * (r - R1) / (R2 - R1)))
    zeta = 3.0 * fc * beta * (-1.0 / 3.0 - h) ** 2
    b = (1.0 + zeta ** n) ** (-1.0 / (2.0 * n)) if zeta > 0 else 1.0
    e1 = math.exp(-alpha * (r - r0))
    return 2.0 * fc * D0 * (e1 * e1 - 2.0 * b * e1)
