"""Brute-force periodic neighbour enumeration (oracle; test infrastructure only).

The cutoff function of Sec. II.A (cosine cutoff f_C) vanishes for r >= R2, so
an atom interacts with every periodic image of every atom closer than R2.  In
small or sheared cells several images of the same atom can be neighbours, and
an atom can neighbour its own image, so minimum-image conventions are not
used: for each pair (i, j) every lattice translation T = n1 a + n2 b + n3 c that
could bring r_j + T within R2 of r_i is tried.

For fractional coordinates s and perpendicular cell widths w_k = V / |a_l x a_m|,
a translation n can only give |r_j + T - r_i| < R2 if
|s_j,k - s_i,k + n_k| * w_k < R2 for every axis k.  The enumeration range per
axis is therefore floor(-R2/w_k - max ds_k) .. ceil(R2/w_k - min ds_k).
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def perpendicular_widths(cell: np.ndarray) -> np.ndarray:
    a, b, c = cell
    vol = abs(float(np.dot(a, np.cross(b, c))))
    return np.array([vol / np.linalg.norm(np.cross(b, c)),
                     vol / np.linalg.norm(np.cross(c, a)),
                     vol / np.linalg.norm(np.cross(a, b))])


def neighbor_list(pos: np.ndarray, cell: np.ndarray, R2: float):
    """All directed neighbour entries (i, j, n) with 0 < |r_j + n.cell - r_i| < R2.

    Returns (i [nb] int64, j [nb] int64, shift [nb, 3] int64), sorted by
    (i, j, n1, n2, n3).  Raises ValueError for coincident atoms (distance 0).
    """
    pos = np.asarray(pos, dtype=np.float64)
    cell = np.asarray(cell, dtype=np.float64)
    n = pos.shape[0]
    frac = pos @ np.linalg.inv(cell)
    widths = perpendicular_widths(cell)
    ds = frac[None, :, :] - frac[:, None, :]            # [i, j, 3]
    lo = np.floor(-R2 / widths - ds.max(axis=(0, 1))).astype(int)
    hi = np.ceil(R2 / widths - ds.min(axis=(0, 1))).astype(int)
    out_i, out_j, out_s = [], [], []
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    for n1 in range(lo[0], hi[0] + 1):
        for n2 in range(lo[1], hi[1] + 1):
            for n3 in range(lo[2], hi[2] + 1):
                T = n1 * cell[0] + n2 * cell[1] + n3 * cell[2]
                d = pos[None, :, :] + T[None, None, :] - pos[:, None, :]
                r2 = np.einsum("ijk,ijk->ij", d, d)
                if (n1, n2, n3) == (0, 0, 0):
                    same = ii == jj
                    if np.any((r2 == 0.0) & ~same):
                        raise ValueError("coincident atoms")
                    mask = (r2 < R2 * R2) & ~same
                else:
                    if np.any(r2 == 0.0):
                        raise ValueError("atom coincides with a periodic image")
                    mask = r2 < R2 * R2
                if mask.any():
                    out_i.append(ii[mask])
                    out_j.append(jj[mask])
                    out_s.append(np.tile([n1, n2, n3], (int(mask.sum()), 1)))
    if not out_i:
        return (np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros((0, 3), np.int64))
    i = np.concatenate(out_i).astype(np.int64)
    j = np.concatenate(out_j).astype(np.int64)
    s = np.concatenate(out_s).astype(np.int64)
    order = np.lexsort((s[:, 2], s[:, 1], s[:, 0], j, i))
    return i[order], j[order], s[order]


def neighbor_list_naive(pos: np.ndarray, cell: np.ndarray, R2: float, nmax: int = 3):
    """Pure-Python triple loop over atoms and a fixed image box |n_k| <= nmax.

    Only for tiny inputs: it cross-checks the vectorised enumeration above.
    """
    out = []
    n = len(pos)
    for i in range(n):
        for j in range(n):
            for n1, n2, n3 in itertools.product(range(-nmax, nmax + 1), repeat=3):
                if i == j and (n1, n2, n3) == (0, 0, 0):
                    continue
                d = [pos[j][k] + n1 * cell[0][k] + n2 * cell[1][k] + n3 * cell[2][k] - pos[i][k]
                     for k in range(3)]
                r = math.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
                if 0.0 < r < R2:
                    out.append((i, j, n1, n2, n3))
    return sorted(out)


def neighbor_list_set(structs, R2: float):
    """Neighbour entries of every structure of a StructureSet, with global atom
    indices.  Returns (i, j, shift [nb,3], struct_of_bond [nb])."""
    I, J, Sh, St = [], [], [], []
    for s in range(structs.n_struct):
        pos, cell = structs.structure(s)
        i, j, sh = neighbor_list(pos, cell, R2)
        base = int(structs.offset[s])
        I.append(i + base)
        J.append(j + base)
        Sh.append(sh)
        St.append(np.full(i.shape[0], s, dtype=np.int64))
    return (np.concatenate(I), np.concatenate(J), np.concatenate(Sh, axis=0),
            np.concatenate(St))
