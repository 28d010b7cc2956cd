"""Velocity-Verlet molecular dynamics with the oracle's forces (test
infrastructure only; imported by tests/ and nothing in the product path).

The potential's application (Sec. IV.C) runs equilibrium MD and homogeneous
non-equilibrium MD (HNEMD) of diamond Si.  Written out plainly:

  v <- v + dt/2 a,   r <- r + dt v,   (forces at the new r),   v <- v + dt/2 a,
  a_i = (F_i + F_ext,i - mean_j F_ext,j) / (m_i 103.642691)   [A/fs^2, F in eV/A, m in u]

with the HNEMD driving force F_ext,i = W_i^T F_e from the per-atom virial W_i
(the oracle's, from bond-vector gradients).  Its power sum_i F_ext,i . v_i is
F_e . J for the heat current J = sum_i W_i v_i; removing the mean keeps the
total momentum.  Without F_e the scheme is plain NVE velocity Verlet.
"""
from __future__ import annotations

import numpy as np

from . import tersoff as T

MV2_TO_EV = 103.642691          # 1 u A^2 / fs^2 in eV


def forces(pos, cell, x, R1=2.8, R2=3.2):
    """(E, F [N,3], W_i [N,3,3]) of one periodic cell."""
    out = T.evaluate(pos, cell, x, R1, R2, atom_virial=True)
    return float(out["E"][0]), out["F"], out["Wi"]


def driving_force(Wi, fe):
    """F_ext,i = W_i^T F_e minus its mean over atoms."""
    ext = np.einsum("a,iab->ib", np.asarray(fe, dtype=np.float64), Wi)
    return ext - ext.mean(axis=0)


def heat_current(Wi, vel):
    """J = sum_i W_i v_i (eV A/fs)."""
    return np.einsum("iab,ib->a", Wi, vel)


def kinetic_energy(vel, masses):
    return 0.5 * float(np.sum(masses[:, None] * vel * vel)) * MV2_TO_EV


def velocity_verlet(pos, vel, masses, cell, x, dt, n_steps, fe=None, R1=2.8, R2=3.2):
    """n_steps of velocity Verlet from (pos, vel); returns the final positions,
    velocities and per-step records (E_pot, E_kin, momentum)."""
    pos = np.array(pos, dtype=np.float64)
    vel = np.array(vel, dtype=np.float64)
    m = np.asarray(masses, dtype=np.float64)[:, None] * MV2_TO_EV
    E, F, Wi = forces(pos, cell, x, R1, R2)
    rec = []
    for _ in range(n_steps):
        Ft = F + (driving_force(Wi, fe) if fe is not None else 0.0)
        vel = vel + 0.5 * dt * Ft / m
        pos = pos + dt * vel
        E, F, Wi = forces(pos, cell, x, R1, R2)
        Ft = F + (driving_force(Wi, fe) if fe is not None else 0.0)
        vel = vel + 0.5 * dt * Ft / m
        rec.append({"epot": E, "ekin": kinetic_energy(vel, masses),
                    "momentum": (np.asarray(masses)[:, None] * vel).sum(axis=0), "Wi": Wi})
    return pos, vel, rec
