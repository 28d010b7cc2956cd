"""Pins of the oracle's velocity-Verlet MD (oracle/md.py): second-order energy
conservation, time reversibility, momentum conservation under the HNEMD
driving force, and the power identity sum_i F_ext,i . v_i = F_e . J that
defines the driving force (Sec. IV.C)."""
import numpy as np
import pytest

import workloads as W
from oracle import md as M

X = np.array(W.TABLE2_X)


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def thermal_cell(seed, T=600.0):
    pos, cell = W.diamond(1, 1, 1)
    g = rng(seed)
    pos = W.displace(g, pos, 0.03)
    m = np.full(pos.shape[0], W.M_SI_AMU)
    v = g.normal(0.0, np.sqrt(W.KB_EV * T / (m[:, None] * W.AMU_A2_FS2_EV)), size=pos.shape)
    v -= (m[:, None] * v).sum(0) / m.sum()
    return pos, cell, m, v


def test_energy_error_is_second_order_in_the_time_step():
    pos, cell, m, v = thermal_cell(1)
    spread = []
    for dt in (1.0, 0.5):
        _, _, rec = M.velocity_verlet(pos, v, m, cell, X, dt, int(40 / dt))
        e = np.array([r["epot"] + r["ekin"] for r in rec])
        spread.append(np.ptp(e))
    assert spread[0] < 1e-3 * 8                     # eV over 8 atoms at 1 fs
    assert 3.0 < spread[0] / spread[1] < 5.0        # ~ dt^2


def test_time_reversibility():
    pos, cell, m, v = thermal_cell(2)
    p1, v1, _ = M.velocity_verlet(pos, v, m, cell, X, 1.0, 20)
    p2, v2, _ = M.velocity_verlet(p1, -v1, m, cell, X, 1.0, 20)
    assert np.abs(p2 - pos).max() < 1e-9
    assert np.abs(v2 + v).max() < 1e-10


def test_driving_force_conserves_momentum_and_its_power_is_fe_dot_j():
    pos, cell, m, v = thermal_cell(3)
    fe = np.array([0.0, 0.0, 2e-3])
    p1, v1, rec = M.velocity_verlet(pos, v, m, cell, X, 1.0, 15, fe=fe)
    mom = np.array([r["momentum"] for r in rec])
    assert np.abs(mom).max() < 1e-12
    Wi = rec[-1]["Wi"]
    ext = np.einsum("a,iab->ib", fe, Wi)
    assert abs(np.sum(ext * v1) - fe @ M.heat_current(Wi, v1)) < 1e-14 * (1 + abs(fe @ M.heat_current(Wi, v1)))
    # the mean-free driving force changes the trajectory
    p0, _, _ = M.velocity_verlet(pos, v, m, cell, X, 1.0, 15)
    assert np.abs(p1 - p0).max() > 1e-8
