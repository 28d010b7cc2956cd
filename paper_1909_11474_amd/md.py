"""Molecular dynamics on the GPU evaluation path (the potential's application,
Sec. IV.C: equilibrium MD and homogeneous non-equilibrium MD of diamond Si).

One structure (a periodic cell) per run.  A step is velocity Verlet:
  mt_md_kick(dt/2), mt_md_drift(dt), position update,
  tersoff_eval (forces, virial, per-atom virial, heat current), mt_md_kick(dt/2),
then, with a thermostat, a velocity rescaling toward the target temperature
(Berendsen: lambda^2 = 1 + dt/tau (T0/T - 1)).  With a driving force F_e the
kicks add F_ext,i = W_i^T F_e minus its mean (HNEMD); the heat current J of
every step is kept for the thermal-conductivity estimate
kappa = <J> . F_e / (T V |F_e|^2) (Sec. IV.C).

The position update rebuilds the neighbour lists (mt_set_update_positions)
when skin = 0; with a Verlet skin the lists hold pairs within R2 + skin and
only the bond geometry is recomputed (mt_set_update_geometry) until some atom
has moved skin/2 since the last rebuild (mt_md_max_disp).

Every step runs in the library's kernels; the host keeps only per-step
scalars (potential energy, kinetic sums, J and the skin's displacement check),
read back with one copy.  Inside run() without a thermostat the next step's
first kick, drift and displacement check are issued before that copy, so a
step waits on the host once instead of twice; the arithmetic and its order
are unchanged.  The library calls' argument lists are marshalled once at
construction, and the run uses the torch stream that is current then.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from . import api

KB_EV = 8.617333262e-5           # Boltzmann constant (eV/K)
MV2_TO_EV = 103.642691           # 1 u A^2 / fs^2 in eV

# natural silicon: 28Si, 29Si, 30Si (mass in u, abundance)
SI_ISOTOPES = ((27.97692653, 0.9223), (28.97649472, 0.0467), (29.97377022, 0.0310))


def isotope_masses(n: int, rng: np.random.Generator) -> np.ndarray:
    """Masses of n Si atoms drawn with the natural isotope abundances (u)."""
    m = np.array([v for v, _ in SI_ISOTOPES])
    p = np.array([a for _, a in SI_ISOTOPES])
    return m[rng.choice(len(m), size=n, p=p / p.sum())]


class MD:
    """Velocity-Verlet MD of one periodic cell with the Tersoff potential x
    ([6] minimal or [9] Tersoff form), float64 state on the GPU."""

    def __init__(self, pos, cell, x, masses, velocities, dt: float, R1: float = 2.8, R2: float = 3.2,
                 precision: str = "fp64", fe: Optional[Sequence[float]] = None,
                 thermostat: Optional[tuple] = None, max_nbr: int = L.MT_MAX_NBR,
                 skin: float = 0.0):
        pos = np.asarray(pos, dtype=np.float64)
        self.N = pos.shape[0]
        self.cell = np.asarray(cell, dtype=np.float64)
        self.volume = abs(float(np.linalg.det(self.cell)))
        self.dt = float(dt)
        self.ts = api.TersoffSet(pos, self.cell[None], [0, self.N], R1, R2, max_nbr)
        self._lib, self.dev = self.ts._lib, self.ts.device
        kw = dict(dtype=torch.float64, device=self.dev)
        x = np.asarray(x, dtype=np.float64)
        self.x = torch.as_tensor(x[None], **kw).contiguous()
        self._eval = self._lib.tersoff_eval_tf if x.shape[0] == 9 else self._lib.tersoff_eval
        self.prec = api._prec(precision)
        self.pos = torch.as_tensor(pos.T.copy(), **kw).contiguous()           # [3][N]
        self.vel = torch.as_tensor(np.asarray(velocities, np.float64).T.copy(), **kw).contiguous()
        m = np.asarray(masses, dtype=np.float64)
        self.mass = torch.as_tensor(m, **kw)
        self.inv_mass = torch.as_tensor(1.0 / m, **kw)
        # per-step scalars in one buffer: E [1][1], J [1][3], kinetic sums [4],
        # squared largest displacement since the last list build [1]
        self._sc = torch.zeros(9, **kw)
        self._sc_host = torch.empty(9, dtype=torch.float64, pin_memory=True)
        self._sc_np = self._sc_host.numpy()
        self.E = self._sc[0:1].view(1, 1)
        self.J = self._sc[1:4].view(1, 3)
        self.kin = self._sc[4:8]
        self.disp = self._sc[8:9]
        self._ahead = False               # next step's first half already issued
        self.F = torch.empty(1, 3, self.N, **kw)
        self.W = torch.empty(1, 1, 6, **kw)
        self.Wi = torch.empty(1, 9, self.N, **kw)
        self.fe = None if fe is None else (ctypes.c_double * 3)(*[float(v) for v in fe])
        self.fe_vec = None if fe is None else np.asarray(fe, dtype=np.float64)
        self.thermostat = thermostat       # (T0 in K, tau in fs) or None
        self.step_count = 0
        self.skin = float(skin)
        self.rebuilds = 0
        self._tstream = torch.cuda.current_stream(self.dev)
        self._st = ctypes.c_void_p(self._tstream.cuda_stream)
        if self.skin > 0:
            L.check(self._lib.mt_set_list_skin(self.ts._handle, self.skin, self._st), "mt_set_list_skin")
            self.ref = self.pos.clone()
        self._marshal()
        self._forces()

    # -- library calls -------------------------------------------------------------
    def _p(self, t):
        return ctypes.c_void_p(t.data_ptr())

    def _marshal(self):
        """Argument lists of the per-step calls (every buffer is allocated once)."""
        P, st, drive = self._p, self._st, self.fe is not None
        self._a_forces = (self.ts._handle, P(self.x), 1, self.prec, L.MT_BATCHED, P(self.E), P(self.F),
                          P(self.W), P(self.Wi), P(self.vel), P(self.J), st)
        self._a_kick = (self.N, P(self.vel), P(self.F), P(self.Wi) if drive else None,
                        P(self.W) if drive else None, self.fe if drive else None, P(self.inv_mass),
                        ctypes.c_double(0.5 * self.dt), st)
        self._a_drift = (self.N, P(self.pos), P(self.vel), ctypes.c_double(self.dt), st)
        self._a_kinetic = (self.N, P(self.vel), P(self.mass), P(self.kin), st)
        self._a_geometry = (self.ts._handle, P(self.pos), st)
        if self.skin > 0:
            self._a_disp = (self.N, P(self.pos), P(self.ref), P(self.disp), st)
            self._disp_limit = (0.5 * self.skin) ** 2

    def _forces(self):
        L.check(self._eval(*self._a_forces), "tersoff_eval")

    def _kick(self):
        L.check(self._lib.mt_md_kick(*self._a_kick), "mt_md_kick")

    def _first_half(self):
        """Kick, drift and, with a skin, the displacement check (on the GPU)."""
        self._kick()
        L.check(self._lib.mt_md_drift(*self._a_drift), "mt_md_drift")
        if self.skin > 0:
            L.check(self._lib.mt_md_max_disp(*self._a_disp), "mt_md_max_disp")

    def _read_scalars(self):
        with torch.cuda.stream(self._tstream):
            self._sc_host.copy_(self._sc)                     # synchronous

    def _update_positions(self):
        """Bond geometry at the drifted positions; the lists are rebuilt when the
        displacement read back with the step's scalars reaches skin/2."""
        if self.skin > 0:
            if float(self._sc_np[8]) < self._disp_limit:
                L.check(self._lib.mt_set_update_geometry(*self._a_geometry), "mt_set_update_geometry")
                return
            with torch.cuda.stream(self._tstream):
                self.ref.copy_(self.pos)
        L.check(self._lib.mt_set_update_positions(*self._a_geometry), "mt_set_update_positions")
        self.rebuilds += 1

    def kinetic(self):
        """(kinetic energy in eV, total momentum [3] in u A/fs)."""
        L.check(self._lib.mt_md_kinetic(*self._a_kinetic), "mt_md_kinetic")
        with torch.cuda.stream(self._tstream):
            k = self.kin.cpu().numpy()
        return 0.5 * k[0] * MV2_TO_EV, k[1:].copy()

    def temperature(self, ekin: float) -> float:
        return 2.0 * ekin / (3.0 * self.N * KB_EV)

    # -- stepping ------------------------------------------------------------------
    def step(self, _issue_next: bool = False) -> dict:
        if not self._ahead:
            self._first_half()
            if self.skin > 0:
                self._read_scalars()                          # the displacement
        self._ahead = False
        self._update_positions()
        self._forces()
        self._kick()
        L.check(self._lib.mt_md_kinetic(*self._a_kinetic), "mt_md_kinetic")
        # without a thermostat the next step's first half needs nothing from
        # the host: issue it before the read-back (it writes only velocities,
        # positions and the displacement slot, not E, J or the kinetic sums)
        if _issue_next and self.thermostat is None:
            self._first_half()
            self._ahead = True
        self._read_scalars()
        sc = self._sc_np
        epot, J, ekin, p = float(sc[0]), sc[1:4].copy(), 0.5 * sc[4] * MV2_TO_EV, sc[5:8].copy()
        T = self.temperature(ekin)
        if self.thermostat is not None:
            T0, tau = self.thermostat
            lam = np.sqrt(max(1.0 + self.dt / tau * (T0 / max(T, 1e-12) - 1.0), 0.0))
            L.check(self._lib.mt_md_scale(self.N, self._p(self.vel), float(lam), self._st), "mt_md_scale")
            ekin, p, T = ekin * lam * lam, p * lam, T * lam * lam
        self.step_count += 1
        return {"step": self.step_count, "epot": epot, "ekin": ekin, "etot": epot + ekin, "T": T,
                "momentum": p, "J": J}

    def run(self, n: int, every: int = 1) -> list:
        out = []
        for k in range(n):
            rec = self.step(_issue_next=k + 1 < n)
            if (k + 1) % every == 0:
                out.append(rec)
        return out

    def positions(self) -> np.ndarray:
        return self.pos.t().cpu().numpy().copy()

    def velocities(self) -> np.ndarray:
        return self.vel.t().cpu().numpy().copy()

    def external_power(self) -> float:
        """sum_i F_ext,i . v_i (eV/fs) of the current state, before the mean is
        removed; equals F_e . J."""
        Wi = self.Wi[0].cpu().numpy().reshape(3, 3, self.N)
        v = self.vel.cpu().numpy()
        return float(np.einsum("a,abi,bi->", self.fe_vec, Wi, v))

    def close(self):
        self.ts.close()


def kappa_hnemd(J_mean: np.ndarray, fe: Sequence[float], T: float, volume: float) -> float:
    """Thermal conductivity along F_e from the time-averaged heat current:
    kappa = <J> . F_e / (T V |F_e|^2), J in eV A/fs, F_e in 1/A, T in K, V in A^3;
    returned in W/(m K)."""
    fe = np.asarray(fe, dtype=np.float64)
    k = float(np.dot(J_mean, fe)) / (T * volume * float(np.dot(fe, fe)))   # eV/(fs A K)
    return k * 1.602176634e-19 / 1e-15 / 1e-10                              # W/(m K)
