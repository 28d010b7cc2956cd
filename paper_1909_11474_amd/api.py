"""Python binding of the C ABI (include/mt_tersoff.h).

Only argument marshalling happens here: tensors are moved to the GPU in the
layouts the ABI documents and their data pointers are handed to the library,
together with the current HIP stream.  Every computation runs in the HIP
kernels of libmt_tersoff.so.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L

_PREC = {"fp64": L.MT_FP64, "fp32": L.MT_FP32_ACC64, L.MT_FP64: L.MT_FP64,
         L.MT_FP32_ACC64: L.MT_FP32_ACC64}
_SCHED = {"batched": L.MT_BATCHED, "plain": L.MT_PLAIN, L.MT_BATCHED: L.MT_BATCHED,
          L.MT_PLAIN: L.MT_PLAIN}


def _prec(p) -> int:
    try:
        return _PREC[p]
    except KeyError:
        raise ValueError(f"precision must be 'fp32' or 'fp64', got {p!r}") from None


def _sched(s) -> int:
    try:
        return _SCHED[s]
    except KeyError:
        raise ValueError(f"schedule must be 'batched' or 'plain', got {s!r}") from None


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class TersoffSet:
    """A set of periodic structures on one GPU, with neighbour lists and bond
    geometry built once, and optional reference data for the fitness.

    pos     [N, 3] Cartesian positions (A), structures concatenated
    cell    [S, 3, 3] lattice vectors as rows (A)
    offset  [S + 1] first atom of every structure, offset[S] = N
    """

    def __init__(self, pos, cell, offset, R1: float = 2.8, R2: float = 3.2,
                 max_nbr: int = L.MT_MAX_NBR, device=None):
        self._lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("TersoffSet needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self._handle = ctypes.c_void_p()
        off = np.ascontiguousarray(np.asarray(offset), dtype=np.int64)
        self.offset = off
        self.S = int(off.shape[0] - 1)
        self.N = int(off[-1])
        pos_t = torch.as_tensor(np.asarray(pos, dtype=np.float64) if not torch.is_tensor(pos) else pos)
        cell_t = torch.as_tensor(np.asarray(cell, dtype=np.float64) if not torch.is_tensor(cell) else cell)
        if tuple(pos_t.shape) != (self.N, 3):
            raise ValueError(f"pos must be [{self.N}, 3], got {tuple(pos_t.shape)}")
        if tuple(cell_t.shape) != (self.S, 3, 3):
            raise ValueError(f"cell must be [{self.S}, 3, 3], got {tuple(cell_t.shape)}")
        with torch.cuda.device(self.device):
            pos_soa = pos_t.to(torch.float64).t().contiguous().to(self.device)
            cell_d = cell_t.to(torch.float64).contiguous().to(self.device)
            rc = self._lib.mt_set_create(ctypes.byref(self._handle), self.S,
                                         off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                         _ptr(pos_soa), _ptr(cell_d), float(R1), float(R2),
                                         int(max_nbr), self._stream())
        L.check(rc, "mt_set_create")
        self.R1, self.R2 = float(R1), float(R2)
        self.sizes = np.diff(off)

    # -- plumbing ---------------------------------------------------------------
    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _x(self, x, widths=(6, 9)) -> torch.Tensor:
        """[P, 6] minimal-potential or [P, 9] Tersoff-form parameter sets."""
        xt = torch.as_tensor(x) if not torch.is_tensor(x) else x
        xt = xt.detach().to(device=self.device, dtype=torch.float64)
        if xt.dim() == 1:
            xt = xt[None]
        if xt.dim() != 2 or xt.shape[1] not in widths:
            want = " or ".join(f"[P, {w}]" for w in widths)
            raise ValueError(f"x must be {want}, got {tuple(xt.shape)}")
        return xt.contiguous()

    def close(self):
        if getattr(self, "_handle", None) is not None and self._handle.value:
            self._lib.mt_set_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- queries ----------------------------------------------------------------
    def stats(self) -> dict:
        out = (ctypes.c_int64 * 8)()
        L.check(self._lib.mt_set_stats(self._handle, out), "mt_set_stats")
        keys = ("n_struct", "n_atoms", "n_bonds", "n_triplets", "max_coordination",
                "max_atoms", "n_batched", "n_large")
        return {k: int(v) for k, v in zip(keys, out)}

    def neighbors(self):
        """(i, j, shift [nb, 3]) as numpy int64 arrays, grouped by centre atom."""
        nb = self.stats()["n_bonds"]
        with torch.cuda.device(self.device):
            i = torch.empty(max(nb, 1), dtype=torch.int32, device=self.device)
            j = torch.empty(max(nb, 1), dtype=torch.int32, device=self.device)
            sh = torch.empty(3 * max(nb, 1), dtype=torch.int32, device=self.device)
            L.check(self._lib.mt_set_neighbors(self._handle, _ptr(i), _ptr(j), _ptr(sh),
                                               self._stream()), "mt_set_neighbors")
            torch.cuda.current_stream(self.device).synchronize()
        shift = sh.view(3, -1)[:, :nb].t().cpu().numpy().astype(np.int64)
        return i[:nb].cpu().numpy().astype(np.int64), j[:nb].cpu().numpy().astype(np.int64), shift

    # -- reference data ---------------------------------------------------------
    def attach_reference(self, e_ref, w_ref, f_ref):
        """e_ref [S] eV/atom, w_ref [S, 6] eV/atom (xx yy zz yz zx xy), f_ref [N, 3] eV/A."""
        def dev(a, shape):
            t = torch.as_tensor(np.asarray(a, dtype=np.float64) if not torch.is_tensor(a) else a)
            t = t.to(torch.float64)
            if tuple(t.shape) != shape:
                raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
            return t
        e = dev(e_ref, (self.S,)).contiguous().to(self.device)
        w = dev(w_ref, (self.S, 6)).contiguous().to(self.device)
        f = dev(f_ref, (self.N, 3)).t().contiguous().to(self.device)
        with torch.cuda.device(self.device):
            L.check(self._lib.mt_set_attach_reference(self._handle, _ptr(e), _ptr(w), _ptr(f),
                                                      self._stream()), "mt_set_attach_reference")

    # -- evaluation -------------------------------------------------------------
    def tersoff_eval(self, x, precision="fp32", schedule="batched", energy=True, forces=True,
                     virial=True, atom_virial=False, velocities=None):
        """Energies [P,S], forces [P,N,3], virials [P,S,6], per-atom virials [P,N,3,3]
        and heat current [P,3] (when velocities [N,3] in A/fs are given).  x is
        [P, 6] (minimal potential) or [P, 9] (Tersoff form: tersoff_eval_tf)."""
        xt = self._x(x)
        P = xt.shape[0]
        kw = dict(dtype=torch.float64, device=self.device)
        out = {}
        with torch.cuda.device(self.device):
            E = torch.empty(P, self.S, **kw) if energy else None
            F = torch.empty(P, 3, self.N, **kw) if forces else None
            W = torch.empty(P, self.S, 6, **kw) if virial else None
            Wi = torch.empty(P, 9, self.N, **kw) if atom_virial else None
            vel = None
            J = None
            if velocities is not None:
                v = torch.as_tensor(np.asarray(velocities, dtype=np.float64) if not torch.is_tensor(velocities) else velocities)
                vel = v.to(torch.float64).t().contiguous().to(self.device)
                J = torch.empty(P, 3, **kw)
            name = "tersoff_eval_tf" if xt.shape[1] == 9 else "tersoff_eval"
            rc = getattr(self._lib, name)(self._handle, _ptr(xt), P, _prec(precision),
                                          _sched(schedule), _ptr(E), _ptr(F), _ptr(W), _ptr(Wi),
                                          _ptr(vel), _ptr(J), self._stream())
        L.check(rc, name)
        if E is not None:
            out["E"] = E
        if F is not None:
            out["F"] = F.transpose(1, 2)
        if W is not None:
            out["W"] = W
        if Wi is not None:
            out["Wi"] = Wi.view(P, 3, 3, self.N).permute(0, 3, 1, 2)
        if J is not None:
            out["J"] = J
        return out

    def fitness(self, x, weights=(1.0, 1.0, 1.0), precision="fp32", schedule="batched",
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """[P, 4] = Z, Z_e, Z_v, Z_f (device tensor, float64); x is [P, 6] or, for
        the Tersoff form (fitness_eval_tf), [P, 9]."""
        xt = self._x(x)
        P = xt.shape[0]
        w = (ctypes.c_double * 3)(*[float(v) for v in weights])
        with torch.cuda.device(self.device):
            Z = out if out is not None else torch.empty(P, 4, dtype=torch.float64, device=self.device)
            name = "fitness_eval_tf" if xt.shape[1] == 9 else "fitness_eval"
            rc = getattr(self._lib, name)(self._handle, _ptr(xt), P, w, _prec(precision),
                                          _sched(schedule), _ptr(Z), self._stream())
        L.check(rc, name)
        return Z

    def fitness_call(self, x: torch.Tensor, Z: torch.Tensor, weights=(1.0, 1.0, 1.0),
                     precision="fp32", schedule="batched") -> "FitnessCall":
        """A pre-marshalled fitness_eval(x -> Z) for repeated calls on the same
        device buffers (a GA generation loop): the arguments are converted once."""
        return FitnessCall(self, x, Z, weights, precision, schedule)

    def eval_call(self, x, precision="fp32", atom_virial=False, velocities=None) -> "EvalCall":
        """A pre-marshalled tersoff_eval (energies, forces, virials; per-atom
        virials and heat current on request) into buffers allocated once, for
        repeated force calls on the same parameters (molecular dynamics)."""
        return EvalCall(self, x, precision, atom_virial, velocities)

    def fitness_grad(self, x, weights=(1.0, 1.0, 1.0), precision="fp32"):
        """(Z [P, 4], dZ/dx [P, 6]) as device tensors; for Tersoff-form x [P, 9]
        (fitness_grad_tf) dZ/dx is [P, 9]."""
        xt = self._x(x)
        P, nx = xt.shape
        w = (ctypes.c_double * 3)(*[float(v) for v in weights])
        name = "fitness_grad_tf" if nx == 9 else "fitness_grad"
        with torch.cuda.device(self.device):
            Z = torch.empty(P, 4, dtype=torch.float64, device=self.device)
            G = torch.empty(P, nx, dtype=torch.float64, device=self.device)
            rc = getattr(self._lib, name)(self._handle, _ptr(xt), P, w, _prec(precision), _ptr(Z),
                                          _ptr(G), self._stream())
        L.check(rc, name)
        return Z, G

    def fitness_terms(self, x):
        """Per-structure terms of the last fitness call on this set with the
        parameter sets x (its P and form): dict of device float64 tensors
        e [P, S] (eV/atom), w [P, S, 6] (eV/atom) and rf [P, S] (squared force
        residual, eV^2/A^2)."""
        xt = self._x(x)
        P = xt.shape[0]
        with torch.cuda.device(self.device):
            e = torch.empty(P, self.S, dtype=torch.float64, device=self.device)
            w = torch.empty(P, self.S, 6, dtype=torch.float64, device=self.device)
            rf = torch.empty(P, self.S, dtype=torch.float64, device=self.device)
            rc = self._lib.fitness_terms(self._handle, _ptr(xt), P, _ptr(e), _ptr(w), _ptr(rf),
                                         self._stream())
        L.check(rc, "fitness_terms")
        return {"e": e, "w": w, "rf": rf}

    def profile(self, enable: bool = True):
        """Bracket each batched / adjoint kernel launch with HIP events."""
        L.check(self._lib.mt_profile_enable(self._handle, 1 if enable else 0), "mt_profile_enable")

    def profile_read(self):
        """{'batched': (ms, launches), 'adjoint': (ms, launches)} since the last read."""
        ms = (ctypes.c_double * 2)()
        n = (ctypes.c_int64 * 2)()
        L.check(self._lib.mt_profile_read(self._handle, ms, n), "mt_profile_read")
        return {"batched": (ms[0], int(n[0])), "adjoint": (ms[1], int(n[1]))}

    def profile_fitness_kernels(self, x, precision="fp32", reps: int = 100):
        """(ms per pass, launches per pass) of reps back-to-back passes of the
        batched fitness kernels for x [P, 6] or [P, 9], between one event pair."""
        xt = self._x(x)
        P, nx = xt.shape
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        with torch.cuda.device(self.device):
            rc = self._lib.mt_profile_fitness_kernels(self._handle, _ptr(xt), nx, P, _prec(precision),
                                                      int(reps), ctypes.byref(ms), ctypes.byref(n),
                                                      self._stream())
        L.check(rc, "mt_profile_fitness_kernels")
        return ms.value, int(n.value)

    def profile_fitness_launches(self, x, precision="fp32", reps: int = 100, max_launches: int = 16):
        """Each launch of the batched fitness plan timed alone, reps back to back:
        list of (ms per launch, coordination class) and, per structure, the index
        of the launch that evaluates it (-1: two-pass path)."""
        xt = self._x(x)
        P, nx = xt.shape
        ms = (ctypes.c_double * max_launches)()
        mc = (ctypes.c_int * max_launches)()
        sl = (ctypes.c_int * self.S)()
        n = ctypes.c_int()
        with torch.cuda.device(self.device):
            rc = self._lib.mt_profile_fitness_launches(self._handle, _ptr(xt), nx, P, _prec(precision),
                                                       int(reps), max_launches, ms, mc, sl,
                                                       ctypes.byref(n), self._stream())
        L.check(rc, "mt_profile_fitness_launches")
        return [(ms[k], mc[k]) for k in range(n.value)], list(sl)

    def autotune(self, P: int, precision="fp32", cache_path: Optional[str] = None):
        with torch.cuda.device(self.device):
            rc = self._lib.mt_autotune(self._handle, int(P), _prec(precision),
                                       cache_path.encode() if cache_path else None)
        L.check(rc, "mt_autotune")


class FitnessCall:
    """fitness_eval bound to fixed device tensors x [P, 6] (fitness_eval_tf for
    [P, 9]) and Z [P, 4] (float64, contiguous, on the set's device).  Calling it
    enqueues one evaluation on the current stream; the contents of x may change
    between calls."""

    def __init__(self, tset: TersoffSet, x: torch.Tensor, Z: torch.Tensor, weights, precision, schedule):
        if not (torch.is_tensor(x) and x.dtype == torch.float64 and x.is_contiguous()
                and x.device == tset.device and x.dim() == 2 and x.shape[1] in (6, 9)):
            raise ValueError("x must be a contiguous float64 [P, 6] or [P, 9] tensor on the set's device")
        P = x.shape[0]
        if not (torch.is_tensor(Z) and Z.dtype == torch.float64 and Z.is_contiguous()
                and Z.device == tset.device and tuple(Z.shape) == (P, 4)):
            raise ValueError("Z must be a contiguous float64 [P, 4] tensor on the set's device")
        self.tset, self.x, self.Z = tset, x, Z
        self._name = "fitness_eval_tf" if x.shape[1] == 9 else "fitness_eval"
        self._fn = getattr(tset._lib, self._name)
        self._w = (ctypes.c_double * 3)(*[float(v) for v in weights])
        self._args = (tset._handle, ctypes.c_void_p(x.data_ptr()), int(P), self._w,
                      _prec(precision), _sched(schedule), ctypes.c_void_p(Z.data_ptr()))

    def __call__(self, stream: Optional[torch.cuda.Stream] = None):
        s = stream if stream is not None else torch.cuda.current_stream(self.tset.device)
        rc = self._fn(*self._args, ctypes.c_void_p(s.cuda_stream))
        if rc:
            L.check(rc, self._name)
        return self.Z


class EvalCall:
    """tersoff_eval (or tersoff_eval_tf) bound to buffers allocated once.
    Calling it enqueues one evaluation on the current stream and returns the
    output tensors (overwritten by the next call)."""

    def __init__(self, tset: TersoffSet, x, precision, atom_virial, velocities):
        self.tset = tset
        self.x = tset._x(x)
        P = self.x.shape[0]
        kw = dict(dtype=torch.float64, device=tset.device)
        self.E = torch.empty(P, tset.S, **kw)
        self.F = torch.empty(P, 3, tset.N, **kw)
        self.W = torch.empty(P, tset.S, 6, **kw)
        self.Wi = torch.empty(P, 9, tset.N, **kw) if atom_virial else None
        self.vel = None
        self.J = None
        if velocities is not None:
            v = torch.as_tensor(np.asarray(velocities, dtype=np.float64)
                                if not torch.is_tensor(velocities) else velocities)
            self.vel = v.to(torch.float64).t().contiguous().to(tset.device)
            self.J = torch.empty(P, 3, **kw)
        self._name = "tersoff_eval_tf" if self.x.shape[1] == 9 else "tersoff_eval"
        self._fn = getattr(tset._lib, self._name)
        self._args = (tset._handle, _ptr(self.x), int(P), _prec(precision), L.MT_BATCHED,
                      _ptr(self.E), _ptr(self.F), _ptr(self.W), _ptr(self.Wi), _ptr(self.vel),
                      _ptr(self.J))

    def __call__(self, stream: Optional[torch.cuda.Stream] = None):
        s = stream if stream is not None else torch.cuda.current_stream(self.tset.device)
        rc = self._fn(*self._args, ctypes.c_void_p(s.cuda_stream))
        if rc:
            L.check(rc, self._name)
        out = {"E": self.E, "F": self.F.transpose(1, 2), "W": self.W}
        if self.Wi is not None:
            out["Wi"] = self.Wi.view(-1, 3, 3, self.tset.N).permute(0, 3, 1, 2)
        if self.J is not None:
            out["J"] = self.J
        return out


def from_structures(structs, R1: float = 2.8, R2: float = 3.2, max_nbr: int = L.MT_MAX_NBR,
                    device=None) -> TersoffSet:
    """Build a TersoffSet from an object with .pos [N,3], .cell [S,3,3], .offset [S+1]."""
    return TersoffSet(structs.pos, structs.cell, structs.offset, R1, R2, max_nbr, device)


class TersoffFitness(torch.autograd.Function):
    """Z(x) for a population x [P, 6] (or Tersoff-form [P, 9]) as a differentiable function.

    forward: fitness_eval, or fitness_grad when x requires a gradient;
    backward: grad_Z[:, None] * dZ/dx."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, tset: TersoffSet, weights: Sequence[float] = (1.0, 1.0, 1.0),
                precision: str = "fp32"):
        if ctx.needs_input_grad[0]:
            Z, G = tset.fitness_grad(x, weights, precision)
            ctx.save_for_backward(G.to(x.dtype).to(x.device))
        else:
            Z = tset.fitness(x, weights, precision)
        return Z[:, 0].to(x.device)

    @staticmethod
    def backward(ctx, grad_z: torch.Tensor):
        (G,) = ctx.saved_tensors
        return grad_z[:, None] * G, None, None, None


def tersoff_fitness(x: torch.Tensor, tset: TersoffSet, weights=(1.0, 1.0, 1.0), precision="fp32"):
    return TersoffFitness.apply(x, tset, tuple(weights), precision)
