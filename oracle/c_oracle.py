"""ctypes binding of the plain C float64 reference (``tersoff_c.c``) -- TEST
INFRASTRUCTURE ONLY, like the rest of this package.

The C code evaluates the same definitions as ``tersoff.py`` (Sec. II.A
Eqs. 1-9, Sec. II.B Eqs. 10-14, the fitness of Sec. III.B) with the forces and
virial written out by the chain rule instead of taken by autograd, one atom at
a time, with candidates shared out over OpenMP threads.  Its neighbour entries
come from this package's brute-force enumeration (``neighbors.py``).  The CPU
tests hold it to ``tersoff.py``; the benchmark times it as the CPU baseline.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

from .neighbors import neighbor_list_set

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tersoff_c.c")
LIB = os.path.join(HERE, "libtersoff_c.so")

_lib = None
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def build() -> str:
    """Compile the C reference (plain -O2, IEEE float64, OpenMP)."""
    cc = os.environ.get("CC", "gcc")
    tmp = LIB + ".tmp"
    subprocess.run([cc, "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", SRC, "-o", tmp, "-lm"],
                   check=True)
    os.replace(tmp, LIB)
    return LIB


def load(build_if_missing: bool = True):
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        if not build_if_missing:
            raise ImportError(f"{LIB} is missing")
        build()
    lib = ctypes.CDLL(LIB)
    lib.tc_evaluate.restype = ctypes.c_int
    lib.tc_evaluate.argtypes = [ctypes.c_int, ctypes.c_int, _i64p, _i64p, _f64p, _i64p, _f64p, ctypes.c_int,
                                ctypes.c_double, ctypes.c_double, _f64p, _f64p, _f64p]
    lib.tc_fitness.restype = ctypes.c_int
    lib.tc_fitness.argtypes = [ctypes.c_int, ctypes.c_int, _i64p, _i64p, _f64p, _i64p, ctypes.c_int, _f64p,
                               ctypes.c_int, ctypes.c_double, ctypes.c_double, _f64p, _f64p, _f64p, _f64p,
                               _f64p, ctypes.c_int]
    lib.tc_max_threads.restype = ctypes.c_int
    lib.tc_max_threads.argtypes = []
    _lib = lib
    return lib


class CTopology:
    """Neighbour entries of a StructureSet in the layout the C code reads:
    entries grouped by centre atom (CSR offsets), partner index and bond vector
    d = r_j + T - r_i."""

    def __init__(self, structs, R2: float, entries=None):
        """entries: (i, j, shift, struct_of_bond) from ``neighbor_list_set``
        when the caller already has them (e.g. the autograd oracle's topology)."""
        i, j, shift, sob = entries if entries is not None else neighbor_list_set(structs, R2)
        order = np.argsort(i, kind="stable")
        i, j, shift, sob = i[order], j[order], shift[order], sob[order]
        pos = np.asarray(structs.pos, dtype=np.float64)
        cell = np.asarray(structs.cell, dtype=np.float64)
        T = np.einsum("ek,ekl->el", shift.astype(np.float64), cell[sob])
        self.N = int(structs.n_atoms)
        self.S = int(structs.n_struct)
        self.start = np.concatenate([[0], np.cumsum(np.bincount(i, minlength=self.N))]).astype(np.int64)
        self.j = np.ascontiguousarray(j, dtype=np.int64)
        self.d = np.ascontiguousarray(pos[j] + T - pos[i], dtype=np.float64)
        self.atom_struct = np.repeat(np.arange(self.S, dtype=np.int64), structs.sizes())


def evaluate_set(structs, x, R1: float, R2: float, topology: Optional[CTopology] = None):
    """E [S], F [N,3], W6 [S,6] (xx yy zz yz zx xy) of one parameter set."""
    lib = load()
    top = topology or CTopology(structs, R2)
    x = np.ascontiguousarray(x, dtype=np.float64)
    full = 1 if x.shape[0] == 9 else 0
    E = np.zeros(top.S)
    F = np.zeros((top.N, 3))
    W = np.zeros((top.S, 6))
    rc = lib.tc_evaluate(top.N, top.S, top.start, top.j, top.d, top.atom_struct, x, full, R1, R2, E, F, W)
    if rc != 0:
        raise RuntimeError(f"tc_evaluate failed with {rc}")
    return {"E": E, "F": F, "W6": W}


def fitness(structs, X, refs, weights=(1.0, 1.0, 1.0), R1: float = 2.8, R2: float = 3.2,
            topology: Optional[CTopology] = None, threads: int = 0) -> np.ndarray:
    """Z, Z_e, Z_v, Z_f [P,4] (Sec. III.B); threads = 0: the OpenMP default."""
    lib = load()
    top = topology or CTopology(structs, R2)
    X = np.ascontiguousarray(np.atleast_2d(X), dtype=np.float64)
    full = 1 if X.shape[1] == 9 else 0
    Z = np.zeros((X.shape[0], 4))
    rc = lib.tc_fitness(top.N, top.S, top.start, top.j, top.d, top.atom_struct, X.shape[0], X, full, R1, R2,
                        np.ascontiguousarray(refs["e"], dtype=np.float64),
                        np.ascontiguousarray(refs["w"], dtype=np.float64),
                        np.ascontiguousarray(refs["f"], dtype=np.float64),
                        np.ascontiguousarray(weights, dtype=np.float64), Z, int(threads))
    if rc != 0:
        raise RuntimeError(f"tc_fitness failed with {rc}")
    return Z


def max_threads() -> int:
    return int(load().tc_max_threads())
