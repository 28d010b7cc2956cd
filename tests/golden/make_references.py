"""Write the reference data of the benchmark workloads with the float64 oracle.

    python tests/golden/make_references.py

For each workload that fits a hidden parameter set (the GA batch of 100
strained 64-atom cells, and the uneven set of 300 structures of 8-512 atoms
that both the uneven-batching and the gradient workloads use), the oracle
evaluates the hidden set on every structure and stores, in the layout of the
Sec. III.B fitness: e [S] energy per atom (eV/atom), w [S, 6] virial per atom
(eV/atom, xx yy zz yz zx xy), f [N, 3] forces (eV/A), with the workload's
seeds and sizes so that a reader can check the file belongs to the inputs it
is used with.  Only oracle/ and the seeded input generators are called.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W                      # noqa: E402
from oracle import tersoff as T            # noqa: E402

FILES = {"config2": "references_ga_batch.npz", "config3": "references_uneven.npz"}


def write(name, wl):
    s = wl.structs
    refs = T.reference_data(s, wl.hidden_x, wl.R1, wl.R2)
    path = os.path.join(HERE, FILES[name])
    np.savez_compressed(path, e=refs["e"], w=refs["w"], f=refs["f"], hidden_x=wl.hidden_x,
                        sizes=s.sizes(), seeds=np.array([wl.seeds["structures"], wl.seeds["hidden"]]),
                        R=np.array([wl.R1, wl.R2]))
    print(f"{path}: {s.n_struct} structures, {s.n_atoms} atoms")


if __name__ == "__main__":
    write("config2", W.config2())
    write("config3", W.config3())
