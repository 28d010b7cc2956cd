"""FP64 CPU oracle for the minimal Tersoff potential -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow reference that the GPU library is checked
against.  It is imported only by the test suite, by the package smoke check and
by the benchmark's CPU-baseline leg; the GPU library never imports, links or
calls it, and it shares no code with the GPU kernels.

What it computes, each item written out from the paper's definitions:

* neighbours: every (j, periodic image) within the outer cutoff of each atom,
  by brute-force image enumeration (``neighbors.py``);
* energy: the site-energy sum of Sec. II.A with the minimal angular function
  of Sec. II.B and the (D0, alpha, r0, S = 2) reparametrisation (``tersoff.py``);
* forces, virial and per-atom virial: derivatives of that energy, taken by
  PyTorch autograd in float64 (forces = -dE/dr, virial = -dE/d(strain));
* the fitness Z = w_e Z_e + w_v Z_v + w_f Z_f of Sec. III.B and its gradient
  with respect to the six parameters, also by autograd;
* a plain C float64 build of the energy, forces, virials and fitness
  (``tersoff_c.c`` through ``c_oracle.py``), with the derivatives written out
  by the chain rule and candidates spread over OpenMP threads: the benchmark's
  CPU baseline, held to the autograd version by the CPU tests.

Parity status: every function here is pinned by the CPU tests against values
the paper prints (cohesive energy, lattice constant, elastic constants) and
against closed forms, finite differences and invariants.
"""
from .neighbors import neighbor_list, neighbor_list_set
from .tersoff import (evaluate, evaluate_set, fitness, fitness_grad, local_forces,
                      derived_params, diamond_closed_form)

__all__ = ["neighbor_list", "neighbor_list_set", "evaluate", "evaluate_set", "fitness",
           "fitness_grad", "local_forces", "derived_params", "diamond_closed_form"]
