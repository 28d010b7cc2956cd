"""The plain C float64 reference (oracle/tersoff_c.c) against the autograd
oracle: energies, forces and virials on structures that exercise every branch
(periodic self-images, several images of one atom, the cutoff's switching
zone, zeta = 0, both angular functions), the fitness Z, the closed-form
diamond energy, and the independence of Z from the OpenMP thread count.

The C code writes the forces and virial out by the chain rule; the autograd
oracle differentiates the energy, so agreement to rounding pins the C
derivatives (Sec. II.A Eqs. 1-9, Sec. II.B Eqs. 10-14, Sec. III.B)."""
import numpy as np
import pytest

import workloads as W
from oracle import tersoff as T
from oracle import c_oracle as C

R1, R2 = 2.8, 3.2
BOX = np.eye(3) * 20.0


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def bcc(g, reps, d=2.6, sigma=0.05):
    a = 2.0 * d / np.sqrt(3.0)
    grid = np.array([[i, j, k] for i in range(reps) for j in range(reps) for k in range(reps)], float)
    frac = (grid[:, None, :] + np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])[None]).reshape(-1, 3)
    return W.displace(g, frac * a, sigma), np.eye(3) * reps * a


@pytest.fixture(scope="module")
def mixed():
    g = rng(3)
    c = np.array([10.0, 10.0, 10.0])
    tri = c + 2.4 * np.array([[0, 0, 0], [1, 0, 0], [0.5, np.sqrt(3) / 2, 0]])
    switching = c + np.array([[0.0, 0, 0], [2.4, 0, 0], [-1.5, 2.6, 0.0]])    # one side at 3.0 A
    s = W.make_set([W.diamond(1, 1, 1), W.random_packing(g, 40), bcc(g, 2), (c[None], BOX),
                    (c + [[0, 0, 0], [0, 3.0, 0]], BOX), (tri, BOX), (switching, BOX)]
                   + W.strained_diamond_cells(5, 2))
    return s, T.topology(s, R2)


@pytest.mark.parametrize("form", ["minimal", "tersoff"])
def test_c_reference_matches_autograd_oracle(mixed, form):
    s, top = mixed
    ctop = C.CTopology(s, R2, entries=(top.i, top.j, top.shift, top.sob))
    X = W.draw_params(rng(7), 3) if form == "minimal" else W.draw_params_full(rng(8), 3)
    for x in X:
        o = T.evaluate_set(s, x, R1, R2, topology=top)
        q = C.evaluate_set(s, x, R1, R2, topology=ctop)
        assert np.abs(o["E"] - q["E"]).max() <= 1e-12 * np.abs(o["E"]).max()
        assert np.abs(o["F"] - q["F"]).max() <= 1e-12 * np.abs(o["F"]).max()
        assert np.abs(o["W6"] - q["W6"]).max() <= 1e-12 * np.abs(o["W6"]).max()


def test_c_fitness_matches_autograd_oracle_at_any_thread_count(mixed):
    s, top = mixed
    refs = T.reference_data(s, W.draw_params(rng(9), 1)[0], R1, R2)
    X = W.draw_params(rng(10), 6)
    w = (1.0, 0.7, 1.3)
    Zo = T.fitness(s, X, refs, w, topology=top)
    ctop = C.CTopology(s, R2, entries=(top.i, top.j, top.shift, top.sob))
    Z1 = C.fitness(s, X, refs, w, topology=ctop, threads=1)
    Z4 = C.fitness(s, X, refs, w, topology=ctop, threads=4)
    assert np.abs(Z1 - Zo).max() <= 1e-12 * np.abs(Zo).max()
    assert np.array_equal(Z1, Z4)
    Xf = W.draw_params_full(rng(11), 2)
    Zf = C.fitness(s, Xf, refs, w, topology=ctop)
    assert np.abs(Zf - T.fitness(s, Xf, refs, w, topology=top)).max() <= 1e-12 * np.abs(Zf).max()


@pytest.mark.parametrize("a", [5.431, 6.8])
def test_c_reference_diamond_closed_form(a):
    pos, cell = W.diamond(1, 1, 1, a=a)
    s = W.make_set([(pos, cell)])
    for x in W.draw_params(rng(12), 3):
        e = C.evaluate_set(s, x, R1, R2)["E"][0] / 8
        ref = T.diamond_closed_form(x, a, R1, R2)
        assert abs(e - ref) <= 1e-12 * abs(ref)
