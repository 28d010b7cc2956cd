"""Oracle pins of the nine-parameter Tersoff form (Sec. II.A Eqs. 2-9 with the
Erhart-Albe parameters of Eqs. 11-14 and a free slope S)."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import tersoff as T
from oracle.neighbors import neighbor_list

R1, R2 = 2.8, 3.2


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def energy(pos, cell, x):
    return float(T.evaluate(pos, cell, x, R1, R2)["E"][0])


def _isolated(points, box=40.0):
    pts = np.asarray(points, dtype=np.float64) + box / 2
    return pts, np.eye(3) * box


def fc(r):
    return 1.0 if r <= R1 else (0.0 if r >= R2 else 0.5 * (1 + math.cos(math.pi * (r - R1) / (R2 - R1))))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dimer_pair_function_and_its_minimum(seed):
    """A dimer has zeta = 0 (b = 1): U = f_C D0/(S-1) [e^{-sqrt(2S) a (r-r0)}
    - S e^{-sqrt(2/S) a (r-r0)}], whose minimum is -D0 at r0 for every S."""
    x = W.draw_params_full(rng(200 + seed), 1)[0]
    D0, alpha, r0, S = x[:4]
    for r in [2.0, 2.3, r0, 2.79, 2.9, 3.1]:
        pos, cell = _isolated([[0, 0, 0], [r, 0, 0]])
        ref = fc(r) * D0 / (S - 1) * (math.exp(-math.sqrt(2 * S) * alpha * (r - r0))
                                      - S * math.exp(-math.sqrt(2 / S) * alpha * (r - r0)))
        assert abs(energy(pos, cell, x) - ref) <= 1e-13 * max(1.0, abs(ref))
    pos, cell = _isolated([[0, 0, 0], [r0, 0, 0]])
    out = T.evaluate(pos, cell, x, R1, R2)
    assert abs(out["E"][0] + D0) < 1e-13 * D0
    assert np.abs(out["F"]).max() < 1e-12


def test_equilateral_trimer_closed_form():
    """Each bond sees one neighbour at 60 degrees: zeta = g^T(cos = 1/2),
    E = 3 [f_R - b f_A]."""
    for x in W.draw_params_full(rng(7), 4):
        D0, alpha, r0, S, gamma, n, c, d, h = x
        s = 2.4
        pos, cell = _isolated([[0, 0, 0], [s, 0, 0], [s / 2, s * math.sqrt(3) / 2, 0]])
        g = gamma * (1 + c * c / (d * d) - c * c / (d * d + (0.5 - h) ** 2))
        b = (1 + g ** n) ** (-1 / (2 * n))
        fr = D0 / (S - 1) * math.exp(-math.sqrt(2 * S) * alpha * (s - r0))
        fa = S * D0 / (S - 1) * math.exp(-math.sqrt(2 / S) * alpha * (s - r0))
        ref = 3 * (fr - b * fa)
        assert abs(energy(pos, cell, x) - ref) <= 1e-13 * 3 * (fr + b * fa)


def test_trimer_with_a_switching_zone_bond_closed_form():
    """Isosceles trimer, apex bonds s <= R1 and base c in (R1, R2), with g^T:
    zeta of an apex bond from the apex carries f_C(s) = 1, of an apex bond from a
    base atom f_C(c), of the base bond f_C(s) (Sec. II.A Eqs. 2-9)."""
    for x in W.draw_params_full(rng(27), 3):
        D0, alpha, r0, S, gamma, n, cc, d, h = x
        s, c = 2.4, 2.95

        def g(cos):
            return gamma * (1 + cc * cc / (d * d) - cc * cc / (d * d + (cos - h) ** 2))

        def bond(r, zeta):
            b = (1 + zeta ** n) ** (-1 / (2 * n))
            fr = D0 / (S - 1) * math.exp(-math.sqrt(2 * S) * alpha * (r - r0))
            fa = S * D0 / (S - 1) * math.exp(-math.sqrt(2 / S) * alpha * (r - r0))
            return fc(r) * (fr - b * fa)

        cos0, cos1 = 1 - c * c / (2 * s * s), c / (2 * s)
        ref = bond(s, fc(s) * g(cos0)) + bond(s, fc(c) * g(cos1)) + bond(c, fc(s) * g(cos1))
        y = math.sqrt(s * s - c * c / 4)
        pos, cell = _isolated([[0, y, 0], [-c / 2, 0, 0], [c / 2, 0, 0]])
        assert abs(energy(pos, cell, x) - ref) <= 1e-13 * max(1.0, abs(ref))


def test_angular_function_approaches_the_minimal_one():
    """Sec. II.B: for c^2/d^2 >> 1, d^2 >> 1 and gamma << 1, g^T approaches
    beta (cos - h)^2 with beta = gamma c^2 / d^4.  With S = 2 and c = 10 d^3
    (gamma = beta / (100 d^2)) g^T - beta t^2 = gamma - beta t^4 / (d^2 + t^2),
    so the energies of the two forms converge as 1 / d^2."""
    pos, cell = W.strained_diamond_cells(51, 1)[0]
    pos2, cell2 = W.random_packing(rng(52), 30)
    for x in [np.array(W.TABLE2_X)] + list(W.draw_params(rng(53), 2)):
        for p, cl in ((pos, cell), (pos2, cell2)):
            e_min = energy(p, cl, x)
            errs = []
            for dd in (10.0, 100.0, 1000.0):
                xf = W.minimal_as_full(x, dd, 10.0 * dd ** 3)
                errs.append(abs(energy(p, cl, xf) - e_min) / abs(e_min))
            assert errs[0] > 50 * errs[1] > 2500 * errs[2]
            assert errs[2] < 1e-5


def _switching_structure():
    pos, cell = W.random_packing(rng(21), 24)
    i, j, sh = neighbor_list(pos, cell, R2)
    r = np.linalg.norm(pos[j] + sh @ cell - pos[i], axis=1)
    assert np.any((r > R1) & (r < R2))
    return pos, cell


def test_forces_and_virial_are_derivatives_of_the_energy():
    pos, cell = _switching_structure()
    x = W.draw_params_full(rng(22), 1)[0]
    out = T.evaluate(pos, cell, x, R1, R2)
    h = 1e-5
    fd = np.zeros_like(pos)
    for a in range(pos.shape[0]):
        for k in range(3):
            p1 = pos.copy(); p1[a, k] += h
            p2 = pos.copy(); p2[a, k] -= h
            fd[a, k] = -(energy(p1, cell, x) - energy(p2, cell, x)) / (2 * h)
    assert np.abs(out["F"] - fd).max() <= 1e-7 * np.abs(out["F"]).max()
    h = 1e-6
    for comp, (m, n) in enumerate(T.VIRIAL6):
        e = []
        for sgn in (+1, -1):
            F = np.eye(3)
            F[m, n] += sgn * h
            e.append(energy(pos @ F.T, cell @ F.T, x))
        fdw = -(e[0] - e[1]) / (2 * h)
        assert abs(out["W6"][0, comp] - fdw) <= 1e-7 * np.abs(out["W6"]).max()


def test_fitness_gradient_over_nine_parameters_matches_central_differences():
    s = W.make_set([_switching_structure(), W.strained_diamond_cells(54, 1)[0]])
    hidden = W.draw_params_full(rng(55), 1)[0]
    refs = T.reference_data(s, hidden, R1, R2)
    top = T.topology(s, R2)
    x = W.draw_params_full(rng(56), 1)[0]
    Z, G = T.fitness_grad(s, x[None], refs, topology=top)
    assert G.shape == (1, 9)
    h = 1e-6
    fd = np.zeros(9)
    for k in range(9):
        xp = x.copy(); xp[k] += h
        xm = x.copy(); xm[k] -= h
        fd[k] = (T.fitness(s, xp[None], refs, topology=top)[0, 0]
                 - T.fitness(s, xm[None], refs, topology=top)[0, 0]) / (2 * h)
    assert np.abs(G[0] - fd).max() <= 1e-6 * np.abs(fd).max()
