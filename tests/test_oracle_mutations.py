"""Planted mistakes in the oracle must be caught by its pins.

Each case swaps one oracle function for a plausible wrong variant (a dropped
factor, a sign, a wrong exponent, a moved cutoff) and checks that at least one
independent pin -- a closed form or a printed value -- rejects it.  Everything
runs on the CPU against the oracle only.
"""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import tersoff as T

R1, R2 = 2.8, 3.2


def _pins_hold() -> bool:
    x = W.TABLE2_X
    # perfect diamond closed form at two lattice constants, and at one whose
    # bonds lie in the switching zone (f_C of the third atom inside zeta)
    for a in (5.3, 5.43, 6.8):
        pos, cell = W.diamond(1, 1, 1, a)
        e = T.evaluate(pos, cell, x, R1, R2)["E"][0] / 8
        if abs(e - T.diamond_closed_form(x, a)) > 1e-12:
            return False
    # cohesive energy printed in the paper (Sec. III.C)
    from scipy.optimize import minimize_scalar
    res = minimize_scalar(lambda a: T.evaluate(*W.diamond(1, 1, 1, a), x, R1, R2)["E"][0] / 8,
                          bounds=(5.2, 5.7), method="bounded", options={"xatol": 1e-6})
    if round(res.fun, 2) != -4.63:
        return False
    # Morse dimer inside and inside the switching zone
    D0, alpha, r0 = x[:3]
    for r in (2.3, 2.95):
        pos = np.array([[20.0, 20, 20], [20.0 + r, 20, 20]])
        e = T.evaluate(pos, np.eye(3) * 40, x, R1, R2)["E"][0]
        fc = 1.0 if r <= R1 else 0.5 * (1 + math.cos(math.pi * (r - R1) / (R2 - R1)))
        if abs(e - fc * D0 * (math.exp(-2 * alpha * (r - r0)) - 2 * math.exp(-alpha * (r - r0)))) > 1e-12:
            return False
    # equilateral trimer closed form
    s = 2.4
    beta, n, h = x[3:]
    pos = np.array([[20, 20, 20], [20 + s, 20, 20], [20 + s / 2, 20 + s * math.sqrt(3) / 2, 20]])
    zeta = beta * (0.5 - h) ** 2
    b = (1 + zeta ** n) ** (-1 / (2 * n))
    e1 = math.exp(-alpha * (s - r0))
    ref = 3 * D0 * (e1 * e1 - 2 * b * e1)
    if abs(T.evaluate(pos, np.eye(3) * 40, x, R1, R2)["E"][0] - ref) > 1e-12:
        return False
    # isosceles trimer with its base bond in the switching zone
    from test_oracle_pins import _isosceles_trimer_energy, isosceles_trimer
    pos, cell = isosceles_trimer(2.4, 2.95)
    if abs(T.evaluate(pos, cell, x, R1, R2)["E"][0] - _isosceles_trimer_energy(x, 2.4, 2.95)) > 1e-12:
        return False
    return True


def test_unmodified_oracle_passes_the_pins():
    assert _pins_hold()


def _site_energies_variant(kind):
    orig = T.site_energies

    def variant(d, center, p, q, n_atoms, x, R1_, R2_):
        beta, n, h = x[3], x[4], x[5]
        A, B, lam, mu = T.derived_params(x)
        r = torch.sqrt((d * d).sum(dim=1))
        fc = T.cutoff(r, R1_, R2_)
        fR = A * torch.exp(-lam * r)
        fA = B * torch.exp(-mu * r)
        pt, qt = torch.as_tensor(p), torch.as_tensor(q)
        cos = (d[pt] * d[qt]).sum(dim=1) / (r[pt] * r[qt])
        hh = -h if kind == "h_sign" else h
        g = beta * (cos - hh) ** 2
        if kind == "no_fc_in_zeta":
            fcq = torch.ones_like(fc[qt])
        elif kind == "fc_ij_in_zeta":
            fcq = fc[pt]                      # the bond's own cutoff instead of the third atom's
        else:
            fcq = fc[qt]
        zeta = torch.zeros_like(r).index_add(0, pt, fcq * g)
        pos = zeta > 0
        zs = torch.where(pos, zeta, torch.ones_like(zeta))
        expo = -1.0 / n if kind == "b_exponent" else -1.0 / (2.0 * n)
        b = torch.where(pos, (1.0 + zs ** n) ** expo, torch.ones_like(zeta))
        half = 1.0 if kind == "no_half" else 0.5
        Uij = fc * (fR - b * fA)
        return torch.zeros(n_atoms, dtype=d.dtype).index_add(0, torch.as_tensor(center), half * Uij)

    return orig, variant


@pytest.mark.parametrize("kind", ["h_sign", "b_exponent", "no_half", "no_fc_in_zeta", "fc_ij_in_zeta"])
def test_planted_energy_mistakes_are_caught(monkeypatch, kind):
    _, variant = _site_energies_variant(kind)
    monkeypatch.setattr(T, "site_energies", variant)
    assert not _pins_hold()


def test_planted_slope_mistake_is_caught(monkeypatch):
    orig = T.derived_params

    def wrong(x):
        A, B, lam, mu = orig(x)
        return A, B, x[1] * math.sqrt(2.0), mu          # lambda = alpha sqrt(S) instead of sqrt(2S)

    monkeypatch.setattr(T, "derived_params", wrong)
    assert not _pins_hold()


def test_planted_cutoff_mistake_is_caught(monkeypatch):
    def wrong(r, R1_, R2_):
        mid = 0.5 * (1.0 + torch.cos(math.pi * (r - R1_) / R2_))   # wrong switching width
        return torch.where(r <= R1_, torch.ones_like(r), torch.where(r >= R2_, torch.zeros_like(r), mid))

    monkeypatch.setattr(T, "cutoff", wrong)
    assert not _pins_hold()
