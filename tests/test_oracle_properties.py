"""Pins of the oracle's 0 K property layer (oracle/properties.py): lattice
constant and cohesive energy (Sec. III.C), elastic constants (Table 3) and
finite-displacement phonons (Fig. 4), checked against the printed values and
against facts that do not depend on the implementation: the acoustic sum rule,
the degeneracies the diamond structure imposes at Gamma and X, and the
long-wavelength limit of the acoustic branches, whose slopes are the sound
velocities sqrt(C/rho) of the stress-strain elastic constants."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import properties as OP

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def table2():
    x = np.array(W.TABLE2_X)
    a0, e0 = OP.lattice_constant(x)
    return x, a0, e0


@pytest.fixture(scope="module")
def phonons(table2):
    x, a0, _ = table2
    phi, pos, cell = OP.force_constants(x, a0, n=3)
    return phi, pos, cell


def test_lattice_constant_and_cohesive_energy(table2, golden):
    _, a0, e0 = table2
    c = golden["cohesive_energy"]
    assert round(e0, c["printed_decimals"]) == c["E_c_eV_per_atom"]
    assert abs(a0 - c["a_A"]) <= 10.0 ** -c["a_printed_decimals"]


def test_elastic_constants_match_table3(table2, golden):
    x, a0, _ = table2
    ec = OP.elastic_constants(x, a0)
    g = golden["elastic_constants"]
    assert abs(ec["C11"] - g["C11_GPa"]) <= 1.0
    assert abs(ec["C12"] - g["C12_GPa"]) <= 1.0
    assert abs(ec["C44"] - g["C44_GPa"]) <= 1.0
    # the internal relaxation can only lower the shear stiffness
    assert ec["C44_unrelaxed"] > ec["C44"]


def test_acoustic_sum_rule_and_gamma_point(phonons, table2):
    phi, pos, cell = phonons
    # a rigid translation costs no force
    assert np.abs(phi.sum(axis=2)).max() < 1e-9
    f = OP.frequencies_thz(phi, pos, cell, np.zeros(3))
    assert np.abs(f[:3]).max() < 1e-3                    # acoustic modes at zero
    assert np.ptp(f[3:]) < 1e-8 and f[3] > 10.0           # triply degenerate optical mode


def test_degeneracies_at_x(phonons, table2):
    """At X = (2 pi / a)(1, 0, 0) the diamond structure pairs the modes: two
    transverse acoustic, LA with LO, two transverse optical."""
    phi, pos, cell = phonons
    a0 = table2[1]
    f = OP.frequencies_thz(phi, pos, cell, np.array([1.0, 0, 0]) * 2 * np.pi / a0)
    assert abs(f[0] - f[1]) < 1e-8 and abs(f[2] - f[3]) < 1e-8 and abs(f[4] - f[5]) < 1e-8
    assert f[1] < f[2] - 1.0 and f[3] < f[4] - 1.0


def _slopes(phi, pos, cell, a0, direction):
    """Acoustic phase velocities (km/s) extrapolated to q -> 0 (Richardson on q, 2q)."""
    d = np.asarray(direction, float) / np.linalg.norm(direction)
    out = []
    for s in (0.01, 0.02):
        q = d * s * 2 * np.pi / a0
        f = OP.frequencies_thz(phi, pos, cell, q)[:3]
        out.append(f * 2 * np.pi * 1e12 / (np.linalg.norm(q) * 1e10) / 1e3)
    return (4 * out[0] - out[1]) / 3


def test_acoustic_slopes_are_the_elastic_sound_velocities(phonons, table2):
    """[100]: v_T = sqrt(C44/rho), v_L = sqrt(C11/rho); [110]: v_T1 = sqrt((C11 - C12)/(2 rho)),
    v_T2 = sqrt(C44/rho), v_L = sqrt((C11 + C12 + 2 C44)/(2 rho)), with the relaxed C44."""
    x, a0, _ = table2
    phi, pos, cell = phonons
    ec = OP.elastic_constants(x, a0)
    v = lambda C: OP.sound_velocity(C, a0)
    s100 = _slopes(phi, pos, cell, a0, [1, 0, 0])
    ref100 = np.array([v(ec["C44"]), v(ec["C44"]), v(ec["C11"])])
    assert np.abs(s100 - ref100).max() <= 1e-5 * ref100.max()
    s110 = _slopes(phi, pos, cell, a0, [1, 1, 0])
    ref110 = np.sort([v((ec["C11"] - ec["C12"]) / 2), v(ec["C44"]),
                      v((ec["C11"] + ec["C12"] + 2 * ec["C44"]) / 2)])
    assert np.abs(s110 - ref110).max() <= 1e-5 * ref110.max()


def test_frequencies_scale_with_inverse_square_root_of_mass(phonons, table2):
    phi, pos, cell = phonons
    q = np.array([0.3, 0.2, 0.1]) * 2 * np.pi / table2[1]
    f1 = OP.frequencies_thz(phi, pos, cell, q)
    f4 = OP.frequencies_thz(phi, pos, cell, q, mass=4 * OP.M_SI_AMU)
    assert np.allclose(f4, f1 / 2, rtol=1e-12)
    assert math.isclose(OP.THZ_PER_SQRT_EV_A2_AMU,
                        math.sqrt(1.602176634e-19 / 1.66053906660e-27) / 1e-10 / (2 * math.pi) / 1e12,
                        rel_tol=1e-6)
