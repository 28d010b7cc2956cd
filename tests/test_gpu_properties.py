"""The 0 K property layer on the GPU path (paper_1909_11474_amd/properties.py:
lattice constants, strains and displaced supercells batched as the structures
of one float64 tersoff_eval call) against the oracle's property layer, for the
Table 2 parameters and for a Tersoff-form set with S = 2.2.

Tolerances: lattice constant 1e-7 A (the oracle's bounded minimisation of a
flat minimum resolves a0 to about 1e-8 A), energy per atom 1e-10 eV; elastic
constants at the same a0 1e-6 GPa (the oracle relaxes every atom to zero force
with a root finder, the GPU path the sublattice shift by Newton steps; the
central-difference stresses amplify round-off by 1/strain); force constants
1e-8 relative (the same central differences on both sides), frequencies
1e-6 THz.
"""
import numpy as np
import pytest

import workloads as W
from oracle import properties as OP

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def PR():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_11474_amd import properties
    return properties


def tersoff_form_x():
    x = W.minimal_as_full(np.array(W.TABLE2_X), 3.0, 270.0)
    x[3] = 2.2
    return x


PARAMS = {"table2": lambda: np.array(W.TABLE2_X), "tersoff_form": tersoff_form_x}


@pytest.mark.parametrize("which", list(PARAMS))
def test_lattice_constant(PR, which):
    x = PARAMS[which]()
    a0, e0 = PR.lattice_constant(x)
    ao, eo = OP.lattice_constant(x)
    print(which, "a0", a0, ao, "e0", e0, eo, flush=True)
    assert abs(a0 - ao) <= 1e-7
    assert abs(e0 - eo) <= 1e-10
    if which == "table2":                       # Sec. III.C
        assert round(e0, 2) == -4.63 and abs(a0 - 5.434) <= 1e-3


@pytest.mark.parametrize("which", list(PARAMS))
def test_elastic_constants(PR, which):
    x = PARAMS[which]()
    ao, _ = OP.lattice_constant(x)
    ec = PR.elastic_constants(x, ao)
    ref = OP.elastic_constants(x, ao)
    print(which, ec, ref, flush=True)
    for k in ("C11", "C12", "C44", "C44_unrelaxed"):
        assert abs(ec[k] - ref[k]) <= 1e-6, k
    if which == "table2":                       # Table 3, mini-Tersoff row
        assert abs(ec["C11"] - 148) <= 1 and abs(ec["C12"] - 65) <= 1 and abs(ec["C44"] - 75) <= 1
    # the relaxed shift is along x for a yz shear (diamond's internal strain)
    s = ec["shift_per_shear"]
    assert abs(s[0]) > 0.1 and abs(s[1]) < 1e-6 * abs(s[0]) + 1e-9 and abs(s[2]) < 1e-6 * abs(s[0]) + 1e-9


@pytest.mark.parametrize("which", list(PARAMS))
def test_phonons(PR, which):
    x = PARAMS[which]()
    a0, _ = OP.lattice_constant(x)
    phi, pos, cell = PR.force_constants(x, a0, n=3)
    phio, poso, cello = OP.force_constants(x, a0, n=3)
    assert np.abs(phi - phio).max() <= 1e-8 * np.abs(phio).max()
    q, _ = PR.dispersion_path(a0, per_segment=9)
    f = PR.frequencies(phi, pos, cell, q)
    fo = np.array([OP.frequencies_thz(phio, poso, cello, qq) for qq in q])
    assert np.abs(f - fo).max() <= 1e-6
    # long-wavelength limit along [100]: sqrt(C44/rho) (twice) and sqrt(C11/rho)
    ec = PR.elastic_constants(x, a0)
    v = []
    for s in (0.01, 0.02):
        qq = np.array([[s, 0, 0]]) * 2 * np.pi / a0
        v.append(PR.frequencies(phi, pos, cell, qq)[0, :3] * 2 * np.pi * 1e12 / (qq[0, 0] * 1e10) / 1e3)
    slope = (4 * v[0] - v[1]) / 3
    ref = np.array([OP.sound_velocity(ec["C44"], a0)] * 2 + [OP.sound_velocity(ec["C11"], a0)])
    assert np.abs(slope - ref).max() <= 1e-5 * ref.max()
