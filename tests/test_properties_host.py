"""Host side of the GPU property layer (paper_1909_11474_amd/properties.py) on
the CPU: its geometry builder and its dynamical-matrix / frequency code, fed
with the oracle's force constants, against the oracle's own."""
import numpy as np
import pytest

import workloads as W
from oracle import properties as OP
from paper_1909_11474_amd import properties as PR


def test_conventional_cell_matches_the_oracle_geometry():
    for n in (1, 2, 3):
        p, c = PR.conventional_cell(5.43, n)
        po, co = OP.diamond_cell(5.43, n)
        assert np.array_equal(c, co) and np.allclose(p, po, atol=1e-14)


def test_unit_constants():
    assert abs(PR.THZ - OP.THZ_PER_SQRT_EV_A2_AMU) < 1e-12
    assert PR.EV_A3_TO_GPA == OP.EV_A3_TO_GPA


def test_frequencies_from_oracle_force_constants():
    x = np.array(W.TABLE2_X)
    a0, _ = OP.lattice_constant(x)
    phi, pos, cell = OP.force_constants(x, a0, n=3)
    q, dist = PR.dispersion_path(a0, per_segment=7)
    f = PR.frequencies(phi, pos, cell, q)
    ref = np.array([OP.frequencies_thz(phi, pos, cell, qq) for qq in q])
    assert np.abs(f - ref).max() < 1e-9
    assert dist[0] == 0.0 and np.all(np.diff(dist) >= 0)
    assert np.allclose(q[0], 0) and np.allclose(q[-1], np.array([0.5, 0.5, 0.5]) * 2 * np.pi / a0)
