"""The stored reference data of the benchmark workloads (written by
tests/golden/make_references.py with the float64 oracle) belong to the
workloads' seeded inputs and equal the oracle's evaluation of the hidden
parameter set: the whole GA batch, and sampled structures of the uneven set."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import tersoff as T

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    return np.load(os.path.join(GOLDEN, name), allow_pickle=False)


def test_ga_batch_references_are_the_oracle_at_the_hidden_set():
    wl = W.config2()
    d = load("references_ga_batch.npz")
    assert np.array_equal(d["sizes"], wl.structs.sizes())
    assert np.array_equal(d["hidden_x"], wl.hidden_x)
    refs = T.reference_data(wl.structs, wl.hidden_x, wl.R1, wl.R2)
    for k in ("e", "w", "f"):
        assert np.array_equal(d[k], refs[k]), k


@pytest.mark.parametrize("k", [0, 57, 123, 199, 254, 299])
def test_uneven_references_sampled(k):
    wl = W.config3()
    s = wl.structs
    d = load("references_uneven.npz")
    assert np.array_equal(d["sizes"], s.sizes())
    pos, cell = s.structure(k)
    o = T.evaluate(pos, cell, wl.hidden_x, wl.R1, wl.R2)
    n = s.sizes()[k]
    assert abs(d["e"][k] - o["E"][0] / n) <= 1e-12 * abs(o["E"][0] / n)
    assert np.abs(d["w"][k] - o["W6"][0] / n).max() <= 1e-12 * max(np.abs(o["W6"][0] / n).max(), 1e-3)
    f = d["f"][s.offset[k]:s.offset[k + 1]]
    assert np.abs(f - o["F"]).max() <= 1e-12 * max(np.abs(o["F"]).max(), 1e-3)
