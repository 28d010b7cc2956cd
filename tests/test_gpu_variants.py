"""Every compiled coordination variant against the oracle.

The batched kernels pick a code variant per wavefront from the largest
coordination M in it (3..16), and a replica group of 8, 16, 32 or 64 lanes
from the structure's padded size.  This set holds one random packing per
(group size, largest coordination) pair from 4 to 16 that a packing of that
size reaches, so each (M, group) code path of every kernel family (fitness,
evaluation, adjoint, both forms, both precisions) runs on at least one
structure, and each structure's own terms are checked: per-structure energies
and squared force residuals from fitness_terms, E/F/W from tersoff_eval,
Z and dZ/dx.

Tolerances: float64 1e-10 relative; float32 arithmetic 1e-4 eV/A force,
1e-5 fitness, 1e-4 gradient (relative to the largest component), and energy
1e-6 eV/atom times max(1, M/8) for a structure of largest coordination M: the
float path keeps zeta as a float sum of M - 1 terms, so its rounding grows
with M (the dense packings here reach M = 16 at twice the density of
crystalline Si).
"""
import numpy as np
import pytest

import workloads as W
from oracle import tersoff as T

pytestmark = pytest.mark.gpu

R1, R2 = 2.8, 3.2

# (atoms, largest coordination) -> (density in atoms/A^3, seed) of a random
# packing (minimum distance 1.9 A) reaching exactly that coordination
COVER = {
    (8, 4): (0.02, 0), (8, 5): (0.02, 2), (8, 6): (0.03, 2), (8, 7): (0.04, 2), (8, 8): (0.05, 2),
    (8, 9): (0.06, 1), (8, 10): (0.06, 5), (8, 11): (0.07, 1), (8, 12): (0.08, 2), (8, 13): (0.08, 0),
    (8, 14): (0.07, 5), (8, 15): (0.1, 0),
    (16, 3): (0.02, 4), (16, 4): (0.02, 0), (16, 5): (0.02, 2), (16, 6): (0.02, 3), (16, 7): (0.04, 3),
    (16, 8): (0.03, 4), (16, 9): (0.04, 5), (16, 10): (0.05, 3), (16, 11): (0.05, 1), (16, 12): (0.07, 0),
    (16, 13): (0.08, 5), (16, 14): (0.09, 5), (16, 15): (0.1, 0),
    (32, 4): (0.02, 0), (32, 5): (0.02, 3), (32, 6): (0.02, 5), (32, 7): (0.03, 3), (32, 8): (0.03, 4),
    (32, 9): (0.05, 0), (32, 10): (0.06, 0), (32, 11): (0.06, 3), (32, 12): (0.06, 2), (32, 13): (0.07, 1),
    (32, 14): (0.08, 0), (32, 15): (0.08, 3), (32, 16): (0.1, 4),
    (64, 5): (0.02, 0), (64, 6): (0.02, 1), (64, 7): (0.03, 0), (64, 8): (0.03, 5), (64, 9): (0.04, 0),
    (64, 10): (0.05, 4), (64, 11): (0.05, 1), (64, 12): (0.06, 0), (64, 13): (0.07, 3), (64, 14): (0.08, 1),
    (64, 15): (0.08, 2), (64, 16): (0.1, 0),
}


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def packing(n, rho, seed):
    return W.random_packing(rng(1000 * n + 10 * seed + int(rho * 100)), n, rho=rho, dmin=1.9)


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_11474_amd import api as A
    return A


@pytest.fixture(scope="module")
def cover():
    keys = sorted(COVER)
    s = W.make_set([packing(n, *COVER[(n, k)]) for n, k in keys])
    top = T.topology(s, R2)
    kmax = np.zeros(s.n_struct, dtype=int)
    coord = np.bincount(top.i, minlength=s.n_atoms)
    off = np.concatenate([[0], np.cumsum(s.sizes())])
    for q in range(s.n_struct):
        kmax[q] = coord[off[q]:off[q + 1]].max()
    # the table reaches what it says
    assert list(kmax) == [k for _, k in keys]
    refs = T.reference_data(s, W.draw_params(rng(70), 1)[0], R1, R2)
    return s, top, kmax, refs


def energy_tol(kmax):
    return 1e-6 * np.maximum(1.0, kmax / 8.0)


@pytest.mark.parametrize("form", ["minimal", "tersoff"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_every_variant_against_the_oracle(api, cover, precision, form):
    s, top, kmax, refs = cover
    X = W.draw_params(rng(71), 2) if form == "minimal" else W.draw_params_full(rng(72), 2)
    ts = api.from_structures(s)
    assert ts.stats()["max_coordination"] == 16
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    sizes = s.sizes().astype(float)
    weights = (1.0, 0.7, 1.3)
    out = ts.tersoff_eval(X, precision=precision)
    E, F, Wv = (out[k].cpu().numpy() for k in ("E", "F", "W"))
    Z = ts.fitness(X, weights, precision=precision).cpu().numpy()
    terms = {k: v.cpu().numpy() for k, v in ts.fitness_terms(X).items()}
    Zg, G = (t.cpu().numpy() for t in ts.fitness_grad(X, weights, precision=precision))
    Zo, Go = T.fitness_grad(s, X, refs, weights, topology=top)
    for c, x in enumerate(X):
        ref = T.evaluate_set(s, x, R1, R2)
        eo = ref["E"] / sizes
        fo = np.asarray(refs["f"])
        rfo = np.array([((ref["F"][a:b] - fo[a:b]) ** 2).sum()
                        for a, b in zip(np.r_[0, np.cumsum(s.sizes())[:-1]], np.cumsum(s.sizes()))])
        if precision == "fp64":
            assert np.abs(E[c] - ref["E"]).max() <= 1e-10 * np.abs(ref["E"]).max()
            assert np.abs(F[c] - ref["F"]).max() <= 1e-10 * np.abs(ref["F"]).max()
            assert np.abs(Wv[c] - ref["W6"]).max() <= 1e-10 * np.abs(ref["W6"]).max()
            assert np.abs(terms["e"][c] - eo).max() <= 1e-10 * np.abs(eo).max()
            assert np.abs(terms["rf"][c] - rfo).max() <= 1e-10 * np.abs(rfo).max()
        else:
            tol = energy_tol(kmax)
            bad = np.nonzero(np.abs(E[c] / sizes - eo) > tol)[0]
            assert bad.size == 0, ("eval energy", c, [(sizes[q], kmax[q], E[c][q] / sizes[q] - eo[q]) for q in bad])
            bad = np.nonzero(np.abs(terms["e"][c] - eo) > tol)[0]
            assert bad.size == 0, ("fitness energy", c, [(sizes[q], kmax[q], terms["e"][c][q] - eo[q]) for q in bad])
            assert np.abs(F[c] - ref["F"]).max() <= 1e-4
            assert np.abs(Wv[c] / sizes[:, None] - ref["W6"] / sizes[:, None]).max() <= 1e-5 * np.maximum(1.0, kmax.max() / 8.0)
            assert np.abs(terms["rf"][c] - rfo).max() <= 1e-5 * np.abs(rfo).max()
        tol = 1e-10 if precision == "fp64" else 1e-4
        assert np.abs(G[c] - Go[c]).max() <= tol * np.abs(Go[c]).max(), (c, G[c], Go[c])
    ztol = 1e-10 if precision == "fp64" else 1e-5
    assert np.abs(Z - Zo).max() <= ztol * np.abs(Zo).max()
    assert np.array_equal(Z, Zg)
    ts.close()
