"""GPU parity of the nine-parameter Tersoff form (Sec. II.A Eqs. 2-9 with
Tersoff's angular function, Eq. 8, and Eqs. 11-14 at a free slope S) against
the oracle, through tersoff_eval_tf and fitness_eval_tf.

Structures: strained 64-atom diamond cells, random packings with coordination
up to 9 (the one-bond-at-a-time backward sweep above 8 neighbours), small
clusters (dimer, trimers, isolated atom) and a 600-atom packing (two-pass
path).  Parameters: uniform inside the nine-parameter box.  Tolerances as in
test_gpu_parity: float64 1e-10 relative to the quantity's scale; float32
arithmetic 1e-6 eV/atom energy, 1e-4 eV/A force, 1e-5 eV/atom virial; fitness
1e-10 (float64) and 1e-5 (float32) relative.
"""
import numpy as np
import pytest

import workloads as W
from oracle import tersoff as T

pytestmark = pytest.mark.gpu

R1, R2 = 2.8, 3.2
BOX = np.eye(3) * 20.0


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_11474_amd import api as A
    return A


def mixed_set(with_large):
    g = rng(61)
    c = np.array([10.0, 10.0, 10.0])
    tri = c + 2.4 * np.array([[0, 0, 0], [1, 0, 0], [0.5, np.sqrt(3) / 2, 0]])
    line = c + np.array([[0, 0, 0], [2.3, 0, 0], [4.6, 0, 0]])
    structs = W.strained_diamond_cells(62, 2) + [
        W.random_packing(g, 40), W.random_packing(g, 90), W.random_packing(g, 9),
        (c[None], BOX), (c + [[0, 0, 0], [2.35, 0, 0]], BOX), (c + [[0, 0, 0], [0, 3.0, 0]], BOX),
        (tri, BOX), (line, BOX)]
    if with_large:
        structs.append(W.random_packing(g, 600))
    return W.make_set(structs)


def check_eval(out, s, X, precision):
    E, F, Wv, Wi = (out[k].cpu().numpy() for k in ("E", "F", "W", "Wi"))
    sizes = s.sizes().astype(float)
    for c, x in enumerate(X):
        print("candidate", c, precision, flush=True)
        ref = T.evaluate_set(s, x, R1, R2, atom_virial=True)
        if precision == "fp64":
            assert np.abs(E[c] - ref["E"]).max() <= 1e-10 * max(np.abs(ref["E"]).max(), 1e-2)
            assert np.abs(F[c] - ref["F"]).max() <= 1e-10 * max(np.abs(ref["F"]).max(), 1e-12) + 1e-12
            assert np.abs(Wv[c] - ref["W6"]).max() <= 1e-10 * max(np.abs(ref["W6"]).max(), 1e-2)
            assert np.abs(Wi[c] - ref["Wi"]).max() <= 1e-10 * max(np.abs(ref["Wi"]).max(), 1e-2)
        else:
            assert np.abs(E[c] / sizes - ref["E"] / sizes).max() <= 1e-6
            assert np.abs(F[c] - ref["F"]).max() <= 1e-4
            assert np.abs(Wv[c] / sizes[:, None] - ref["W6"] / sizes[:, None]).max() <= 1e-5
            assert np.abs(Wi[c] - ref["Wi"]).max() <= 1e-4


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_tersoff_form_eval_matches_oracle(api, precision):
    s = mixed_set(with_large=True)
    ts = api.from_structures(s)
    st = ts.stats()
    assert st["n_large"] == 1 and st["max_coordination"] > 8
    X = W.draw_params_full(rng(63), 3)
    out = ts.tersoff_eval(X, precision=precision, atom_virial=True)
    check_eval(out, s, X, precision)
    ts.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_tersoff_form_fitness_matches_oracle_and_plain(api, precision):
    s = mixed_set(with_large=True)
    hidden = W.draw_params_full(rng(64), 1)[0]
    refs = T.reference_data(s, hidden, R1, R2)
    ts = api.from_structures(s)
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    X = W.draw_params_full(rng(65), 8)
    weights = (1.0, 0.7, 1.3)
    Zb = ts.fitness(X, weights, precision=precision).cpu().numpy()
    Zp = ts.fitness(X, weights, precision=precision, schedule="plain").cpu().numpy()
    idx = [0, 3, 7]
    Zo = T.fitness(s, X[idx], refs, weights, topology=T.topology(s, R2))
    tol = 1e-10 if precision == "fp64" else 1e-5
    assert np.abs(Zb[idx] - Zo).max() <= tol * np.abs(Zo).max()
    if precision == "fp64":
        assert np.array_equal(Zb, Zp)
    else:
        assert np.abs(Zb - Zp).max() <= 1e-5 * np.abs(Zb).max()
    # the hidden set itself: Z = 0 up to the precision's rounding
    Zh = ts.fitness(hidden[None], weights, precision=precision).cpu().numpy()
    assert Zh[0, 0] <= (1e-12 if precision == "fp64" else 1e-5)
    ts.close()


def test_graphs_of_the_two_forms_are_kept_apart(api):
    """Alternating minimal and Tersoff-form fitness calls (captured graphs are
    keyed by form) give the same bits as each form alone."""
    import torch
    wl = W.config2(n_struct=6, pop=8)
    refs = T.reference_data(wl.structs, wl.hidden_x, R1, R2)
    ts = api.from_structures(wl.structs)
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    xm = torch.as_tensor(wl.population, device="cuda")
    xf = torch.as_tensor(W.draw_params_full(rng(66), 8), device="cuda")
    zm = ts.fitness(xm).clone()
    zf = ts.fitness(xf).clone()
    for _ in range(3):
        assert torch.equal(ts.fitness(xm), zm)
        assert torch.equal(ts.fitness(xf), zf)
    zo = T.fitness(wl.structs, xf.cpu().numpy()[:2], refs, topology=T.topology(wl.structs, R2))
    assert np.abs(zf.cpu().numpy()[:2] - zo).max() <= 1e-5 * np.abs(zo).max()
    ts.close()


def test_limit_of_the_tersoff_form_is_the_minimal_potential(api):
    """Sec. II.B: with S = 2, c = 10 d^3 and gamma = beta d^4 / c^2, g^T tends to
    beta (cos - h)^2 as d grows; the GPU energies of the two forms (float64)
    converge as 1 / d^2, as in the oracle."""
    s = W.make_set(W.strained_diamond_cells(67, 1) + [W.random_packing(rng(68), 30)])
    ts = api.from_structures(s)
    for x in [np.array(W.TABLE2_X)] + list(W.draw_params(rng(69), 2)):
        e_min = ts.tersoff_eval(x[None], precision="fp64")["E"].cpu().numpy()[0]
        errs = []
        for dd in (10.0, 100.0, 1000.0):
            xf = W.minimal_as_full(x, dd, 10.0 * dd ** 3)
            e = ts.tersoff_eval(xf[None], precision="fp64")["E"].cpu().numpy()[0]
            errs.append(np.abs((e - e_min) / e_min).max())
        assert errs[0] > 50 * errs[1] > 2500 * errs[2]
        assert errs[2] < 1e-5
    ts.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_out_of_domain_candidates_are_nan_and_isolated(api, precision):
    s = mixed_set(with_large=False)
    hidden = W.draw_params_full(rng(70), 1)[0]
    refs = T.reference_data(s, hidden, R1, R2)
    ts = api.from_structures(s)
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    X = W.draw_params_full(rng(71), 6)
    bad = X.copy()
    bad[0, 3] = 1.0            # S = 1
    bad[1, 7] = 0.0            # d = 0
    bad[2, 5] = 0.0            # n = 0
    bad[3, 4] = -0.1           # gamma < 0
    bad[4, 0] = np.nan
    Z = ts.fitness(bad, precision=precision).cpu().numpy()
    assert np.isnan(Z[:5]).all()
    Z5 = ts.fitness(X[5:6], precision=precision).cpu().numpy()
    assert np.array_equal(Z[5], Z5[0])
    E = ts.tersoff_eval(bad, precision=precision)["E"].cpu().numpy()
    assert np.isnan(E[:5]).all() and np.isfinite(E[5]).all()
    ts.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_tersoff_form_gradient_matches_oracle(api, precision):
    """dZ/dx over the nine parameters (fitness_grad_tf) against the oracle's
    autograd, on small cells and packings with coordination up to 9."""
    s = mixed_set(with_large=False)
    hidden = W.draw_params_full(rng(73), 1)[0]
    refs = T.reference_data(s, hidden, R1, R2)
    ts = api.from_structures(s)
    assert ts.stats()["max_coordination"] <= 12
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    X = W.draw_params_full(rng(74), 4)
    weights = (1.0, 0.7, 1.3)
    Z, G = ts.fitness_grad(X, weights, precision=precision)
    Z, G = Z.cpu().numpy(), G.cpu().numpy()
    assert G.shape == (4, 9)
    Zo, Go = T.fitness_grad(s, X, refs, weights, topology=T.topology(s, R2))
    tol = 1e-10 if precision == "fp64" else 1e-4
    for c in range(4):
        print("candidate", c, precision, "max |dZ/dx|", np.abs(Go[c]).max(), flush=True)
        assert np.abs(G[c] - Go[c]).max() <= tol * np.abs(Go[c]).max()
        assert abs(Z[c, 0] - Zo[c, 0]) <= (1e-10 if precision == "fp64" else 1e-5) * abs(Zo[c, 0])
    ts.close()


def test_tersoff_form_gradient_matches_central_differences_and_autograd(api):
    """On the 18-structure uneven subset (every kind at its size extremes):
    float64 dZ/dx against central differences of the float64 fitness
    (h = 1e-6), and the same gradient through torch.autograd."""
    import torch
    from test_gpu_workloads import sample_structures
    wl = W.config4()
    sub = wl.structs.subset(sample_structures(wl.structs))
    hidden = W.draw_params_full(rng(75), 1)[0]
    refs = T.reference_data(sub, hidden, R1, R2)
    ts = api.from_structures(sub)
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    X = W.draw_params_full(rng(76), 3)
    _, G = ts.fitness_grad(X, precision="fp64")
    G = G.cpu().numpy()
    h = 1e-6
    fd = np.zeros_like(G)
    for k in range(9):
        Xp, Xm = X.copy(), X.copy()
        Xp[:, k] += h
        Xm[:, k] -= h
        fd[:, k] = (ts.fitness(Xp, precision="fp64").cpu().numpy()[:, 0]
                    - ts.fitness(Xm, precision="fp64").cpu().numpy()[:, 0]) / (2 * h)
    for c in range(3):
        assert np.abs(G[c] - fd[c]).max() <= 1e-5 * np.abs(fd[c]).max()
    xt = torch.as_tensor(X, device="cuda").requires_grad_(True)
    api.tersoff_fitness(xt, ts, precision="fp64").sum().backward()
    assert np.array_equal(xt.grad.cpu().numpy(), G)
    ts.close()


def test_ga_over_nine_genes_on_the_gpu_fitness(api):
    """The host GA with gradient refinement over the nine Tersoff-form genes on
    the GPU fitness and fitness_grad_tf: monotone best, elite Z against the
    oracle."""
    from paper_1909_11474_amd import ga as G
    s = mixed_set(with_large=False)
    hidden = W.draw_params_full(rng(77), 1)[0]
    refs = T.reference_data(s, hidden, R1, R2)
    ts = api.from_structures(s)
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    fit, grad = G.gpu_fitness(ts, precision="fp32")
    cfg = G.GAConfig(pop=48, n_par=24, n_gen=30, seed=78, lo=G.TERSOFF_FORM_LO,
                     hi=G.TERSOFF_FORM_HI, refine_top=4)
    ga = G.GA(cfg, fit, grad)
    bests = [ga.step()["best"] for _ in range(20)]
    print("best", bests[0], "->", bests[-1], flush=True)
    assert all(b1 <= b0 for b0, b1 in zip(bests, bests[1:])) and bests[-1] < bests[0]
    z, x = ga.best()
    zo = T.fitness(s, x[None], refs, topology=T.topology(s, R2))[0, 0]
    assert abs(z - zo) <= 1e-5 * abs(zo) + 1e-6
    ts.close()



@pytest.mark.parametrize("form", ["minimal", "tersoff"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_launch_shapes_on_a_mixed_set_give_identical_fitness(api, tmp_path, precision, form):
    """Block size, candidate tile and persistent bins change only the schedule,
    also where one launch holds structures of different padded sizes and hence
    different candidate tiles (64-atom cells at 2 replicas per 128-thread block
    next to clusters at 16): Z is bit-identical across shapes and to the plain
    path, and dZ/dx (the adjoint kernels, same work lists) is bit-identical
    across shapes and matches the oracle, for both parameterisations.  A launch
    whose LDS were sized for one structure's records and another's exchange
    slots would lose the last replica's slots and show here as wrong force
    residuals."""
    s = mixed_set(with_large=False)
    draw = W.draw_params if form == "minimal" else W.draw_params_full
    hidden = draw(rng(79), 1)[0]
    refs = T.reference_data(s, hidden, R1, R2)
    ts = api.from_structures(s)
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    X = draw(rng(80), 20)
    P = X.shape[0]
    ref = ts.fitness(X, precision=precision, schedule="plain").cpu().numpy()
    idx = [1, 7]
    Zo, Go = T.fitness_grad(s, X[idx], refs, topology=T.topology(s, R2))
    if precision == "fp64":
        assert np.abs(ref[idx] - Zo).max() <= 1e-10 * np.abs(Zo).max()
    G0 = None
    st = ts.stats()
    prec = 0 if precision == "fp64" else 1
    key = (f"N={st['n_atoms']} S={st['n_struct']} nb={st['n_bonds']} trip={st['n_triplets']} "
           f"P={P} prec={prec}")
    k = 0
    for block in (128, 256, 512):
        for tile in (1, 8, 32):
            for persistent in (0, 1):
                k += 1
                cache = tmp_path / f"c{k}.txt"
                cache.write_text(f"{key} | block={block} tile={tile} persistent={persistent} ms=0\n")
                ts.autotune(P, precision, str(cache))
                Z = ts.fitness(X, precision=precision).cpu().numpy()
                assert np.array_equal(Z, ref), (block, tile, persistent)
                G = ts.fitness_grad(X, precision=precision)[1].cpu().numpy()
                if G0 is None:
                    G0 = G
                    tol = 1e-10 if precision == "fp64" else 1e-4
                    for c, go in zip(idx, Go):
                        assert np.abs(G[c] - go).max() <= tol * np.abs(go).max(), c
                assert np.array_equal(G, G0), (block, tile, persistent)
    ts.close()
