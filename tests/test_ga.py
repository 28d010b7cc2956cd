"""Host-side GA driver: decoding, selection order, elitism, gradient refinement,
checkpoint/resume.  Runs on the CPU with analytic fitness functions."""
import numpy as np
import pytest

import workloads as W
from paper_1909_11474_amd import ga as G

TARGET = np.array([3.2, 1.43, 2.24, 0.28, 0.6, -0.64])
SPAN = np.asarray(G.DEFAULT_HI) - np.asarray(G.DEFAULT_LO)


def bowl(x):
    return (((np.asarray(x) - TARGET) / SPAN) ** 2).sum(axis=1)


def bowl_grad(x):
    x = np.asarray(x)
    return bowl(x), 2 * (x - TARGET) / SPAN ** 2


def test_limits_agree_with_workload_parameter_box():
    assert tuple(G.DEFAULT_LO) == W.PARAM_LO and tuple(G.DEFAULT_HI) == W.PARAM_HI


def test_decode_is_affine_in_each_gene():
    g = np.array([[0, 0, 0, 0, 0, 0], [1, 1, 1, 1, 1, 1], [0.5] * 6])
    x = G.decode(g, G.DEFAULT_LO, G.DEFAULT_HI)
    assert np.allclose(x[0], G.DEFAULT_LO) and np.allclose(x[1], G.DEFAULT_HI)
    assert np.allclose(x[2], 0.5 * (np.asarray(G.DEFAULT_LO) + G.DEFAULT_HI))


def test_sort_order_puts_nan_last_and_is_stable():
    z = np.array([3.0, np.nan, 1.0, 3.0, np.nan, 0.5])
    assert G.sort_order(z).tolist() == [5, 2, 0, 3, 1, 4]


def test_elitism_makes_best_monotone_and_converges():
    cfg = G.GAConfig(pop=60, n_par=30, n_gen=120, seed=3)
    ga = G.GA(cfg, bowl)
    bests = [ga.step()["best"] for _ in range(cfg.n_gen)]
    assert all(b1 <= b0 for b0, b1 in zip(bests, bests[1:]))
    assert bests[-1] < 1e-3


def test_nan_candidates_never_become_elite():
    def f(x):
        z = bowl(x)
        z[::3] = np.nan
        return z
    ga = G.GA(G.GAConfig(pop=30, n_par=10, n_gen=5, seed=1), f)
    for _ in range(5):
        ga.step()
        assert np.isfinite(ga.z[0])


def test_gradient_refinement_keeps_monotonicity_and_helps():
    cfg = G.GAConfig(pop=40, n_par=20, n_gen=40, seed=5, refine_top=4, refine_steps=2)
    ga = G.GA(cfg, bowl, bowl_grad)
    bests = [ga.step()["best"] for _ in range(cfg.n_gen)]
    assert all(b1 <= b0 for b0, b1 in zip(bests, bests[1:]))
    plain = G.GA(G.GAConfig(pop=40, n_par=20, n_gen=40, seed=5), bowl)
    pb = [plain.step()["best"] for _ in range(40)]
    assert bests[-1] <= pb[-1]


def test_checkpoint_resume_reproduces_the_trajectory(tmp_path):
    cfg = G.GAConfig(pop=24, n_par=12, n_gen=30, seed=9, refine_top=2)
    a = G.GA(cfg, bowl, bowl_grad)
    a.run(10)
    path = str(tmp_path / "ga.npz")
    a.save(path)
    a.run(10)
    b = G.GA(cfg, bowl, bowl_grad)
    b.load(path)
    b.run(10)
    assert np.array_equal(a.genes, b.genes)
    assert np.array_equal(a.z, b.z)
    assert a.generation == b.generation == 20


def test_mutation_rate_falls_to_zero():
    cfg = G.GAConfig(pop=10, n_par=10, n_gen=4, seed=0)
    ga = G.GA(cfg, bowl)
    ga.generation = cfg.n_gen      # p_m = 0: no gene may change except by crossover
    before = ga.genes.copy()
    ga.step()
    assert np.array_equal(np.sort(before, axis=0), np.sort(ga.genes, axis=0))


def test_tersoff_form_limits_and_nine_gene_run():
    """The nine-parameter box matches the workload's, and the driver evolves
    nine genes (the Tersoff form) with refinement, monotone and converging."""
    assert tuple(G.TERSOFF_FORM_LO) == W.FULL_LO and tuple(G.TERSOFF_FORM_HI) == W.FULL_HI
    lo, hi = np.asarray(G.TERSOFF_FORM_LO), np.asarray(G.TERSOFF_FORM_HI)
    target = lo + 0.37 * (hi - lo)

    def f(x):
        return (((np.asarray(x) - target) / (hi - lo)) ** 2).sum(axis=1)

    def fg(x):
        x = np.asarray(x)
        return f(x), 2 * (x - target) / (hi - lo) ** 2

    cfg = G.GAConfig(pop=60, n_par=30, n_gen=80, seed=7, lo=G.TERSOFF_FORM_LO,
                     hi=G.TERSOFF_FORM_HI, refine_top=4)
    ga = G.GA(cfg, f, fg)
    assert ga.genes.shape == (60, 9)
    bests = [ga.step()["best"] for _ in range(cfg.n_gen)]
    assert all(b1 <= b0 for b0, b1 in zip(bests, bests[1:]))
    assert bests[-1] < 1e-4
    with pytest.raises(ValueError):
        G.GA(G.GAConfig(lo=G.TERSOFF_FORM_LO), f)
