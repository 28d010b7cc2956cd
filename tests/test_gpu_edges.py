"""GPU edge cases against the oracle: degenerate structures, sizes around the
wavefront and batching limits, the two-pass fitness path, population extremes.

Tolerances as in test_gpu_parity (float64 1e-10 relative; float32 1e-6
eV/atom, 1e-4 eV/A, 1e-5 eV/atom; fitness 1e-5 relative).
"""
import numpy as np
import pytest

import workloads as W
from oracle import tersoff as T
from oracle.neighbors import neighbor_list_set

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


def check_eval(ts, s, X, precision):
    out = ts.tersoff_eval(X, precision=precision, atom_virial=True)
    E, F, Wv, Wi = (out[k].cpu().numpy() for k in ("E", "F", "W", "Wi"))
    sizes = s.sizes().astype(float)
    for c, x in enumerate(X):
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


def degenerate_set():
    """Isolated atom (no bonds), dimers at 2.35 A and inside the switching zone
    (single neighbour: zeta = 0, b = 1), bent and straight trimers
    (cos theta = -1/2 and -1), and a perfect 8-atom diamond cell."""
    c = np.array([10.0, 10.0, 10.0])
    tri = c + 2.4 * np.array([[0, 0, 0], [1, 0, 0], [0.5, np.sqrt(3) / 2, 0]])
    line = c + np.array([[0, 0, 0], [2.3, 0, 0], [4.6, 0, 0]])
    pos, cell = W.diamond(1, 1, 1)
    return W.make_set([(c[None], BOX), (c + [[0, 0, 0], [2.35, 0, 0]], BOX),
                       (c + [[0, 0, 0], [0, 3.0, 0]], BOX), (tri, BOX), (line, BOX), (pos, cell)])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_degenerate_structures(api, precision):
    s = degenerate_set()
    ts = api.from_structures(s)
    st = ts.stats()
    assert st["n_bonds"] == 0 + 2 + 2 + 6 + 4 + 32
    X = np.vstack([np.asarray(W.TABLE2_X)[None], W.draw_params(rng(31), 3)])
    check_eval(ts, s, X, precision)
    ts.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sizes_around_one_wavefront(api, precision):
    """63, 64 and 65 atoms: the last pads to two wavefronts per replica, the
    second holding one atom; 8 atoms pads to 8 lanes."""
    g = rng(32)
    s = W.make_set([W.random_packing(g, n) for n in (63, 64, 65, 8)])
    ts = api.from_structures(s)
    check_eval(ts, s, W.draw_params(rng(33), 3), precision)
    ts.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fitness_across_the_batching_limit(api, precision):
    """A 512-atom structure (largest batched, 512 lanes per replica) beside a
    600-atom one (two-pass path) and 64-atom cells; batched = plain in float64."""
    g = rng(34)
    big = W.random_packing(g, 600)
    edge = W.random_packing(g, 512)
    s = W.make_set([big, edge] + W.strained_diamond_cells(35, 3))
    hidden = W.draw_params(rng(36), 1)[0]
    refs = T.reference_data(s, hidden, R1, R2)
    ts = api.from_structures(s)
    st = ts.stats()
    assert st["n_large"] == 1 and st["n_batched"] == 4 and st["max_atoms"] == 600
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    X = W.draw_params(rng(37), 6)
    Zb = ts.fitness(X, precision=precision).cpu().numpy()
    Zp = ts.fitness(X, precision=precision, schedule="plain").cpu().numpy()
    Zo = T.fitness(s, X[[0, 5]], refs, topology=T.topology(s, R2))
    tol = 1e-10 if precision == "fp64" else 1e-5
    assert np.abs(Zb[[0, 5]] - Zo).max() <= tol * np.abs(Zo).max()
    if precision == "fp64":
        assert np.array_equal(Zb, Zp)
    ts.close()


def check_grad(ts, s, X, refs, precision, weights=(1.0, 0.7, 1.3)):
    """fitness_grad (fitness_grad_tf for nine-column X) against the oracle's
    autograd: float64 1e-10, float32 1e-4 relative to the largest component."""
    Z, G = (t.cpu().numpy() for t in ts.fitness_grad(X, weights, precision=precision))
    Zo, Go = T.fitness_grad(s, X, refs, weights, topology=T.topology(s, R2))
    tol = 1e-10 if precision == "fp64" else 1e-4
    for c in range(len(X)):
        assert np.abs(G[c] - Go[c]).max() <= tol * np.abs(Go[c]).max(), (c, G[c], Go[c])
    assert np.abs(Z - Zo).max() <= (1e-10 if precision == "fp64" else 1e-5) * np.abs(Zo).max()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fitness_gradient_two_pass(api, precision):
    """The two-pass adjoint: a 600-atom packing (coordination above 4) and a
    640-atom displaced diamond block (coordination 4) over the batching limit,
    a 54-atom BCC cell (coordination 14, above the batched adjoint's 12)
    beside two 64-atom cells on the batched adjoint; both forms against the
    oracle's autograd."""
    g = rng(50)
    pos, cell = W.diamond(4, 4, 5)
    s = W.make_set([W.random_packing(g, 600), (W.displace(g, pos, 0.08), cell), bcc_cell(g, 3)]
                   + W.strained_diamond_cells(51, 2))
    ts = api.from_structures(s)
    st = ts.stats()
    assert st["n_large"] == 2 and st["max_coordination"] >= 13
    refs = T.reference_data(s, W.draw_params(rng(52), 1)[0], R1, R2)
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    check_grad(ts, s, W.draw_params(rng(53), 2), refs, precision)
    check_grad(ts, s, W.draw_params_full(rng(54), 1), refs, precision)
    # a repeated call reuses the staging buffers: same bits
    X = W.draw_params(rng(53), 2)
    G1 = ts.fitness_grad(X, precision=precision)[1].cpu().numpy()
    G2 = ts.fitness_grad(X, precision=precision)[1].cpu().numpy()
    assert np.array_equal(G1, G2)
    ts.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_one_large_structure_set(api, precision):
    """A set of one 600-atom packing (the molecular-dynamics shape: two-pass
    path, all slots summed by the whole block): E, W and the heat current J of
    three candidates, one invalid (NaN and isolated), against the oracle and
    against the same structure beside a 64-atom cell; a repeated call gives the
    same bits."""
    g = rng(34)
    big = W.random_packing(g, 600)
    s1 = W.make_set([big])
    s2 = W.make_set([big] + W.strained_diamond_cells(35, 1))
    X = W.draw_params(rng(80), 3)
    X[1, 0] = -1.0                                          # D0 <= 0
    vel = rng(81).normal(0.0, 0.01, size=(600, 3))
    ts1, ts2 = api.from_structures(s1), api.from_structures(s2)
    assert ts1.stats()["n_large"] == 1 and ts1.stats()["n_struct"] == 1
    o1 = {k: v.cpu().numpy() for k, v in ts1.tersoff_eval(X, precision=precision, velocities=vel).items()}
    o1b = {k: v.cpu().numpy() for k, v in ts1.tersoff_eval(X, precision=precision, velocities=vel).items()}
    for k in o1:
        assert np.array_equal(o1[k], o1b[k], equal_nan=True), k
    vel2 = np.vstack([vel, np.zeros((64, 3))])
    o2 = {k: v.cpu().numpy() for k, v in ts2.tersoff_eval(X, precision=precision, velocities=vel2).items()}
    assert np.isnan(o1["E"][1]).all() and np.isnan(o1["W"][1]).all() and np.isnan(o1["J"][1]).all()
    for c in (0, 2):
        ref = T.evaluate_set(s1, X[c], R1, R2, velocities=vel)
        if precision == "fp64":
            assert abs(o1["E"][c, 0] - ref["E"][0]) <= 1e-10 * abs(ref["E"][0])
            assert np.abs(o1["W"][c, 0] - ref["W6"][0]).max() <= 1e-10 * np.abs(ref["W6"][0]).max()
            assert np.abs(o1["J"][c] - ref["J"]).max() <= 1e-10 * np.abs(ref["J"]).max()
            rel = 1e-12
        else:
            assert abs(o1["E"][c, 0] - ref["E"][0]) / 600 <= 1e-6
            assert np.abs(o1["W"][c, 0] - ref["W6"][0]).max() / 600 <= 1e-5
            assert np.abs(o1["J"][c] - ref["J"]).max() <= 1e-5 * np.abs(ref["J"]).max()
            rel = 1e-12
        # the same slots summed beside another structure
        assert abs(o1["E"][c, 0] - o2["E"][c, 0]) <= rel * abs(o2["E"][c, 0])
        assert np.abs(o1["W"][c, 0] - o2["W"][c, 0]).max() <= rel * np.abs(o2["W"][c, 0]).max()
        assert np.abs(o1["J"][c] - o2["J"][c]).max() <= rel * np.abs(o2["J"][c]).max()
        assert np.abs(o1["F"][c] - o2["F"][c, :600]).max() <= 1e-12 * np.abs(o2["F"][c, :600]).max()
    ts1.close()
    ts2.close()


def honeycomb_sheet(nx, ny, b=2.4, vacuum=20.0):
    """Periodic honeycomb sheet of nx * ny rectangular cells (4 atoms each,
    bond b): every atom has exactly three neighbours within R2 (the second
    shell is at sqrt(3) b = 4.16 A)."""
    r3 = np.sqrt(3.0) * b
    basis = np.array([[0.0, 0.0, 0.0], [r3 / 2, b / 2, 0.0], [r3 / 2, 1.5 * b, 0.0], [0.0, 2 * b, 0.0]])
    grid = np.array([[i * r3, j * 3 * b, 0.0] for i in range(nx) for j in range(ny)])
    pos = (grid[:, None, :] + basis[None]).reshape(-1, 3) + [0.0, 0.0, vacuum / 2]
    return pos, np.diag([nx * r3, ny * 3 * b, vacuum])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_large_structures_below_four_neighbours(api, precision):
    """Two-pass structures of the four-neighbour class whose atoms have fewer
    than four bonds: a 1,024-atom honeycomb sheet (largest coordination 3,
    below the class's four geometry rows) and an 800-site diamond block with
    three vacancies (atoms of three and four bonds in one wavefront).  E, F, W,
    W_i and J against the oracle, fitness and dZ/dx against its autograd."""
    g = rng(90)
    hc = honeycomb_sheet(8, 32)
    pos, cell = W.diamond(5, 5, 4)
    keep = np.setdiff1d(np.arange(len(pos)), g.choice(len(pos), 3, replace=False))
    s = W.make_set([hc, (W.displace(g, pos[keep], 0.03), cell)])
    ts = api.from_structures(s)
    st = ts.stats()
    assert st["n_large"] == 2 and st["max_coordination"] == 4
    counts = np.bincount(neighbor_list_set(s, R2)[0], minlength=s.n_atoms)
    assert counts[:1024].max() == 3 and counts[:1024].min() == 3
    assert counts[1024:].min() == 3 and counts[1024:].max() == 4
    X = W.draw_params(rng(91), 2)
    vel = rng(92).normal(0.0, 0.01, size=(s.n_atoms, 3))
    out = ts.tersoff_eval(X, precision=precision, atom_virial=True, velocities=vel)
    E, F, Wv, Wi, J = (out[k].cpu().numpy() for k in ("E", "F", "W", "Wi", "J"))
    n = s.sizes().astype(float)
    for c, x in enumerate(X):
        ref = T.evaluate_set(s, x, R1, R2, atom_virial=True, velocities=vel)
        if precision == "fp64":
            for got, want in ((E[c], ref["E"]), (F[c], ref["F"]), (Wv[c], ref["W6"]), (Wi[c], ref["Wi"]),
                              (J[c], ref["J"])):
                assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()
        else:
            assert np.abs(E[c] / n - ref["E"] / n).max() <= 1e-6
            assert np.abs(F[c] - ref["F"]).max() <= 1e-4
            assert np.abs(Wv[c] / n[:, None] - ref["W6"] / n[:, None]).max() <= 1e-5
            assert np.abs(Wi[c] - ref["Wi"]).max() <= 1e-4
            assert np.abs(J[c] - ref["J"]).max() <= 1e-5 * np.abs(ref["J"]).max()
    refs = T.reference_data(s, W.draw_params(rng(93), 1)[0], R1, R2)
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    Z = ts.fitness(X, precision=precision).cpu().numpy()
    Zo = T.fitness(s, X, refs, topology=T.topology(s, R2))
    assert np.abs(Z - Zo).max() <= (1e-10 if precision == "fp64" else 1e-5) * np.abs(Zo).max()
    check_grad(ts, s, X[:1], refs, precision)
    ts.close()


def test_graph_replay_after_the_staging_buffer_grows(api):
    """A captured fitness graph holds the address of the two-pass staging
    buffer (structures over 512 atoms).  A float64 call and a larger population
    grow that buffer; the float32 call replayed afterwards must be captured
    again, not replayed into the freed memory: same bits as its first call."""
    import torch
    g = rng(34)
    s = W.make_set([W.random_packing(g, 600)] + W.strained_diamond_cells(35, 1))
    refs = T.reference_data(s, W.draw_params(rng(36), 1)[0], R1, R2)
    ts = api.from_structures(s)
    assert ts.stats()["n_large"] == 1
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    X = torch.as_tensor(W.draw_params(rng(38), 6), device="cuda")
    Z = torch.empty(6, 4, dtype=torch.float64, device="cuda")
    call = ts.fitness_call(X, Z, precision="fp32")
    call()                                          # captured
    Z1 = Z.clone()
    call()                                          # replayed
    assert torch.equal(Z, Z1)
    ts.fitness(X, precision="fp64")                 # 8-byte staging: the buffer grows
    call()
    torch.cuda.synchronize()
    assert torch.equal(Z, Z1)
    ts.fitness(W.draw_params(rng(39), 60), precision="fp32")   # 10x the candidates
    call()
    torch.cuda.synchronize()
    assert torch.equal(Z, Z1)
    Zo = T.fitness(s, X[[0, 5]].cpu().numpy(), refs)
    assert np.abs(Z1[[0, 5]].cpu().numpy() - Zo).max() <= 1e-5 * np.abs(Zo).max()
    ts.close()


def test_population_extremes_give_identical_candidates(api):
    """P = 1 and P = 1000 (the same candidates repeated): every candidate's Z
    is the same bits whatever the population around it."""
    wl = W.config2(n_struct=6, pop=8)
    refs = T.reference_data(wl.structs, wl.hidden_x, R1, R2)
    ts = api.from_structures(wl.structs)
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    X = wl.population
    big = np.tile(X, (125, 1))
    for precision in ("fp64", "fp32"):
        Zbig = ts.fitness(big, precision=precision).cpu().numpy()
        for c in range(len(X)):
            Z1 = ts.fitness(X[c:c + 1], precision=precision).cpu().numpy()
            assert np.array_equal(Z1[0], Zbig[c])
            assert np.array_equal(Zbig[c], Zbig[c + 8 * 124])
    ts.close()


def bcc_cell(g, reps, d=2.6, sigma=0.05):
    """Displaced BCC Si of reps^3 cubic cells with nearest-neighbour distance d:
    8 neighbours at d and 6 at 2d/sqrt(3) (3.0 A for d = 2.6, inside the
    switching zone R1 < r < R2), 14 in all, 13-14 after the displacements."""
    a = 2.0 * d / np.sqrt(3.0)
    grid = np.array([[i, j, k] for i in range(reps) for j in range(reps) for k in range(reps)],
                    dtype=np.float64)
    frac = (grid[:, None, :] + np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])[None]).reshape(-1, 3)
    return W.displace(g, frac * a, sigma), np.eye(3) * reps * a


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_coordination_above_twelve(api, precision):
    """BCC cells of 16 (cell width below 2 R2: several images), 54 and 128
    atoms run the kernels of the largest coordination class beside diamond
    cells in the smallest: energies, forces, virials and fitness against the
    oracle, batched = plain in float64, and the Tersoff form's E, F, W, W_i.
    fitness_grad in both forms against the oracle's autograd (the BCC cells,
    above the batched adjoint's 12 neighbours, take the two-pass adjoint)."""
    g = rng(41)
    s = W.make_set([bcc_cell(g, r) for r in (2, 3, 4)] + W.strained_diamond_cells(42, 2))
    ts = api.from_structures(s)
    st = ts.stats()
    assert st["max_coordination"] == 14 and st["n_large"] == 0
    X = W.draw_params(rng(43), 3)
    check_eval(ts, s, X, precision)
    refs = T.reference_data(s, W.draw_params(rng(44), 1)[0], R1, R2)
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    Zb = ts.fitness(X, precision=precision).cpu().numpy()
    Zp = ts.fitness(X, precision=precision, schedule="plain").cpu().numpy()
    Zo = T.fitness(s, X, refs, topology=T.topology(s, R2))
    tol = 1e-10 if precision == "fp64" else 1e-5
    assert np.abs(Zb - Zo).max() <= tol * np.abs(Zo).max()
    if precision == "fp64":
        assert np.array_equal(Zb, Zp)
    # the nine-parameter Tersoff form through the same coordination class
    Xf = W.draw_params_full(rng(45), 2)
    check_eval(ts, s, Xf, precision)
    check_grad(ts, s, X[:2], refs, precision)
    check_grad(ts, s, Xf[:1], refs, precision)
    ts.close()


def shell16(radii=(2.6, 3.0)):
    """One atom with exactly 16 neighbours (the neighbour cap): 16 atoms on a
    Fibonacci sphere around it, alternately at 2.6 A and at 3.0 A (inside the
    switching zone), at least 2.1 A apart."""
    n = 16
    k = np.arange(n) + 0.5
    phi = np.arccos(1.0 - 2.0 * k / n)
    th = np.pi * (1.0 + 5.0 ** 0.5) * k
    u = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], axis=1)
    r = np.where(np.arange(n) % 2 == 0, radii[0], radii[1])[:, None]
    c = np.array([10.0, 10.0, 10.0])
    return np.vstack([c, c + r * u]), BOX


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_atom_at_the_neighbour_cap(api, precision):
    """An atom with MT_MAX_NBR = 16 neighbours (the largest compiled bond
    count) beside a diamond cell: E, F, W, W_i vs oracle for both forms; one
    fewer slot than the atom needs is MT_ENBR_OVERFLOW."""
    pos, cell = shell16()
    s = W.make_set([(pos, cell), W.diamond(1, 1, 1)])
    ts = api.from_structures(s)
    assert ts.stats()["max_coordination"] == 16
    check_eval(ts, s, W.draw_params(rng(46), 3), precision)
    check_eval(ts, s, W.draw_params_full(rng(47), 2), precision)
    ts.close()
    from paper_1909_11474_amd import _lib as L
    with pytest.raises(L.MTError) as e:
        api.TersoffSet(pos, cell[None], [0, len(pos)], max_nbr=15)
    assert e.value.code == L.MT_ENBR_OVERFLOW
