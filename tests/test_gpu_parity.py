"""GPU parity: the HIP library against the FP64 oracle, element by element.

Tolerances (GPU vs oracle):
* FP64 path: relative 1e-10 against the quantity's scale (max |F| of the set,
  max |W|, |E|), floor 1e-12.
* FP32 arithmetic with FP64 accumulation: |de_s| <= 1e-6 eV/atom,
  |dF| <= 1e-4 eV/A per component, |dw_s| <= 1e-5 eV/atom (virial per atom).
"""
import ctypes
import time

import numpy as np
import pytest

import workloads as W
from oracle import tersoff as T

pytestmark = pytest.mark.gpu

R1, R2 = 2.8, 3.2


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_11474_amd import api as A
    return A


def neighbor_multiset(i, j, sh):
    return sorted(zip(i.tolist(), j.tolist(), *np.asarray(sh).T.tolist()))


def tiny_sets():
    out = []
    pos, cell = W.diamond(1, 1, 1)
    out.append(("8-atom diamond", W.make_set([(W.displace(rng(1), pos, 0.1), cell)])))
    F = np.eye(3); F[0, 1] = 0.3; F[2, 0] = -0.2
    out.append(("sheared 8-atom", W.make_set([(pos @ F.T, cell @ F.T)])))
    cell2 = np.array([[2.5, 0, 0], [0.4, 3.9, 0], [0.3, 0.2, 4.1]])
    out.append(("self-image 2-atom", W.make_set([(np.array([[0.1, 0.2, 0.3], [1.3, 1.9, 2.2]]), cell2)])))
    out.append(("packing 40", W.make_set([W.random_packing(rng(2), 40)])))
    out.append(("mixed", W.make_set([W.random_packing(rng(3), 13), (pos, cell),
                                     W.strained_diamond_cells(4, 1)[0]])))
    return out


@pytest.mark.parametrize("k", range(5))
def test_neighbors_match_brute_force(api, k):
    name, s = tiny_sets()[k]
    print("case", name, flush=True)
    ts = api.from_structures(s)
    i, j, sh = ts.neighbors()
    from oracle.neighbors import neighbor_list_set
    oi, oj, osh, _ = neighbor_list_set(s, R2)
    assert neighbor_multiset(i, j, sh) == neighbor_multiset(oi, oj, osh)
    st = ts.stats()
    assert st["n_bonds"] == len(oi)
    ts.close()


def compare_eval(ts, s, X, precision, schedule="batched", vel=None):
    out = ts.tersoff_eval(X, precision=precision, schedule=schedule, atom_virial=True,
                          velocities=vel)
    E = out["E"].cpu().numpy()
    F = out["F"].cpu().numpy()
    Wv = out["W"].cpu().numpy()
    Wi = out["Wi"].cpu().numpy()
    sizes = s.sizes().astype(float)
    for c, x in enumerate(np.atleast_2d(X)):
        ref = T.evaluate_set(s, x, R1, R2, atom_virial=True, velocities=vel)
        if precision == "fp64":
            scaleF = max(np.abs(ref["F"]).max(), 1e-12)
            assert np.abs(E[c] - ref["E"]).max() <= 1e-10 * max(np.abs(ref["E"]).max(), 1e-2)
            assert np.abs(F[c] - ref["F"]).max() <= 1e-10 * scaleF + 1e-12
            assert np.abs(Wv[c] - ref["W6"]).max() <= 1e-10 * max(np.abs(ref["W6"]).max(), 1e-2)
            assert np.abs(Wi[c] - ref["Wi"]).max() <= 1e-10 * max(np.abs(ref["Wi"]).max(), 1e-2)
            if vel is not None:
                J = out["J"].cpu().numpy()
                assert np.abs(J[c] - ref["J"]).max() <= 1e-10 * max(np.abs(ref["J"]).max(), 1e-6)
        else:
            assert np.abs(E[c] / sizes - ref["E"] / sizes).max() <= 1e-6
            assert np.abs(F[c] - ref["F"]).max() <= 1e-4
            assert np.abs(Wv[c] / sizes[:, None] - ref["W6"] / sizes[:, None]).max() <= 1e-5
            assert np.abs(Wi[c] - ref["Wi"]).max() <= 1e-4


@pytest.mark.parametrize("k", range(5))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_eval_tiny_cells(api, k, precision):
    name, s = tiny_sets()[k]
    print("case", name, precision, flush=True)
    ts = api.from_structures(s)
    X = W.draw_params(rng(10 + k), 3)
    compare_eval(ts, s, X, precision)
    ts.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("schedule", ["batched", "plain"])
def test_eval_config1(api, precision, schedule):
    wl = W.config1()
    ts = api.from_structures(wl.structs)
    vel = W.maxwell_boltzmann(rng(5), wl.structs.n_atoms, 300.0)
    compare_eval(ts, wl.structs, wl.population, precision, schedule, vel=vel)
    ts.close()


def small_training(n=12):
    wl = W.config2(n_struct=n, pop=20)
    refs = T.reference_data(wl.structs, wl.hidden_x, R1, R2)
    return wl, refs


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fitness_config2_subset(api, precision):
    wl, refs = small_training()
    ts = api.from_structures(wl.structs)
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    weights = (1.0, 0.5, 2.0)
    Zb = ts.fitness(wl.population, weights, precision, "batched").cpu().numpy()
    Zp = ts.fitness(wl.population, weights, precision, "plain").cpu().numpy()
    top = T.topology(wl.structs, R2)
    idx = [0, 7, 19]
    Zo = T.fitness(wl.structs, wl.population[idx], refs, weights, topology=top)
    if precision == "fp64":
        assert np.abs(Zb[idx] - Zo).max() <= 1e-10 * np.abs(Zo).max()
        assert np.array_equal(Zb, Zp)
    else:
        assert np.abs(Zb[idx] - Zo).max() <= 1e-5 * np.abs(Zo).max()
        assert np.abs(Zb - Zp).max() <= 1e-6 * np.abs(Zb).max()
    ts.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fitness_gradient(api, precision):
    wl, refs = small_training(6)
    ts = api.from_structures(wl.structs)
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    weights = (1.0, 0.7, 1.3)
    X = wl.population[:4]
    Z, G = ts.fitness_grad(X, weights, precision)
    Z, G = Z.cpu().numpy(), G.cpu().numpy()
    top = T.topology(wl.structs, R2)
    Zo, Go = T.fitness_grad(wl.structs, X, refs, weights, topology=top)
    tol = 1e-10 if precision == "fp64" else 1e-4
    for c in range(len(X)):
        assert np.abs(G[c] - Go[c]).max() <= tol * np.abs(Go[c]).max()
    assert np.abs(Z - Zo).max() <= (1e-10 if precision == "fp64" else 1e-5) * np.abs(Zo).max()
    ts.close()


def test_invalid_candidates_are_nan_and_isolated(api):
    wl, refs = small_training(4)
    ts = api.from_structures(wl.structs)
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    X = np.array(wl.population[:6])
    Z0 = ts.fitness(X, precision="fp64").cpu().numpy()
    X[1, 0] = -1.0          # D0 <= 0
    X[3, 4] = np.nan        # n not finite
    Z1 = ts.fitness(X, precision="fp64").cpu().numpy()
    assert np.all(np.isnan(Z1[[1, 3]]))
    ok = [0, 2, 4, 5]
    assert np.array_equal(Z1[ok], Z0[ok])
    ts.close()


def test_error_paths(api):
    from paper_1909_11474_amd import _lib as L
    # neighbour capacity overflow: diamond has 4 neighbours per atom
    pos, cell = W.diamond(1, 1, 1)
    with pytest.raises(L.MTError) as e:
        api.TersoffSet(pos, cell[None], [0, 8], max_nbr=3)
    assert e.value.code == L.MT_ENBR_OVERFLOW
    # coincident atoms
    p2 = pos.copy(); p2[1] = p2[0]
    with pytest.raises(L.MTError) as e:
        api.TersoffSet(p2, cell[None], [0, 8])
    assert e.value.code == L.MT_ECOINCIDENT
    # fitness without reference
    ts = api.TersoffSet(pos, cell[None], [0, 8])
    with pytest.raises(L.MTError) as e:
        ts.fitness(np.array([W.TABLE2_X]))
    assert e.value.code == L.MT_ENOREF
    ts.close()


def _force_cfg(ts, P, precision, cache, block, tile, persistent):
    st = ts.stats()
    prec = 0 if precision == "fp64" else 1
    key = (f"N={st['n_atoms']} S={st['n_struct']} nb={st['n_bonds']} trip={st['n_triplets']} "
           f"P={P} prec={prec}")
    cache.write_text(f"{key} | block={block} tile={tile} persistent={persistent} ms=0\n")
    ts.autotune(P, precision, str(cache))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_launch_shapes_give_identical_fitness(api, tmp_path, precision):
    """Block size, candidate tile and persistent bins change only the schedule:
    the reduction order is fixed, so Z is bit-identical across launch shapes
    (and to the plain path)."""
    wl, refs = small_training(12)
    ts = api.from_structures(wl.structs)
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    X = wl.population
    P = X.shape[0]
    ref = ts.fitness(X, precision=precision, schedule="plain").cpu().numpy()
    k = 0
    for block in (64, 256, 512):
        for tile in (1, 8, 32):
            for persistent in (0, 1):
                k += 1
                _force_cfg(ts, P, precision, tmp_path / f"c{k}.txt", block, tile, persistent)
                Z = ts.fitness(X, precision=precision).cpu().numpy()
                assert np.array_equal(Z, ref), (block, tile, persistent)
    ts.close()


def test_cached_launch_shape_out_of_range_is_rejected(api, tmp_path):
    """A cache entry whose shape the batched kernels cannot run (more than 512
    threads per block, or not whole wavefronts) is refused on the host with
    MT_EINVAL before anything is launched; the set keeps working."""
    from paper_1909_11474_amd import _lib as L
    wl, refs = small_training(4)
    ts = api.from_structures(wl.structs)
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    X = wl.population
    P = X.shape[0]
    Z0 = ts.fitness(X, precision="fp64").cpu().numpy()
    for k, block in enumerate((1024, 96, 0)):
        with pytest.raises(L.MTError) as e:
            _force_cfg(ts, P, "fp64", tmp_path / f"bad{k}.txt", block, 8, 0)
        assert e.value.code == L.MT_EINVAL
    assert np.array_equal(ts.fitness(X, precision="fp64").cpu().numpy(), Z0)
    ts.close()


def test_repeated_graph_replays_are_identical(api):
    """Graph replays of the same generation give the same Z every time, and a
    replay picks up new parameter values written into the bound buffer."""
    import torch
    wl, refs = small_training(8)
    ts = api.from_structures(wl.structs)
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    X = torch.tensor(wl.population, dtype=torch.float64, device="cuda")
    Z = torch.empty(X.shape[0], 4, dtype=torch.float64, device="cuda")
    call = ts.fitness_call(X, Z, precision="fp32")
    first = call().clone()
    for _ in range(20):
        call()
        torch.cuda.synchronize()
        assert torch.equal(Z, first)
    X2 = X.clone()
    X2[:, 3] *= 1.1                      # new parameters, same buffers
    X.copy_(X2)
    changed = call().clone()
    assert not torch.equal(changed, first)
    ts.close()


def test_back_to_back_kernel_timing(api):
    """mt_profile_fitness_kernels: one launch per pass for a set of 64-atom
    cells, a positive time, Z of later fitness calls unchanged (graph replay
    and direct), both parameterisations; error codes for bad arguments."""
    import torch
    from paper_1909_11474_amd import _lib as L
    wl, refs = small_training(6)
    ts = api.from_structures(wl.structs)
    X = np.array(wl.population[:8])
    with pytest.raises(L.MTError) as e:
        ts.profile_fitness_kernels(X, "fp32", 4)
    assert e.value.code == L.MT_ENOREF
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    Z0 = ts.fitness(X, precision="fp32").clone()
    for x in (X, W.draw_params_full(np.random.Generator(np.random.PCG64(5)), 8)):
        for precision in ("fp32", "fp64"):
            ms, n = ts.profile_fitness_kernels(x, precision, 4)
            assert n == 1 and 0.0 < ms < 1000.0, (ms, n)
    assert torch.equal(ts.fitness(X, precision="fp32"), Z0)
    xt = torch.as_tensor(X, device="cuda").contiguous()
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    for nx, reps in ((7, 4), (6, 0)):
        rc = ts._lib.mt_profile_fitness_kernels(ts._handle, ctypes.c_void_p(xt.data_ptr()), nx, 8, 1,
                                                reps, ctypes.byref(ms), ctypes.byref(n), None)
        assert rc == L.MT_EINVAL, (nx, reps)
    ts.close()


def test_per_launch_kernel_timing(api):
    """mt_profile_fitness_launches on a set with two coordination classes
    (64-atom cells and packings): one entry per launch with its class, every
    structure mapped to the launch that evaluates it, the per-launch times
    adding up to about the per-pass time; too small a capacity is refused."""
    import torch
    from paper_1909_11474_amd import _lib as L
    g = np.random.Generator(np.random.PCG64(81))
    s = W.make_set(W.strained_diamond_cells(82, 4) + [W.random_packing(g, n) for n in (120, 300)])
    refs = T.reference_data(s, W.draw_params(np.random.Generator(np.random.PCG64(83)), 1)[0], R1, R2)
    ts = api.from_structures(s)
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    X = torch.as_tensor(W.draw_params(np.random.Generator(np.random.PCG64(84)), 40), device="cuda")
    # an idle GPU needs a moment of work to reach its clock: without it the
    # first timed launches (the per-launch pass) run slow and the two
    # timings disagree
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.3:
        ts.fitness(X, precision="fp32")
        torch.cuda.synchronize()
    launches, sl = ts.profile_fitness_launches(X, "fp32", 8)
    classes = sorted(mc for _, mc in launches)
    assert classes[0] == 4 and classes[-1] > 4
    assert all(0.0 < ms < 1000.0 for ms, _ in launches)
    assert sl[:4] == [sl[0]] * 4 and launches[sl[0]][1] == 4
    assert all(launches[l][1] > 4 for l in sl[4:])
    ms, n = ts.profile_fitness_kernels(X, "fp32", 8)
    assert n == len(launches)
    assert abs(sum(m for m, _ in launches) - ms) <= 0.5 * ms
    with pytest.raises(L.MTError) as e:
        ts.profile_fitness_launches(X, "fp32", 4, max_launches=1)
    assert e.value.code == L.MT_EINVAL
    ts.close()
