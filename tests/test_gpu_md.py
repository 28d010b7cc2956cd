"""GPU molecular dynamics (paper_1909_11474_amd/md.py: mt_md_kick / drift /
kinetic / scale and mt_set_update_positions around tersoff_eval) against the
oracle's velocity Verlet (oracle/md.py), and the invariants of the scheme.

Tolerances (float64): 20 steps of 1 fs on a thermal 64-atom cell, positions
1e-9 A, velocities 1e-10 A/fs, energies 1e-9 eV (rounding differences grow
slowly over a short chaotic trajectory); momentum 1e-10 u A/fs.
"""
import ctypes

import numpy as np
import pytest

import workloads as W
from oracle import md as OM

pytestmark = pytest.mark.gpu
X = np.array(W.TABLE2_X)


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


@pytest.fixture(scope="module")
def MDm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_11474_amd import md
    return md


def thermal(n, seed, T=500.0, masses=None):
    pos, cell = W.diamond(n, n, n)
    g = rng(seed)
    pos = W.displace(g, pos, 0.03)
    m = np.full(pos.shape[0], W.M_SI_AMU) if masses is None else masses
    v = g.normal(0.0, 1.0, size=pos.shape) * np.sqrt(W.KB_EV * T / (m[:, None] * W.AMU_A2_FS2_EV))
    v -= (m[:, None] * v).sum(0) / m.sum()
    return pos, cell, m, v


@pytest.mark.parametrize("drive", [False, True])
def test_trajectory_matches_the_oracle(MDm, drive):
    pos, cell, m, v = thermal(2, 81, masses=MDm.isotope_masses(64, rng(82)))
    fe = np.array([0.0, 0.0, 3e-3]) if drive else None
    md = MDm.MD(pos, cell, X, m, v, dt=1.0, fe=fe)
    recs = md.run(20)
    po, vo, ro = OM.velocity_verlet(pos, v, m, cell, X, 1.0, 20, fe=fe)
    print("max |dr|", np.abs(md.positions() - po).max(), "max |dv|", np.abs(md.velocities() - vo).max(), flush=True)
    assert np.abs(md.positions() - po).max() <= 1e-9
    assert np.abs(md.velocities() - vo).max() <= 1e-10
    for r, o in zip(recs, ro):
        assert abs(r["epot"] - o["epot"]) <= 1e-9 and abs(r["ekin"] - o["ekin"]) <= 1e-9
        assert np.abs(r["momentum"]).max() <= 1e-10
    md.close()


def test_heat_current_and_driving_power(MDm):
    """The kernel's J equals sum_i W_i v_i, and the driving force's power is F_e . J."""
    pos, cell, m, v = thermal(2, 83)
    fe = np.array([1e-3, -2e-3, 4e-3])
    md = MDm.MD(pos, cell, X, m, v, dt=1.0, fe=fe)
    md.run(5)
    md._forces()                          # J at the current (full-step) velocities
    Wi = md.Wi[0].cpu().numpy().reshape(3, 3, md.N)
    vel = md.vel.cpu().numpy()
    J = np.einsum("abi,bi->a", Wi, vel)
    Jk = md.J[0].cpu().numpy()
    assert np.abs(Jk - J).max() <= 1e-12 * max(np.abs(J).max(), 1.0)
    assert abs(md.external_power() - fe @ Jk) <= 1e-12 * max(abs(fe @ Jk), 1e-6)
    md.close()


def test_nve_energy_conservation_and_thermostat(MDm):
    """512 atoms: NVE total energy stays within 2e-4 eV/atom over 200 fs; a
    Berendsen thermostat brings 100 K to 600 K."""
    pos, cell, m, v = thermal(4, 84, T=600.0)
    md = MDm.MD(pos, cell, X, m, v, dt=1.0)
    e = np.array([r["etot"] for r in md.run(200)])
    print("NVE spread per atom", np.ptp(e) / md.N, flush=True)
    assert np.ptp(e) / md.N < 2e-4
    md.close()
    pos, cell, m, v = thermal(4, 85, T=100.0)
    md = MDm.MD(pos, cell, X, m, v, dt=1.0, thermostat=(600.0, 20.0))
    T = np.array([r["T"] for r in md.run(300)])
    print("T start", T[0], "end", T[-20:].mean(), flush=True)
    assert abs(T[-50:].mean() - 600.0) < 60.0
    md.close()


def test_hnemd_estimator_units(MDm):
    """kappa = <J> . F_e / (T V |F_e|^2) converts eV/(fs A K) to W/(m K)."""
    k = MDm.kappa_hnemd(np.array([0.0, 0.0, 1.0]), [0.0, 0.0, 1.0], 1.0, 1.0)
    assert abs(k - 1.602176634e6) < 1e-3


def test_position_update_semantics(MDm):
    """Updating to the same positions reproduces the bits; an update drops the
    reference data (MT_ENOREF until it is attached again); an update that
    overflows the neighbour capacity leaves the set unusable (MT_ESTATE)."""
    import torch
    from paper_1909_11474_amd import api, _lib as L
    from oracle import tersoff as T
    wl = W.config2(n_struct=3, pop=4)
    refs = T.reference_data(wl.structs, wl.hidden_x, 2.8, 3.2)
    ts = api.from_structures(wl.structs)
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    E0 = ts.tersoff_eval(wl.population, precision="fp64")["E"].clone()
    Z0 = ts.fitness(wl.population, precision="fp64").clone()
    pos = torch.as_tensor(wl.structs.pos.T.copy(), device="cuda").contiguous()
    L.check(ts._lib.mt_set_update_positions(ts._handle, ctypes_ptr(pos), None), "update")
    assert torch.equal(ts.tersoff_eval(wl.population, precision="fp64")["E"], E0)
    with pytest.raises(L.MTError) as e:
        ts.fitness(wl.population, precision="fp64")
    assert e.value.code == L.MT_ENOREF
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    assert torch.equal(ts.fitness(wl.population, precision="fp64"), Z0)
    ts.close()
    # capacity 4: a squeezed cell gives atoms more than 4 neighbours
    pos, cell = W.diamond(1, 1, 1)
    ts = api.TersoffSet(pos, cell[None], [0, 8], 2.8, 3.2, max_nbr=4)
    squeezed = torch.as_tensor((pos * 0.8).T.copy(), device="cuda").contiguous()
    rc = ts._lib.mt_set_update_positions(ts._handle, ctypes_ptr(squeezed), None)
    assert rc == L.MT_ENBR_OVERFLOW
    with pytest.raises(L.MTError) as e:
        ts.tersoff_eval(X[None], precision="fp64")
    assert e.value.code == L.MT_ESTATE
    ts.close()


def ctypes_ptr(t):
    import ctypes
    return ctypes.c_void_p(t.data_ptr())


def test_verlet_skin_gives_the_same_trajectory(MDm):
    """With a 0.5 A skin (geometry-only updates between rebuilds) the
    trajectory matches the oracle's as closely as with a rebuild every step,
    and the lists are rebuilt only when an atom has moved skin/2."""
    pos, cell, m, v = thermal(2, 86, T=900.0)
    md = MDm.MD(pos, cell, X, m, v, dt=1.0, skin=0.5, fe=(0.0, 2e-3, 0.0))
    md.run(40)
    po, vo, _ = OM.velocity_verlet(pos, v, m, cell, X, 1.0, 40, fe=(0.0, 2e-3, 0.0))
    print("skin rebuilds", md.rebuilds, "max |dr|", np.abs(md.positions() - po).max(), flush=True)
    assert np.abs(md.positions() - po).max() <= 1e-9
    assert np.abs(md.velocities() - vo).max() <= 1e-10
    assert md.rebuilds < 40
    md.close()


def test_eval_call_matches_tersoff_eval(MDm):
    """The pre-marshalled force call returns the same bits as tersoff_eval."""
    import torch
    from paper_1909_11474_amd import api
    pos, cell, m, v = thermal(2, 87)
    ts = api.TersoffSet(pos, cell[None], [0, pos.shape[0]])
    X = np.vstack([W.TABLE2_X, W.draw_params(rng(88), 1)])
    ref = ts.tersoff_eval(X, precision="fp64", atom_virial=True, velocities=v)
    call = ts.eval_call(X, precision="fp64", atom_virial=True, velocities=v)
    for _ in range(2):
        out = call()
        for k in ("E", "F", "W", "Wi", "J"):
            assert torch.equal(out[k], ref[k]), k
    X9 = W.draw_params_full(rng(89), 2)
    assert torch.equal(ts.eval_call(X9, precision="fp64")()["E"], ts.tersoff_eval(X9, precision="fp64")["E"])
    ts.close()


def test_force_calls_replay_in_a_graph(MDm):
    """Ten pre-marshalled force calls captured in one HIP graph replay to the
    eager result, with eager work between the replays."""
    import torch
    from paper_1909_11474_amd import api
    pos, cell, m, v = thermal(3, 90)
    ts = api.TersoffSet(pos, cell[None], [0, pos.shape[0]])
    call = ts.eval_call(np.array(W.TABLE2_X), precision="fp32", atom_virial=True, velocities=v)
    ref = {k: t.clone() for k, t in call().items()}
    other = ts.eval_call(W.draw_params(rng(91), 2), precision="fp64")
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cs):
        call()
    torch.cuda.current_stream().wait_stream(cs)
    with torch.cuda.graph(g):
        for _ in range(10):
            call()
    for _ in range(3):
        call.E.zero_(); call.F.zero_(); call.Wi.zero_(); call.J.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(call.E, ref["E"]) and torch.equal(call.F.transpose(1, 2), ref["F"])
        assert torch.equal(call.Wi.view(1, 3, 3, -1).permute(0, 3, 1, 2), ref["Wi"])
        assert torch.equal(call.J, ref["J"])
        other()                                          # eager work between replays
        torch.cuda.synchronize()
    del g
    ts.close()


def test_run_with_look_ahead_equals_single_steps(MDm):
    """run() issues the next step's kick, drift and displacement check before
    reading the step's scalars; stepping one call at a time does not.  Both
    give the same bits: records, positions, velocities and list rebuilds
    (0.5 A skin at 900 K, with the driving force)."""
    pos, cell, m, v = thermal(2, 92, T=900.0)
    a = MDm.MD(pos, cell, X, m, v, dt=1.0, skin=0.5, fe=(1e-3, 0.0, 2e-3))
    b = MDm.MD(pos, cell, X, m, v, dt=1.0, skin=0.5, fe=(1e-3, 0.0, 2e-3))
    ra = a.run(60)
    rb = [b.step() for _ in range(60)]
    print("rebuilds", a.rebuilds, b.rebuilds, flush=True)
    for x, y in zip(ra, rb):
        assert x["epot"] == y["epot"] and x["ekin"] == y["ekin"]
        assert np.array_equal(x["J"], y["J"]) and np.array_equal(x["momentum"], y["momentum"])
    assert np.array_equal(a.positions(), b.positions())
    assert np.array_equal(a.velocities(), b.velocities())
    assert a.rebuilds == b.rebuilds and a.rebuilds > 0
    a.close()
    b.close()


def test_float_path_after_position_updates(MDm):
    """The float path's geometry tables (packed bonds and the angle-cosine pair
    table) follow both kinds of position update: after mt_set_update_positions
    the float32 results equal those of a set built at the new positions bit for
    bit; after mt_set_update_geometry (0.5 A skin, atoms moved 0.02 A) they meet
    the float32 bar against the oracle (1e-6 eV/atom, 1e-4 eV/A, 1e-5 eV/atom
    virial)."""
    import torch
    from paper_1909_11474_amd import api, _lib as L
    from oracle import tersoff as T
    wl = W.config2(n_struct=4, pop=3)
    s = wl.structs
    g = rng(120)
    pos1 = W.displace(g, s.pos, 0.05)
    ts = api.from_structures(s)
    s1 = W.make_set([(pos1[s.offset[k]:s.offset[k + 1]], s.cell[k]) for k in range(s.n_struct)])
    fresh = api.from_structures(s1)
    p1 = torch.as_tensor(pos1.T.copy(), device="cuda").contiguous()
    L.check(ts._lib.mt_set_update_positions(ts._handle, ctypes_ptr(p1), None), "update")
    a = ts.tersoff_eval(wl.population, precision="fp32")
    b = fresh.tersoff_eval(wl.population, precision="fp32")
    for k in ("E", "F", "W"):
        assert torch.equal(a[k], b[k]), k
    fresh.close()
    L.check(ts._lib.mt_set_list_skin(ts._handle, ctypes.c_double(0.5), None), "skin")
    pos2 = W.displace(g, pos1, 0.02)
    p2 = torch.as_tensor(pos2.T.copy(), device="cuda").contiguous()
    L.check(ts._lib.mt_set_update_geometry(ts._handle, ctypes_ptr(p2), None), "geometry")
    out = ts.tersoff_eval(wl.population, precision="fp32")
    E, F, Wv = (out[k].cpu().numpy() for k in ("E", "F", "W"))
    s2 = W.make_set([(pos2[s.offset[k]:s.offset[k + 1]], s.cell[k]) for k in range(s.n_struct)])
    n = s2.sizes().astype(float)
    for c, x in enumerate(wl.population):
        ref = T.evaluate_set(s2, x, 2.8, 3.2)
        assert np.abs(E[c] / n - ref["E"] / n).max() <= 1e-6
        assert np.abs(F[c] - ref["F"]).max() <= 1e-4
        assert np.abs(Wv[c] / n[:, None] - ref["W6"] / n[:, None]).max() <= 1e-5
    ts.close()
