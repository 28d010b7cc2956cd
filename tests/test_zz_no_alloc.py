"""fitness_eval_noalloc (the allocation-free fitness entry point) against
fitness_eval: the same bits on two calls in a row, the second with fewer
candidates, in both precisions; its refusals (no work list yet, scratch too
small, two-pass structures)."""
import ctypes

import numpy as np
import pytest

import workloads as W
from oracle import tersoff as T

pytestmark = pytest.mark.gpu

R1, R2 = 2.8, 3.2


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1909_11474_amd import api, _lib
    # 64-atom cells (one wavefront per replica) and packings of 100-250 atoms
    # (several wavefronts per replica, coordination classes above 4)
    g = rng(71)
    structs = W.make_set(W.strained_diamond_cells(72, 6) +
                         [W.random_packing(g, n) for n in (100, 180, 250)])
    refs = T.reference_data(structs, W.draw_params(rng(73), 1)[0], R1, R2)
    ts = api.from_structures(structs)
    ts.attach_reference(refs["e"], refs["w"], refs["f"])
    yield torch, api, _lib, ts, structs, refs
    ts.close()


def noalloc(L, ts, X, Z, precision, w=(1.0, 1.0, 1.0)):
    import torch
    lib = L.load()
    wt = (ctypes.c_double * 3)(*w)
    prec = L.MT_FP64 if precision == "fp64" else L.MT_FP32_ACC64
    rc = lib.fitness_eval_noalloc(ts._handle, ctypes.c_void_p(X.data_ptr()), X.shape[0], wt, prec,
                                  ctypes.c_void_p(Z.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_matches_fitness_eval(env, precision):
    torch, api, L, ts, structs, refs = env
    w = (1.0, 0.7, 1.3)
    for P, seed in ((40, 74), (12, 75)):          # the second call with fewer candidates
        X = torch.as_tensor(W.draw_params(rng(seed), P), device="cuda").contiguous()
        Zref = ts.fitness(X, w, precision=precision)          # builds the work list
        Z = torch.full((P, 4), float("nan"), dtype=torch.float64, device="cuda")
        assert noalloc(L, ts, X, Z, precision, w) == L.MT_OK, L.load().mt_last_error()
        torch.cuda.synchronize()
        print(f"{precision} P={P}: max |Z_noalloc - Z| = {float((Z - Zref).abs().max()):.3e}", flush=True)
        assert torch.equal(Z, Zref)
        Zo = T.fitness(structs, X[[0, P - 1]].cpu().numpy(), refs, w)
        tol = 1e-10 if precision == "fp64" else 1e-5
        assert np.abs(Z[[0, P - 1]].cpu().numpy() - Zo).max() <= tol * np.abs(Zo).max()


def test_noalloc_refusals(env):
    torch, api, L, ts, structs, refs = env
    X = torch.as_tensor(W.draw_params(rng(76), 7), device="cuda").contiguous()
    Z = torch.empty(7, 4, dtype=torch.float64, device="cuda")
    assert noalloc(L, ts, X, Z, "fp64") == L.MT_ESTATE          # no work list for P = 7 yet
    ts.fitness(X, precision="fp64")
    assert noalloc(L, ts, X, Z, "fp64") == L.MT_OK
    # P x slots x 64 bytes beyond the fixed array: refused before any launch
    # (x and Z are not read)
    nslots_min = structs.n_struct
    P_big = L.MT_NOALLOC_SCRATCH_BYTES // (64 * nslots_min) + 1
    lib = L.load()
    wt = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    rc = lib.fitness_eval_noalloc(ts._handle, ctypes.c_void_p(X.data_ptr()), P_big, wt, L.MT_FP64,
                                  ctypes.c_void_p(Z.data_ptr()), None)
    assert rc == L.MT_EINVAL
    # a structure over 512 atoms (two-pass path)
    big = W.make_set([W.random_packing(rng(77), 600)])
    refs2 = T.reference_data(big, W.draw_params(rng(78), 1)[0], R1, R2)
    ts2 = api.from_structures(big)
    ts2.attach_reference(refs2["e"], refs2["w"], refs2["f"])
    ts2.fitness(X, precision="fp64")
    assert noalloc(L, ts2, X, Z, "fp64") == L.MT_EINVAL
    ts2.close()
