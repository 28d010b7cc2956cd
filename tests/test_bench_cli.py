"""bench.py's host-side contract, on the CPU: more than one GPU is refused
with a JSON message, the algorithmic flop count per atom follows its stated
formula, and the recorded HBM traffic is reported only for the kernel sources
it was measured on."""
import importlib.util
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_flops_per_atom_formula():
    b = load_bench()
    # algorithmic: 44 per directed pair + 55 per ordered triplet; diamond 836
    assert b.flops_per_atom(np.array([4]))[0] == 4 * 44 + 12 * 55 == 836
    assert b.flops_per_atom(np.array([0]))[0] == 0
    # the kernel's formulation: 6 bond pairs x 31 + 4 bonds x 70 + 9 for diamond
    assert b.kernel_flops_per_atom(np.array([4]))[0] == 6 * 31 + 4 * 70 + 9 == 475
    assert b.kernel_flops_per_atom(np.array([12]))[0] == 66 * 31 + 12 * 70 + 9


def test_gradient_and_force_call_flop_models():
    b = load_bench()
    # 13 x the forward count + 36 per bond; per-atom virial and heat current
    assert b.grad_flops_per_atom(np.array([4]))[0] == 13 * 836 + 144 == 11012
    assert b.force_call_flops_per_atom(np.array([4]))[0] == 836 + 72 + 18 == 926
    assert b.FORCE_CALL_BYTES_PER_ATOM == 144


def test_stored_references_are_checked_against_the_workload():
    import pytest

    import workloads as W
    b = load_bench()
    wl = W.config2()
    e, w, f = b.load_references(wl, "config2")
    assert e.shape == (100,) and w.shape == (100, 6) and f.shape == (6400, 3)
    other = W.config2(hidden_seed=99)
    with pytest.raises(SystemExit):
        b.load_references(other, "config2")


def test_traffic_is_tied_to_the_measured_sources(tmp_path):
    b = load_bench()
    t = b.measured_traffic()
    assert t is None or abs(t - (b.PMC_TRAFFIC["fetch_bytes"] + b.PMC_TRAFFIC["write_bytes"])) < 1
    b.PMC_TRAFFIC = dict(b.PMC_TRAFFIC, sha256_16="0" * 16)
    assert b.measured_traffic() is None


def test_cpu_oracle_legs_on_a_small_set():
    """The CPU-oracle legs time the oracle's fitness and its gradient on a
    bounded sample; the neighbour topology is built once per structure set and
    reported as setup."""
    import argparse

    import torch

    import workloads as W
    from oracle import tersoff as T

    b = load_bench()
    wl = W.config2(n_struct=3, pop=4)
    r = T.reference_data(wl.structs, wl.hidden_x, wl.R1, wl.R2)
    refs = tuple(torch.as_tensor(r[k]) for k in ("e", "w", "f"))
    args = argparse.Namespace(cpu_seconds=0.3)
    fit = b.oracle_rate(args, torch, wl, refs, grad=False)
    grad = b.oracle_rate(args, torch, wl, refs, grad=True)
    for leg in (fit, grad):
        assert leg["kind"] == "oracle" and leg["value"] > 0 and leg["cores"] >= 1
    assert grad["unit"].endswith("fitness-grad evals/s")
    assert grad["setup_s"]["topology"] < fit["setup_s"]["topology"] + 1e-3
    assert len(b._ORACLE_TOPOLOGY) == 1
