"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (RoundPlan with a preallocated workspace, internal device sketch)."""
import sys

import numpy as np
import pytest

import oracle as O
import tt_inputs as G

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def dev(cores):
    return [torch.from_numpy(np.ascontiguousarray(c)).cuda() for c in cores]


def host(cores):
    torch.cuda.synchronize()
    return [c.detach().cpu().numpy() for c in cores]


def test_single_tt_workload_fp64(gpu_lib):
    # N=30, I=100, rank 200 -> sketch 60 -> rank 50
    say("single TT workload N=30 I=100 R=200")
    w = G.workload_single_tt()
    X = w["X"]
    dims = [c.shape[1] for c in X]
    ranks = O.ranks_of(X)
    plan = gpu_lib.RoundPlan(dims, ranks, w["target"], w["oversample"], "f64", "cuda")
    Xd = dev(X)
    out = host(plan.run(Xd, seed=w["sketch_seed"]))
    ref = O.round_rand(X, w["target"], w["oversample"], seed=w["sketch_seed"])
    assert O.ranks_of(out) == O.ranks_of(ref) == [1] + [50] * 29 + [1]
    err = O.rel_diff(out, ref)
    print(f"rel err vs oracle {err:.3e}")
    assert err < 1e-10
    # a second call on the same plan (workspace reuse) is bitwise identical
    out2 = host(plan.run(Xd, seed=w["sketch_seed"]))
    for a, b in zip(out, out2):
        np.testing.assert_array_equal(a, b)


def test_small_sum_workload_fp64(gpu_lib):
    say("A+A workload (assembled) and as a sum")
    w = G.workload_small_sum()
    twoA = [2.0 * w["A"][0]] + [c.copy() for c in w["A"][1:]]
    out = host(gpu_lib.round_rand(dev(w["X"]), w["target"], w["oversample"],
                                  seed=w["sketch_seed"]))
    assert O.rel_diff(out, twoA) <= 1e-12
    outs = host(gpu_lib.sum_round([dev(w["A"]), dev(w["A"])], None, w["target"],
                                  w["oversample"], seed=w["sketch_seed"]))
    assert O.rel_diff(outs, twoA) <= 1e-12


def test_gmres_sum_workload_fp64(gpu_lib):
    # 20 summands, N=16, I=128, rank 20 each (formal 400) -> sketch 70 -> rank 60
    say("GMRES-like sum workload s=20 N=16 I=128")
    w = G.workload_gmres_sum()
    out = host(gpu_lib.sum_round([dev(t) for t in w["summands"]], w["coeffs"], w["target"],
                                 w["oversample"], seed=w["sketch_seed"]))
    ref = O.round_sum_rand(w["summands"], w["coeffs"], w["target"], w["oversample"],
                           seed=w["sketch_seed"])
    assert O.ranks_of(out) == O.ranks_of(ref)
    err = O.rel_diff(out, ref)
    print(f"rel err vs oracle {err:.3e}")
    assert err < 1e-10
