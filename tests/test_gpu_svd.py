"""Deterministic TT-rounding on the GPU (Algorithms 1 and 2) against the FP64
oracle's round_svd on the same inputs.  Outputs are compared as tensors
(the gauge of intermediate cores is not unique when a bond rank drops), plus
the orthogonality of the output cores and the eps bound of Algorithm 2."""
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


def dev(cores, dtype=None):
    dtype = dtype or torch.float64
    return [torch.from_numpy(np.ascontiguousarray(c)).to(dtype).cuda() for c in cores]


def host(cores):
    torch.cuda.synchronize()
    return [c.detach().cpu().double().numpy() for c in cores]


def left_orth_dev(cores):
    dev_ = 0.0
    for c in cores[:-1]:
        Vn = c.reshape(-1, c.shape[2])
        dev_ = max(dev_, float(np.abs(Vn.T @ Vn - np.eye(Vn.shape[1])).max()))
    return dev_


@pytest.mark.parametrize("case", [
    ([5, 6, 4, 5, 3, 4], [1, 5, 8, 8, 6, 4, 1], 4),   # fixed rank
    ([3, 4, 5, 3], [1, 3, 8, 6, 1], 3),                # bonds above the mode sizes
    ([7, 9], [1, 7, 1], 2),                            # N = 2
    ([10] * 8, [1] + [20] * 7 + [1], 10),              # A+A sized
])
def test_round_svd_fixed_rank(gpu_lib, case):
    dims, ranks, k = case
    say(f"round_svd fixed rank dims={dims} ranks={ranks} k={k}")
    Y = G.random_tt(301, dims, ranks, scale="nominal")
    out = host(gpu_lib.round_svd(dev(Y), eps0=0.0, max_rank=k))
    ref, rr, _ = O.round_svd(Y, 0.0, k)
    assert O.ranks_of(out) == rr
    err = O.rel_diff(out, ref)
    print(f"rel err vs oracle {err:.3e}")
    assert err <= 1e-10
    assert left_orth_dev(out) <= 1e-12


@pytest.mark.parametrize("eps0", [1e-3, 1e-7])
def test_round_svd_eps(gpu_lib, eps0):
    # singular values with clear gaps: X1 (rank 4) + 1e-5 X2 (rank 6)
    say(f"round_svd eps0={eps0}")
    Y = G.near_low_rank_tt(311, [6] * 7, 4, 6, 1e-5)
    out_t = gpu_lib.round_svd(dev(Y), eps0=eps0)
    out = host(out_t)
    ref, rr, _ = O.round_svd(Y, eps0)
    assert O.ranks_of(out) == rr
    assert O.rel_diff(out, ref) <= 1e-9
    assert O.rel_diff(out, Y) <= eps0 * (1 + 1e-9)
    assert left_orth_dev(out) <= 1e-12


def test_round_svd_A_plus_A(gpu_lib):
    say("round_svd A+A -> 2A")
    w = G.workload_small_sum()
    out = host(gpu_lib.round_svd(dev(w["X"]), eps0=1e-10))
    twoA = [2.0 * w["A"][0]] + [c.copy() for c in w["A"][1:]]
    assert O.ranks_of(out) == O.ranks_of(w["A"])
    assert O.rel_diff(out, twoA) <= 1e-12


def test_round_svd_f32(gpu_lib):
    say("round_svd f32")
    Y = [O.round_f32(c) for c in G.near_low_rank_tt(321, [5] * 6, 3, 5, 1e-3)]
    out = host(gpu_lib.round_svd(dev(Y, torch.float32), eps0=0.0, max_rank=3, prec="f32"))
    ref, rr, _ = O.round_svd(Y, 0.0, 3)
    assert O.ranks_of(out) == rr
    assert O.rel_diff(out, ref) <= 1e-5


def test_round_svd_single_core(gpu_lib):
    Y = G.random_tt(5, [7], [1, 1])
    out = host(gpu_lib.round_svd(dev(Y), eps0=0.1))
    np.testing.assert_array_equal(out[0], Y[0])


def test_round_svd_largest_bond(gpu_lib):
    # bond rank 96, the largest the comparator takes (the Cholesky and Jacobi
    # solvers of n = 96), kept rank 50: the configuration bench.py times it on
    # (there N = 30, I = 100)
    say("round_svd N=6 I=100 R=96 -> 50")
    Y = G.random_tt(303, [100] * 6, [1] + [96] * 5 + [1], scale="nominal")
    out = host(gpu_lib.round_svd(dev(Y), eps0=0.0, max_rank=50))
    ref, rr, _ = O.round_svd(Y, 0.0, 50)
    assert O.ranks_of(out) == rr
    err = O.rel_diff(out, ref)
    print(f"rel err vs oracle {err:.3e}")
    assert err <= 1e-10
    assert left_orth_dev(out) <= 1e-12
