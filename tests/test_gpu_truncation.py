"""Truncation of the RtO output where kept singular directions lie far below
the largest one (near-low-rank inputs X1 + eps X2 of section 4.1 with the
target rank above the rank of X1): the GPU's Gram-based first pass is
followed by its second pass there.  Compared with the oracle's SVD
truncation as represented tensors, and the right-orthogonality of cores
2..N is checked."""
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


def right_orth_defect(cores):
    d = 0.0
    for c in cores[1:]:
        Hn = O.H(c)
        d = max(d, float(np.abs(Hn @ Hn.T - np.eye(Hn.shape[0])).max()))
    return d


@pytest.mark.parametrize("eig", ["auto", "jacobi"])
@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-8])
def test_truncation_keeps_weak_directions(gpu_lib, eps, eig, monkeypatch):
    # rank 8 + eps rank 40, sketch 16, target 12: four of the kept directions
    # are weak (singular values about eps of the strong ones)
    if eig == "jacobi":
        monkeypatch.setenv("TT_EIG", "jacobi")
    say(f"weak kept directions eps={eps} eig={eig}")
    Y = G.near_low_rank_tt(123, [40] * 5, 8, 40, eps)
    out = host(gpu_lib.round_rand(dev(Y), 12, 4, seed=3))
    ref = O.round_rand(Y, 12, 4, seed=3)
    assert O.ranks_of(out) == O.ranks_of(ref)
    err = O.rel_diff(out, ref)
    orth = right_orth_defect(out)
    print(f"rel diff {err:.3e}  right-orthogonality defect {orth:.3e}")
    assert err < 1e-10
    assert orth < 1e-12


def test_truncation_weak_directions_above_76(gpu_lib):
    # sketch rank 90 (> 76: the Jacobi solve of the first pass), target 80,
    # strong rank 70
    say("weak kept directions, l = 90")
    Y = G.near_low_rank_tt(321, [100] * 4, 70, 40, 1e-7)
    out = host(gpu_lib.round_rand(dev(Y), 80, 10, seed=4))
    ref = O.round_rand(Y, 80, 10, seed=4)
    assert O.ranks_of(out) == O.ranks_of(ref)
    err = O.rel_diff(out, ref)
    orth = right_orth_defect(out)
    print(f"rel diff {err:.3e}  right-orthogonality defect {orth:.3e}")
    assert err < 1e-10
    assert orth < 1e-12


def test_truncation_near_low_rank_workload_full_size(gpu_lib):
    # the near-low-rank benchmark input: N=30, I=100, rank 40 + 1e-6 rank 160,
    # sketch 60, target 50 (ten weak directions kept at every bond)
    say("near-low-rank workload N=30 I=100 40+1e-6*160 -> 60 -> 50")
    Y = G.near_low_rank_tt(1001, [100] * 30, 40, 160, 1e-6)
    out = host(gpu_lib.round_rand(dev(Y), 50, 10, seed=2001))
    ref = O.round_rand(Y, 50, 10, seed=2001)
    assert O.ranks_of(out) == O.ranks_of(ref)
    err = O.rel_diff(out, ref)
    orth = right_orth_defect(out)
    print(f"rel diff {err:.3e}  right-orthogonality defect {orth:.3e}")
    assert err < 1e-10
    assert orth < 1e-12


def test_truncation_target_above_exact_rank(gpu_lib):
    # A + A rounded with target 12 > rank(A) = 10 (sketch 15): two kept
    # directions carry only rounding noise; the result is still 2A and the
    # cores still right-orthogonal
    say("A+A target 12 > exact rank 10")
    w = G.workload_small_sum()
    twoA = [2.0 * w["A"][0]] + [c.copy() for c in w["A"][1:]]
    out = host(gpu_lib.round_rand(dev(w["X"]), 12, 3, seed=w["sketch_seed"]))
    err = O.rel_diff(out, twoA)
    orth = right_orth_defect(out)
    print(f"rel diff to 2A {err:.3e}  right-orthogonality defect {orth:.3e}")
    assert err <= 1e-12
    assert orth < 1e-10
