"""The speculative form of tt_round_rand / tt_sum_round (the guarded rescue
launches left out, the device flags read back once, the rounding redone in
the guarded form when one is set) against the guarded form alone
(TT_SPECULATE=0): the same kernels run on the same operands, so the results
agree bit for bit, both where no flag is set and where the redo takes over
(pivot breakdowns in the thin QR, the truncation's second pass, the
Householder rescue of a rank-deficient sketch).  Each case also meets the
oracle."""
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


def both_forms(monkeypatch, run):
    monkeypatch.delenv("TT_SPECULATE", raising=False)
    spec = host(run())
    monkeypatch.setenv("TT_SPECULATE", "0")
    guarded = host(run())
    monkeypatch.delenv("TT_SPECULATE", raising=False)
    return spec, guarded


def same_bits(a, b):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        assert x.shape == y.shape
        assert np.array_equal(x.view(np.uint64), y.view(np.uint64))


def test_well_conditioned_single_tt(gpu_lib, monkeypatch):
    say("speculative vs guarded: random TT N=12 I=20 R=30 -> 12 (+4)")
    Y = G.random_tt(4100, [20] * 12, [1] + [30] * 11 + [1])
    spec, guarded = both_forms(monkeypatch, lambda: gpu_lib.round_rand(dev(Y), 12, 4, seed=7))
    same_bits(spec, guarded)
    ref = O.round_rand(Y, 12, 4, seed=7)
    assert O.rel_diff(spec, ref) < 1e-10


def test_near_low_rank_redo(gpu_lib, monkeypatch):
    # strong rank 8 + 1e-8 rank 40, target 12: shifted CholeskyQR3 and the
    # truncation's second pass, so the speculative run is redone
    say("speculative vs guarded: near-low-rank 8 + 1e-8 * 40, target 12")
    Y = G.near_low_rank_tt(123, [40] * 5, 8, 40, 1e-8)
    spec, guarded = both_forms(monkeypatch, lambda: gpu_lib.round_rand(dev(Y), 12, 4, seed=3))
    same_bits(spec, guarded)
    ref = O.round_rand(Y, 12, 4, seed=3)
    assert O.rel_diff(spec, ref) < 1e-10


def test_rank_deficient_sum_redo(gpu_lib, monkeypatch):
    # A + A with target 12 > rank(A) = 10: the sketch is rank deficient, the
    # Householder rescue and null-row completion run in the redo
    say("speculative vs guarded: A+A, target 12 > rank 10")
    w = G.workload_small_sum()
    A = w["A"]
    run = lambda: gpu_lib.sum_round([dev(A), dev(A)], [1.0, 1.0], 12, 3, seed=w["sketch_seed"])
    spec, guarded = both_forms(monkeypatch, run)
    same_bits(spec, guarded)
    twoA = [2.0 * A[0]] + [c.copy() for c in A[1:]]
    assert O.rel_diff(spec, twoA) <= 1e-12


def test_benchmark_input_no_redo_bits(gpu_lib, monkeypatch):
    # the benchmark's single TT (N=30, I=100, R=200 -> 60 -> 50): no flag is
    # set, the speculative result is the guarded one
    say("speculative vs guarded: benchmark input N=30 I=100 R=200")
    w = G.workload_single_tt()
    X = w["X"]
    spec, guarded = both_forms(
        monkeypatch, lambda: gpu_lib.round_rand(dev(X), w["target"], w["oversample"],
                                                seed=w["sketch_seed"]))
    same_bits(spec, guarded)
