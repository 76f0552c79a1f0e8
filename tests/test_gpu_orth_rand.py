"""Orthogonalize-then-Randomize (Algorithm 4, tt_round_orth_rand) against the
oracle's round_orth_rand on the same inputs and Gaussian matrices: FP64 core
by core within 1e-10 (the output is unique under the diag(R) >= 0 rule when
every sketch has full column rank) or as tensors after a truncation; exact
on A + A; FP32 on a near-low-rank input within 1e-5."""
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


def dev(cores, dtype=torch.float64):
    return [torch.from_numpy(np.ascontiguousarray(c)).to(dtype).cuda() for c in cores]


def host(cores):
    torch.cuda.synchronize()
    return [c.detach().cpu().double().numpy() for c in cores]


@pytest.mark.parametrize("case", [
    (4, 5, 6, 3, 0),       # tiny, no truncation
    (6, 9, 12, 5, 3),      # truncated
    (5, 40, 50, 20, 6),    # several tiles
    (3, 7, 12, 4, 2),      # wide last panel: I_N = 7 < R = 12 (bond drops to 7)
    (5, 100, 96, 40, 10),  # the largest supported bond rank
])
def test_orth_rand_matches_oracle(gpu_lib, case):
    N, I, R, t, p = case
    say(f"OtR {case}")
    dims, ranks = G.uniform_tt_shape(N, I, R)
    Y = G.random_tt(300 + N, dims, ranks, scale="nominal")
    out = host(gpu_lib.round_orth_rand(dev(Y), t, p, seed=7))
    ref = O.round_orth_rand(Y, t, p, seed=7)
    assert O.ranks_of(out) == O.ranks_of(ref)
    err = O.rel_diff(out, ref)
    print(f"rel diff vs oracle {err:.3e}")
    assert err < 1e-10
    if p == 0:  # no truncation: the cores themselves
        for a, b in zip(out, ref):
            np.testing.assert_allclose(a, b, atol=1e-10 * max(1.0, np.abs(b).max()))


def test_orth_rand_exact_on_small_sum_workload(gpu_lib):
    say("OtR A + A")
    w = G.workload_small_sum()
    twoA = [2.0 * w["A"][0]] + [c.copy() for c in w["A"][1:]]
    out = host(gpu_lib.round_orth_rand(dev(w["X"]), w["target"], w["oversample"], seed=3))
    assert O.rel_diff(out, twoA) <= 1e-12


def test_orth_rand_fp32_near_low_rank(gpu_lib):
    say("OtR FP32 near-low-rank")
    Y = [O.round_f32(c) for c in G.near_low_rank_tt(11, [20] * 6, 5, 10, 1e-6)]
    out = host(gpu_lib.round_orth_rand(dev(Y, torch.float32), 8, 4, seed=12, prec="f32"))
    ref = O.round_orth_rand(Y, 8, 4, seed=12)
    err = O.rel_diff(out, ref)
    print(f"f32 rel diff vs oracle {err:.3e}")
    assert err < 1e-5
