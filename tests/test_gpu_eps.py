"""Rounding to a tolerance with ranks not known in advance
(tt_round_rand_eps / tt_sum_round_eps; section 3.2, remark after
Algorithm 5) against the oracle's round_rand_eps on the same sketch: same
ranks at every bond, represented tensors within 1e-10 (FP64), and the bound
||X_out - X|| <= eps0 ||X|| of the truncation."""
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


@pytest.mark.parametrize("eps0", [1e-2, 1e-4, 1e-8])
@pytest.mark.parametrize("case", [
    (6, 12, 5, 10, 1e-6, 16),      # rank 5 + 1e-6 rank 10, sketch 16
    (8, 30, 12, 20, 1e-3, 24),     # several GEMM tiles
    (5, 40, 20, 40, 1e-9, 40),     # the sketch keeps weak directions (second pass)
])
def test_round_rand_eps_matches_oracle(gpu_lib, case, eps0):
    N, I, rl, rh, eps, ell = case
    say(f"eps rounding {case} eps0={eps0}")
    Y = G.near_low_rank_tt(61 + N, [I] * N, rl, rh, eps)
    out = host(gpu_lib.round_rand_eps(dev(Y), ell, eps0, seed=62))
    ref, rranks, _ = O.round_rand_eps(Y, ell, eps0, seed=62)
    X = O.round_rand(Y, ell, 0, seed=62, truncate=False)
    print("ranks", O.ranks_of(out))
    assert O.ranks_of(out) == rranks
    assert O.rel_diff(out, ref) < 1e-10
    assert O.rel_diff(out, X) <= eps0 * (1 + 1e-9)
    for c in out[1:]:
        Hn = O.H(c)
        assert np.abs(Hn @ Hn.T - np.eye(Hn.shape[0])).max() < 1e-12


def test_round_rand_eps_near_low_rank_workload(gpu_lib):
    # N=30, I=100, rank 40 + 1e-6 rank 160, sketch rank 60, eps0 1e-4: the
    # tolerance recovers rank 40 at every bond
    say("eps rounding of the near-low-rank workload, eps0 1e-4")
    Y = G.near_low_rank_tt(1001, [100] * 30, 40, 160, 1e-6)
    out = host(gpu_lib.round_rand_eps(dev(Y), 60, 1e-4, seed=2001))
    ref, rranks, _ = O.round_rand_eps(Y, 60, 1e-4, seed=2001)
    assert O.ranks_of(out) == rranks == [1] + [40] * 29 + [1]
    err = O.rel_diff(out, ref)
    print(f"rel diff vs oracle {err:.3e}; vs input {O.rel_diff(out, Y):.3e}")
    assert err < 1e-10


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_sum_round_eps_matches_oracle(gpu_lib, prec):
    # 6 summands, multiples of two base TTs of rank 3 and one 1e-7 TT of rank 4
    say(f"eps rounding of a sum, {prec}")
    N, I = 7, 10
    dims = [I] * N
    base = [G.random_tt(71 + b, dims, [1] + [3] * (N - 1) + [1]) for b in range(2)]
    weak = [1e-7 * c if n == 0 else c for n, c in
            enumerate(G.random_tt(79, dims, [1] + [4] * (N - 1) + [1]))]
    summands = [base[j % 2] for j in range(5)] + [weak]
    coeffs = [0.5, -1.25, 2.0, 0.75, 1.5, 1.0]
    if prec == "f32":
        summands = [[O.round_f32(c) for c in t] for t in summands]
    dt = torch.float64 if prec == "f64" else torch.float32
    out = host(gpu_lib.sum_round_eps([dev(t, dt) for t in summands], coeffs, 12, 1e-4,
                                     seed=72, prec=prec))
    sk = O.make_sketch(72, dims, O.sum_plan(summands, 12, 0)[0])
    if prec == "f32":
        sk = [O.round_f32(c) for c in sk]
    ref, rranks, _ = O.round_sum_rand_eps(summands, coeffs, 12, 1e-4, sketch=sk)
    assert O.ranks_of(out) == rranks == [1] + [6] * (N - 1) + [1]
    err = O.rel_diff(out, ref)
    print(f"{prec}: rel diff vs oracle {err:.3e}")
    assert err < (1e-10 if prec == "f64" else 1e-5)


def test_round_rand_eps_zero_keeps_sketch_ranks(gpu_lib):
    say("eps rounding with eps0 = 0")
    dims, ranks = G.uniform_tt_shape(5, 6, 4)
    Y = G.random_tt(81, dims, ranks, scale="nominal")
    out = host(gpu_lib.round_rand_eps(dev(Y), 7, 0.0, seed=82))
    ref = O.round_rand(Y, 7, 0, seed=82, truncate=False)
    assert O.ranks_of(out) == O.ranks_of(ref)
    assert O.rel_diff(out, ref) < 1e-12
