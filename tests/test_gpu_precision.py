"""Reduced-precision modes (FP32, and the BF16 partial contractions with FP32
accumulation) against the FP64 oracle run on the same inputs and the same
sketch values (the oracle's draw rounded to FP32, or to FP32 then bfloat16).

Tolerances.  FP32 storage has unit roundoff u32 = 2^-24 ~ 6e-8; the BF16
operands of the partial contractions carry u16 = 2^-9 ~ 2e-3 each.
* W chain in FP32: relative error per level <= 1e-5 (about 100 u32 for
  chains of a few levels with K up to a few thousand).
* W chain in BF16, last level only (products of bf16-exact inputs, FP32
  accumulation): <= 1e-5.  Longer BF16 chains: <= 3e-2 (each level rounds
  its operands to bf16, a relative perturbation of ~ 2 u16 per level).
* Rounding of a TT whose rank is within the sketch (A + A, or
  X1 + 1e-6 X2 with rank(X1) <= target): the output is insensitive to the
  sketch to first order, because range(Z_n W_n) stays inside range(Z_n)
  whatever W_n is, so both modes must match the oracle to <= 1e-4
  (the accuracy asked of the BF16 path), FP32 to <= 1e-5.
* Flat-spectrum inputs (every singular value of every unfolding alike) move
  with the sketch to first order; there the number is reported and only
  bounded loosely (no parity claim).
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


def dev(cores, dtype):
    return [torch.from_numpy(np.ascontiguousarray(c)).to(dtype).cuda() for c in cores]


def host(cores):
    torch.cuda.synchronize()
    return [c.detach().cpu().double().numpy() for c in cores]


def f32(cores):
    return [O.round_f32(c) for c in cores]


def oracle_sketch(prec, seed, dims, sr):
    sk = O.make_sketch(seed, dims, sr)
    return [O.round_bf16(c) if prec == "bf16" else O.round_f32(c) for c in sk]


# ------------------------------------------------------------------ sketch

def test_bf16_sketch_matches_oracle(gpu_lib):
    dims, sr = [100, 37, 100], [1, 60, 53, 1]
    say(f"bf16 sketch {dims} {sr}")
    S = host(gpu_lib.make_sketch(2001, dims, sr, dtype=torch.bfloat16))
    R = [O.round_bf16(c) for c in O.make_sketch(2001, dims, sr)]
    for a, b in zip(S, R):
        np.testing.assert_array_equal(a, b)


# ------------------------------------------------------------------ W chain

@pytest.mark.parametrize("mode", ["fused", "gemm"])
@pytest.mark.parametrize("case", [(5, 3, 4, 3), (6, 17, 37, 21), (4, 100, 200, 60),
                                  (4, 9, 30, 75), (4, 9, 32, 75), (4, 1, 4, 1)])
def test_wchain_f32(gpu_lib, case, mode, monkeypatch):
    if mode == "gemm":
        monkeypatch.setenv("TT_WCHAIN", "gemm")
    N, I, R, l = case
    say(f"W chain f32 {mode} N={N} I={I} R={R} l={l}")
    dims, ranks = G.uniform_tt_shape(N, I, R)
    X = f32(G.random_tt(11, dims, ranks, scale="nominal"))
    Y = f32(G.random_tt(12, dims, [1] + [l] * (N - 1) + [1], scale="def31"))
    W = gpu_lib.partial_contractions_rl(dev(X, torch.float32), dev(Y, torch.float32), prec="f32")
    Wo = O.partial_contractions_rl(X, Y)
    for n in range(1, N):
        a = W[n].double().cpu().numpy()
        err = np.linalg.norm(a - Wo[n]) / np.linalg.norm(Wo[n])
        assert err <= 1e-5, (n, err)


@pytest.mark.parametrize("IR", [(100, 61, 45), (7, 3, 5), (257, 33, 70)])
def test_wchain_bf16_last_level(gpu_lib, IR):
    # N = 2: W_1 = H(X_2) H(Y_2)^T with bf16-exact operands; only the FP32
    # accumulation rounds.  K = I spans whole 32-wide chunks and a ragged tail.
    I, R, l = IR
    say(f"W chain bf16 N=2 I={I} R={R} l={l}")
    X = [O.round_bf16(c) for c in G.random_tt(21, [5, I], [1, R, 1], scale="unit")]
    Y = [O.round_bf16(c) for c in G.random_tt(22, [5, I], [1, l, 1], scale="unit")]
    W = gpu_lib.partial_contractions_rl(dev(X, torch.float32), dev(Y, torch.float32),
                                        prec="bf16")
    Wo = O.partial_contractions_rl(X, Y)
    a = W[1].double().cpu().numpy()
    err = np.linalg.norm(a - Wo[1]) / np.linalg.norm(Wo[1])
    assert err <= 1e-5, err


@pytest.mark.parametrize("mode", ["fused", "gemm"])
@pytest.mark.parametrize("case", [(6, 40, 30, 20), (6, 40, 32, 20), (5, 17, 36, 70),
                                  (4, 100, 200, 60)])
def test_wchain_bf16_chain(gpu_lib, case, mode, monkeypatch):
    # R = 30: always the two products; R a multiple of 4: one fused kernel
    # per level (four or eight c-blocks) unless mode is "gemm"
    if mode == "gemm":
        monkeypatch.setenv("TT_WCHAIN", "gemm")
    N, I, R, l = case
    say(f"W chain bf16 {mode} N={N} I={I} R={R} l={l}")
    dims, ranks = G.uniform_tt_shape(N, I, R)
    X = f32(G.random_tt(31, dims, ranks, scale="nominal"))
    Y = f32(G.random_tt(32, dims, [1] + [l] * (N - 1) + [1], scale="def31"))
    W = gpu_lib.partial_contractions_rl(dev(X, torch.float32), dev(Y, torch.float32),
                                        prec="bf16")
    Wo = O.partial_contractions_rl(X, Y)
    errs = []
    for n in range(1, N):
        a = W[n].double().cpu().numpy()
        errs.append(np.linalg.norm(a - Wo[n]) / np.linalg.norm(Wo[n]))
    print("bf16 W chain errors per level", ["%.2e" % e for e in errs])
    assert max(errs) <= 3e-2
    assert max(errs) >= 1e-5  # the operands really went through bf16


@pytest.mark.parametrize("case", [(6, 40, 32, 20), (5, 17, 36, 70), (4, 100, 200, 60),
                                  (3, 9, 8, 17), (4, 1, 4, 1), (3, 2, 8, 96)])
def test_wchain_bf16_fused_matches_two_products(gpu_lib, case, monkeypatch):
    # both forms round Y_n, W_n, V(Y_n) W_n and the sketch to bf16 and
    # accumulate in fp32; they differ in the order of the fp32 sums only.
    # That order moves a Z entry by ~1e-5 relative after cancellation, so a
    # fraction p ~ 1e-5 / 2^-8 of the Z entries round to the neighbouring
    # bf16 value; each such entry is off by 2^-8, which moves a level by
    # about sqrt(p) 2^-8 ~ 2e-4 (compounding over the levels).  A wrong index
    # or a dropped block gives O(1) differences.
    N, I, R, l = case
    say(f"W chain bf16 fused vs two products N={N} I={I} R={R} l={l}")
    dims, ranks = G.uniform_tt_shape(N, I, R)
    X = dev(f32(G.random_tt(41, dims, ranks, scale="nominal")), torch.float32)
    Y = dev(f32(G.random_tt(42, dims, [1] + [l] * (N - 1) + [1], scale="def31")), torch.float32)
    Wf = [w.double().cpu().numpy() for w in gpu_lib.partial_contractions_rl(X, Y, prec="bf16")[1:]]
    monkeypatch.setenv("TT_WCHAIN", "gemm")
    Wg = [w.double().cpu().numpy() for w in gpu_lib.partial_contractions_rl(X, Y, prec="bf16")[1:]]
    for n, (a, b) in enumerate(zip(Wf, Wg), start=1):
        err = np.linalg.norm(a - b) / np.linalg.norm(b)
        assert err <= 2e-3, (n, err)


# ------------------------------------------------------------------ rounding

@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_round_A_plus_A(gpu_lib, prec):
    say(f"A+A -> 2A, {prec}")
    w = G.workload_small_sum()
    X = f32(w["X"])
    A = w["A"]
    twoA = [2.0 * A[0]] + [c.copy() for c in A[1:]]
    out = host(gpu_lib.round_rand(dev(X, torch.float32), w["target"], w["oversample"],
                                  seed=w["sketch_seed"], prec=prec))
    err = O.rel_diff(out, twoA)
    print(f"{prec}: rel err vs 2A {err:.3e}")
    assert err <= (1e-5 if prec == "f32" else 1e-4)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("shape", [(8, 12, 5, 20, 8, 4), (12, 30, 10, 30, 12, 5)])
def test_round_near_low_rank(gpu_lib, prec, shape):
    N, I, rlow, rhigh, target, over = shape
    say(f"near-low-rank {prec} N={N} I={I} rank {rlow}+1e-6*{rhigh} -> {target}")
    X = f32(G.near_low_rank_tt(41, [I] * N, rlow, rhigh, 1e-6))
    dims, ranks = O.dims_of(X), O.ranks_of(X)
    ell, _ = O.plan_ranks(dims, ranks, target, over)
    sk = oracle_sketch(prec, 4242, dims, ell)
    out = host(gpu_lib.round_rand(dev(X, torch.float32), target, over, seed=4242, prec=prec))
    ref = O.round_rand(X, target, over, sketch=sk)
    err = O.rel_diff(out, ref)
    print(f"{prec}: rel err vs oracle {err:.3e}")
    assert O.ranks_of(out) == O.ranks_of(ref)
    assert err <= (1e-5 if prec == "f32" else 1e-4)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_round_given_sketch(gpu_lib, prec):
    # caller-given FP32 sketch; the BF16 mode rounds it to bf16 itself
    N, I, target, over = 7, 9, 4, 3
    say(f"given sketch {prec}")
    X = f32(G.near_low_rank_tt(51, [I] * N, 3, 8, 1e-6))
    dims, ranks = O.dims_of(X), O.ranks_of(X)
    ell, _ = O.plan_ranks(dims, ranks, target, over)
    sk = f32(O.make_sketch(52, dims, ell))
    out = host(gpu_lib.round_rand(dev(X, torch.float32), target, over, prec=prec,
                                  sketch=dev(sk, torch.float32)))
    sk_used = [O.round_bf16(c) for c in sk] if prec == "bf16" else sk
    ref = O.round_rand(X, target, over, sketch=sk_used)
    err = O.rel_diff(out, ref)
    assert err <= (1e-5 if prec == "f32" else 1e-4), err


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_round_flat_spectrum_reported(gpu_lib, prec):
    # parity unpinned: the output moves with the sketch to first order
    N, I, R, target, over = 10, 20, 30, 10, 5
    say(f"flat spectrum {prec} N={N} I={I} R={R}")
    dims, ranks = G.uniform_tt_shape(N, I, R)
    X = f32(G.random_tt(61, dims, ranks, scale="nominal"))
    ell, _ = O.plan_ranks(dims, ranks, target, over)
    sk = oracle_sketch(prec, 62, dims, ell)
    out = host(gpu_lib.round_rand(dev(X, torch.float32), target, over, seed=62, prec=prec))
    ref = O.round_rand(X, target, over, sketch=sk)
    err = O.rel_diff(out, ref)
    print(f"{prec}: flat-spectrum rel err vs oracle {err:.3e}")
    # measured: FP32 3.2e-6, BF16 4.7e-2 (the BF16 operands move W_n by
    # about 2^-9 per level, and the output with it to first order)
    assert err <= (1e-4 if prec == "f32" else 0.2)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_long_train_renormalisation(gpu_lib, prec):
    # the partial contractions of this train fall far below the FP32 range
    # (checked on the oracle first); the power-of-two renormalisation keeps
    # the FP32 and BF16 chains finite and the result exact to tolerance
    N, I, target, over = 60, 16, 6, 4
    say(f"long train N={N} {prec}")
    X = f32(G.near_low_rank_tt(71, [I] * N, 4, 8, 1e-6))
    dims, ranks = O.dims_of(X), O.ranks_of(X)
    ell, _ = O.plan_ranks(dims, ranks, target, over)
    sk = oracle_sketch(prec, 72, dims, ell)
    W = O.partial_contractions_rl(X, sk)
    assert min(np.abs(w).max() for w in W[1:]) < 1e-45
    out = host(gpu_lib.round_rand(dev(X, torch.float32), target, over, seed=72, prec=prec))
    ref = O.round_rand(X, target, over, sketch=sk)
    err = O.rel_diff(out, ref)
    print(f"{prec}: long train rel err {err:.3e}")
    assert np.isfinite(err) and err <= (1e-5 if prec == "f32" else 1e-4)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_sum_near_low_rank(gpu_lib, prec):
    # 6 summands, multiples of two base TTs of rank 3 (exact rank <= 6 <= target)
    say(f"sum of 6 TTs {prec}")
    N, I = 8, 14
    dims = [I] * N
    base = [G.random_tt(81 + b, dims, [1] + [3] * (N - 1) + [1], scale="def31")
            for b in range(2)]
    summands = [f32(base[j % 2]) for j in range(6)]
    coeffs = [0.5, -1.25, 2.0, 0.75, -0.5, 1.0]
    target, over = 8, 4
    ell, _ = O.sum_plan(summands, target, over)
    sk = oracle_sketch(prec, 83, dims, ell)
    out = host(gpu_lib.sum_round([dev(t, torch.float32) for t in summands], coeffs, target, over,
                                 seed=83, prec=prec))
    ref = O.round_sum_rand(summands, coeffs, target, over, sketch=sk)
    err = O.rel_diff(out, ref)
    print(f"{prec}: sum rel err vs oracle {err:.3e}")
    assert O.ranks_of(out) == O.ranks_of(ref)
    assert err <= (1e-5 if prec == "f32" else 1e-4)


def test_dtype_mode_mismatch_rejected(gpu_lib):
    from paper_2110_04393_amd import _lib as L
    X = dev(G.random_tt(1, [4, 4, 4], [1, 2, 2, 1]), torch.float64)
    p = gpu_lib.RoundPlan([4, 4, 4], [1, 2, 2, 1], 2, 0, "f32", "cuda", dtype=torch.float32)
    with pytest.raises(L.TTError) as e:
        p.run(X, seed=1)
    assert e.value.status == L.TT_EINVAL
