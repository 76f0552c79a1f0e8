"""Hand-written adjoint of randomized rounding (tt_round_rand_backward, and
the torch.autograd.Function around it) against the FP64 adjoint oracle and
central finite differences.

Tolerances: FP64 gradients vs the oracle <= 1e-9 relative per core (the QR
adjoint applies R^{-T}; the sketches here have modest condition numbers).
FP32 gradients vs the FP64 oracle <= 2e-4 relative per core (u32 = 6e-8
amplified by the sweep's conditioning).  Finite differences: central, FP64
with h = 1e-6 (error ~1e-9); the loss of the differentiation workload with
h = 1e-3 in FP64 (truncation error ~1e-6 relative).
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


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def case(seed, N, I, R, ell):
    dims, ranks = G.uniform_tt_shape(N, I, R)
    Y = G.random_tt(seed, dims, ranks, scale="nominal")
    ellv, outr = O.plan_ranks(dims, ranks, ell, 0)
    S = O.make_sketch(seed + 7, dims, ellv)
    rng = np.random.default_rng(seed + 11)
    Gc = [rng.standard_normal((outr[n], dims[n], outr[n + 1])) for n in range(N)]
    return Y, S, Gc, ell


@pytest.mark.parametrize("shape", [(4, 5, 6, 3), (6, 8, 10, 5), (2, 7, 4, 3), (5, 17, 33, 9)])
def test_backward_fp64_matches_oracle(gpu_lib, shape):
    from oracle.tt_adjoint import rto_vjp
    N, I, R, ell = shape
    say(f"adjoint fp64 N={N} I={I} R={R} l={ell}")
    Y, S, Gc, ell = case(101, N, I, R, ell)
    gi = host(gpu_lib.round_rand_backward(dev(Y), dev(Gc), ell, 0, seed=108))
    ref = rto_vjp(Y, S, Gc)
    errs = [rel(a, b) for a, b in zip(gi, ref)]
    print("per-core rel err", ["%.1e" % e for e in errs])
    assert max(errs) <= 1e-9


def test_backward_fp64_directional_fd(gpu_lib):
    # the GPU forward differenced against the GPU backward
    N, I, R, ell = 5, 6, 7, 4
    say("adjoint fp64 vs finite differences of the GPU forward")
    Y, S, Gc, ell = case(121, N, I, R, ell)
    rng = np.random.default_rng(5)
    D = [rng.standard_normal(c.shape) for c in Y]

    def f(t):
        out = host(gpu_lib.round_rand(dev([y + t * d for y, d in zip(Y, D)]), ell, 0, seed=128))
        return sum(float(np.sum(g * o)) for g, o in zip(Gc, out))

    h = 1e-6
    fd = (f(h) - f(-h)) / (2 * h)
    gi = host(gpu_lib.round_rand_backward(dev(Y), dev(Gc), ell, 0, seed=128))
    an = sum(float(np.sum(g * d)) for g, d in zip(gi, D))
    print(f"fd {fd:.10e} analytic {an:.10e}")
    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


def _diff_workload():
    # N=12, I=64, rank 64 rounded to 32 (no oversampling, no truncation);
    # T a random rank-32 TT; loss ||round(X) - T||^2
    N, I, R, ell = 12, 64, 64, 32
    dims, ranks = G.uniform_tt_shape(N, I, R)
    X = G.random_tt(1004, dims, ranks, scale="nominal")
    T = G.random_tt(1104, dims, [1] + [ell] * (N - 1) + [1], scale="nominal")
    return X, T, ell, 2004


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_autograd_loss_gradient_vs_oracle(gpu_lib, prec):
    from oracle.tt_adjoint import loss_round_minus_target, rto_torch
    say(f"autograd loss gradient, differentiation workload, {prec}")
    X, T, ell, seed = _diff_workload()
    dt = torch.float64 if prec == "f64" else torch.float32
    Xd = [c.requires_grad_(True) for c in dev(X, dt)]
    out = gpu_lib.round_rand_ad(Xd, ell, 0, seed=seed, prec=prec)
    Tt = [torch.from_numpy(c) for c in T]
    loss = loss_round_minus_target([o.double().cpu() for o in out], Tt)
    grads = host(torch.autograd.grad(loss, Xd))
    # oracle: same loss through the torch FP64 transcription, same sketch
    dims, ranks = O.dims_of(X), O.ranks_of(X)
    ellv, _ = O.plan_ranks(dims, ranks, ell, 0)
    S = O.make_sketch(seed, dims, ellv)
    if prec == "f32":
        X = [O.round_f32(c) for c in X]
        S = [O.round_f32(c) for c in S]
    Xt = [torch.tensor(c, requires_grad=True) for c in X]
    lo = loss_round_minus_target(rto_torch(Xt, [torch.tensor(c) for c in S]), Tt)
    ref = [g.numpy() for g in torch.autograd.grad(lo, Xt)]
    errs = [rel(a, b) for a, b in zip(grads, ref)]
    lg, lr = float(loss.detach()), float(lo.detach())
    print(f"loss gpu {lg:.6e} oracle {lr:.6e}; grad rel err max {max(errs):.2e}")
    assert abs(lg - lr) <= (1e-10 if prec == "f64" else 1e-4) * abs(lr)
    assert max(errs) <= (1e-8 if prec == "f64" else 2e-4)


def test_autograd_loss_fd_eps_1e3(gpu_lib):
    # directional finite difference with eps 1e-3 of the FP64 GPU loss
    from oracle.tt_adjoint import loss_round_minus_target
    say("loss finite difference, eps 1e-3")
    X, T, ell, seed = _diff_workload()
    Tt = [torch.from_numpy(c) for c in T]
    rng = np.random.default_rng(77)
    D = [rng.standard_normal(c.shape) * np.linalg.norm(c) / np.sqrt(c.size) for c in X]

    def loss_at(t):
        out = gpu_lib.round_rand(dev([x + t * d for x, d in zip(X, D)]), ell, 0, seed=seed)
        return float(loss_round_minus_target([o.cpu() for o in out], Tt).detach())

    h = 1e-3
    fd = (loss_at(h) - loss_at(-h)) / (2 * h)
    Xd = [c.requires_grad_(True) for c in dev(X)]
    out = gpu_lib.round_rand_ad(Xd, ell, 0, seed=seed)
    loss = loss_round_minus_target([o.cpu() for o in out], Tt)
    grads = host(torch.autograd.grad(loss, Xd))
    an = sum(float(np.sum(g * d)) for g, d in zip(grads, D))
    print(f"fd {fd:.8e} analytic {an:.8e}")
    assert abs(fd - an) <= 1e-4 * abs(an)


def test_backward_rejects_truncation(gpu_lib):
    from paper_2110_04393_amd import _lib as L
    Y = dev(G.random_tt(3, [5, 5, 5], [1, 4, 4, 1]))
    with pytest.raises(L.TTError) as e:
        gpu_lib.round_rand_backward(Y, [None, None, None], 2, 1, seed=1)
    assert e.value.status == L.TT_EUNSUPPORTED


@pytest.mark.parametrize("qr", ["auto", "householder"])
def test_backward_near_low_rank_fp64(gpu_lib, qr, monkeypatch):
    # X1 (rank 4) + 1e-4 X2 (rank 8) with sketch rank 6: every sketched
    # matrix Y_n has two weak columns (condition number about 1e4).  The
    # adjoint's R_n comes from the Q_n the forward produced (forced
    # Householder: the fallback path of the thin QR).
    from oracle.tt_adjoint import rto_vjp
    if qr == "householder":
        monkeypatch.setenv("TT_QR", "householder")
    say(f"adjoint fp64 near-low-rank qr={qr}")
    Y = G.near_low_rank_tt(131, [12] * 5, 4, 8, 1e-4)
    dims, ranks = O.dims_of(Y), O.ranks_of(Y)
    ellv, outr = O.plan_ranks(dims, ranks, 6, 0)
    S = O.make_sketch(138, dims, ellv)
    rng = np.random.default_rng(139)
    Gc = [rng.standard_normal((outr[n], dims[n], outr[n + 1])) for n in range(5)]
    gi = host(gpu_lib.round_rand_backward(dev(Y), dev(Gc), 6, 0, seed=138))
    ref = rto_vjp(Y, S, Gc)
    errs = [rel(a, b) for a, b in zip(gi, ref)]
    print("per-core rel err", ["%.1e" % e for e in errs])
    assert max(errs) <= 1e-7
    # and a directional finite difference of the GPU forward
    D = [rng.standard_normal(c.shape) for c in Y]

    def f(t):
        out = host(gpu_lib.round_rand(dev([y + t * d for y, d in zip(Y, D)]), 6, 0, seed=138))
        return sum(float(np.sum(g * o)) for g, o in zip(Gc, out))

    # the map is strongly curved here (its derivative carries 1/eps): a small
    # step keeps the central difference's h^2 term below the tolerance
    h = 1e-9
    fd = (f(h) - f(-h)) / (2 * h)
    an = sum(float(np.sum(g * d)) for g, d in zip(gi, D))
    print(f"fd {fd:.10e} analytic {an:.10e}")
    assert abs(fd - an) <= 1e-5 * max(1.0, abs(an))


def test_backward_reports_rank_deficient_sketch(gpu_lib):
    # A + A (exact rank 4) with sketch rank 6: the sketched matrices are
    # rank deficient and the adjoint of their thin QR is undefined
    from paper_2110_04393_amd import _lib as L
    say("adjoint of a rank-deficient sketch reports TT_ENUMERIC")
    A = G.random_tt(141, [8] * 4, [1, 4, 4, 4, 1])
    Y = G.block_sum([A, A])
    dims, ranks = O.dims_of(Y), O.ranks_of(Y)
    _, outr = O.plan_ranks(dims, ranks, 6, 0)
    Gc = [np.ones((outr[n], dims[n], outr[n + 1])) for n in range(4)]
    with pytest.raises(L.TTError) as e:
        gpu_lib.round_rand_backward(dev(Y), dev(Gc), 6, 0, seed=142)
    assert e.value.status == L.TT_ENUMERIC
