"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics
(brute force on tiny tensors, closed forms, exact identities, invariants,
error bounds).  CPU only."""
import math

import numpy as np
import pytest

import oracle as O
import tt_inputs as G

RNG_SEEDS = [0, 1, 2]


def tiny_tt(seed, N=5, I=3, R=4, scale="unit"):
    dims, ranks = G.uniform_tt_shape(N, I, R)
    return G.random_tt(seed, dims, ranks, scale=scale)


# ---------------------------------------------------------------- generator

def _mix_int(z):
    M = (1 << 64) - 1
    z &= M
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return z ^ (z >> 31)


def test_splitmix64_matches_python_integers():
    # the numpy uint64 version must equal arbitrary-precision integer arithmetic
    for state in [0, 1, 12345, (1 << 64) - 1, 0x0123456789ABCDEF]:
        idx = np.arange(1, 40, dtype=np.uint64)
        got = O.splitmix64_stream(state, idx)
        want = [_mix_int(state + int(k) * 0x9E3779B97F4A7C15) for k in range(1, 40)]
        assert [int(x) for x in got] == want


def test_gaussian_stream_box_muller_closed_form():
    key = O.sketch_core_key(7, 3)
    z = O.gaussian_stream(key, 9)
    M = (1 << 64) - 1
    for p in range(5):
        a = _mix_int((key + (2 * p + 1) * 0x9E3779B97F4A7C15) & M)
        b = _mix_int((key + (2 * p + 2) * 0x9E3779B97F4A7C15) & M)
        u1 = ((a >> 11) + 1) / 2.0 ** 53
        u2 = (b >> 11) / 2.0 ** 53
        r = math.sqrt(-2.0 * math.log(u1))
        assert z[2 * p] == pytest.approx(r * math.cos(2 * math.pi * u2), rel=0, abs=1e-14)
        if 2 * p + 1 < 9:
            assert z[2 * p + 1] == pytest.approx(r * math.sin(2 * math.pi * u2), rel=0, abs=1e-14)


def test_sketch_distribution_definition_31():
    # Definition 3.1: iid N(0, 1/(l_{n-1} I_n l_n)) entries, E||core||^2 = 1
    dims = [40, 50, 30]
    ell = [1, 40, 30, 1]
    S = O.make_sketch(99, dims, ell)
    for c in S:
        x = c.ravel()
        n = x.size
        var = 1.0 / n
        assert abs(x.mean()) < 6 * math.sqrt(var / n)
        assert abs(x.var() / var - 1.0) < 6 * math.sqrt(2.0 / n)
        kurt = np.mean(x ** 4) / np.mean(x ** 2) ** 2
        assert abs(kurt - 3.0) < 0.2
    # seeds and cores give distinct streams
    S2 = O.make_sketch(100, dims, ell)
    assert not np.allclose(S[1], S2[1])
    assert O.sketch_core_key(1, 0) != O.sketch_core_key(1, 1)


# ---------------------------------------------------------------- plan

def test_plan_ranks_small_sum_workload():
    # A+A assembled: N=8, I=10, formal rank 20, target 10, oversample 5
    ell, out = O.plan_ranks([10] * 8, [1] + [20] * 7 + [1], 10, 5)
    assert ell == [1, 10, 15, 15, 15, 15, 15, 10, 1]
    assert out == [1] + [10] * 7 + [1]


def test_plan_ranks_clamps():
    ell, out = O.plan_ranks([2, 2, 2, 2], [1, 2, 4, 2, 1], 6, 2)
    assert ell == [1, 2, 4, 2, 1]
    assert out == [1, 2, 4, 2, 1]
    for n in range(1, 4):
        assert ell[n] <= ell[n - 1] * 2


# ---------------------------------------------------------------- Algorithm 3

@pytest.mark.parametrize("seed", RNG_SEEDS)
def test_partial_contractions_brute_force(seed):
    # closed form W_n = H(X_{n+1:N}) H(Y_{n+1:N})^T by dense partial products
    X = tiny_tt(seed, N=5, I=3, R=4)
    Y = G.random_tt(seed + 50, [3] * 5, [1, 2, 3, 3, 2, 1], scale="unit")
    W = O.partial_contractions_rl(X, Y)
    for n in range(1, 5):
        A = O.full_with_left_rank(X[n:])
        B = O.full_with_left_rank(Y[n:])
        np.testing.assert_allclose(W[n], A @ B.T, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", RNG_SEEDS)
def test_inner_product_is_sum_of_squares(seed):
    # appendix A: Algorithm 3 with both tensors equal yields ||Y||^2
    Y = tiny_tt(seed, N=6, I=3, R=3)
    T = O.full(Y)
    assert O.inner(Y, Y) == pytest.approx(float(np.sum(T * T)), rel=1e-12)
    assert O.tt_norm(Y) == pytest.approx(float(np.linalg.norm(T)), rel=1e-12)


def test_sum_stacking_identity():
    # section 3.4: W^{Y+Z}_n = [W^Y_n ; W^Z_n]
    A = tiny_tt(3, N=5, I=3, R=3)
    B = G.random_tt(4, [3] * 5, [1, 2, 4, 2, 2, 1], scale="unit")
    S = G.random_tt(5, [3] * 5, [1, 3, 3, 3, 3, 1], scale="unit")
    X = G.block_sum([A, B])
    WX = O.partial_contractions_rl(X, S)
    WA = O.partial_contractions_rl(A, S)
    WB = O.partial_contractions_rl(B, S)
    for n in range(1, 5):
        np.testing.assert_allclose(WX[n], np.vstack([WA[n], WB[n]]), rtol=0, atol=1e-14)


# ---------------------------------------------------------------- Algorithm 5

def _sketch(seed, Y, target, over):
    ell, out = O.plan_ranks(O.dims_of(Y), O.ranks_of(Y), target, over)
    return O.make_sketch(seed, O.dims_of(Y), ell), ell, out


@pytest.mark.parametrize("seed", RNG_SEEDS)
def test_rto_equals_dense_range_finder(seed):
    # Algorithm 5 is the sequential range finder on unfoldings in factored form
    Y = tiny_tt(seed, N=5, I=4, R=5)
    S, ell, _ = _sketch(seed + 10, Y, 3, 0)
    X = O.rto_sweep(Y, O.partial_contractions_rl(Y, S))
    D = O.dense_rto(O.full(Y), S)
    for a, b in zip(X, D):
        assert a.shape == b.shape
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-11 * max(1.0, np.abs(b).max()))


def test_rto_exact_on_small_sum_workload():
    # rounding A+A (rank 10 formally 20) to 10 through a 15 sketch returns 2A
    w = G.workload_small_sum()
    X = O.round_rand(w["X"], w["target"], w["oversample"], seed=w["sketch_seed"])
    twoA = [2.0 * w["A"][0]] + [c.copy() for c in w["A"][1:]]
    assert O.rel_diff(X, twoA) <= 1e-12
    assert O.ranks_of(X) == [1] + [10] * 7 + [1]


@pytest.mark.parametrize("seed", RNG_SEEDS)
def test_rto_output_left_orthogonal(seed):
    Y = tiny_tt(seed, N=6, I=4, R=6, scale="nominal")
    S, ell, _ = _sketch(seed, Y, 4, 1)
    X = O.rto_sweep(Y, O.partial_contractions_rl(Y, S))
    for c in X[:-1]:
        Vn = O.V(c)
        assert np.abs(Vn.T @ Vn - np.eye(Vn.shape[1])).max() < 1e-13


def test_rto_exact_when_ranks_suffice():
    # every unfolding rank <= l_n  =>  X == Y
    Y = tiny_tt(11, N=6, I=3, R=3, scale="nominal")
    X = O.round_rand(Y, 3, 2, seed=5)
    assert O.rel_diff(X, Y) < 1e-13


def test_rto_gauge_invariance():
    # Y_n <- Y_n G, Y_{n+1} <- G^{-1} Y_{n+1} leaves the output unchanged
    Y = tiny_tt(21, N=5, I=4, R=5, scale="nominal")
    rng = np.random.default_rng(0)
    Y2 = [c.copy() for c in Y]
    for n in range(4):
        Gm = rng.standard_normal((5, 5)) + 3 * np.eye(5)
        Y2[n] = (O.V(Y2[n]) @ Gm).reshape(Y2[n].shape)
        Y2[n + 1] = (np.linalg.solve(Gm, O.H(Y2[n + 1]))).reshape(Y2[n + 1].shape)
    S, ell, _ = _sketch(3, Y, 3, 0)
    X1 = O.rto_sweep(Y, O.partial_contractions_rl(Y, S))
    X2 = O.rto_sweep(Y2, O.partial_contractions_rl(Y2, S))
    for a, b in zip(X1, X2):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-10 * max(1, np.abs(a).max()))


def test_rto_sketch_scale_invariance():
    # Q depends only on the range of the sketch: positive core scalings cancel
    Y = tiny_tt(22, N=5, I=4, R=5, scale="nominal")
    S, ell, _ = _sketch(4, Y, 3, 0)
    S2 = [c * s for c, s in zip(S, [2.0 ** 30, 3.0, 0.25, 7.0, 1e-20])]
    X1 = O.rto_sweep(Y, O.partial_contractions_rl(Y, S))
    X2 = O.rto_sweep(Y, O.partial_contractions_rl(Y, S2))
    for a, b in zip(X1, X2):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-11 * max(1, np.abs(a).max()))


@pytest.mark.parametrize("seed", RNG_SEEDS)
def test_randomized_error_lower_bounds(seed):
    # Eckart-Young on every unfolding, and TT-SVD quasi-optimality
    Y = tiny_tt(seed, N=5, I=4, R=6, scale="nominal")
    X = O.round_rand(Y, 3, 1, seed=seed + 7)
    T = O.full(Y)
    err = np.linalg.norm(O.full(X) - T)
    dims = O.dims_of(Y)
    for n in range(1, 5):
        s = np.linalg.svd(T.reshape(int(np.prod(dims[:n])), -1), compute_uv=False)
        r = O.ranks_of(X)[n]
        assert err >= math.sqrt(np.sum(s[r:] ** 2)) * (1 - 1e-12)
    Xs, _, _ = O.round_svd(Y, 0.0, 3)
    assert err >= np.linalg.norm(O.full(Xs) - T) / math.sqrt(4) * (1 - 1e-12)


# ---------------------------------------------------------------- truncation

def test_truncation_equals_dense_tt_svd_from_the_right():
    # R->L truncation of a left-orthogonal TT == TT-SVD of the mode-reversed tensor
    Y = tiny_tt(31, N=5, I=4, R=6, scale="nominal")
    S, ell, out = _sketch(8, Y, 3, 3)
    X = O.rto_sweep(Y, O.partial_contractions_rl(Y, S))
    Xt, tails = O.truncate_rl(X, out)
    assert O.ranks_of(Xt) == out
    T = O.full(X)
    Trev = np.transpose(T, axes=list(range(4, -1, -1)))
    D = O.dense_tt_svd(Trev, out[::-1])
    Dfull = np.transpose(O.full(D), axes=list(range(4, -1, -1)))
    np.testing.assert_allclose(O.full(Xt), Dfull, rtol=0, atol=1e-12)
    # discarded energy adds up (orthogonal projections)
    err2 = np.sum((O.full(Xt) - T) ** 2)
    assert err2 == pytest.approx(sum(tails), rel=1e-8, abs=1e-28)
    # cores 2..N right-orthogonal
    for c in Xt[1:]:
        Hn = O.H(c)
        assert np.abs(Hn @ Hn.T - np.eye(Hn.shape[0])).max() < 1e-12


# ---------------------------------------------------------------- Algorithm 7

@pytest.mark.parametrize("s", [2, 3, 5])
def test_sum_rto_equals_rto_on_assembled_sum(s):
    dims = [4] * 5
    tts = [G.random_tt(40 + j, dims, [1, 2 + j % 2, 3, 2, 2 + j % 3, 1], scale="nominal")
           for j in range(s)]
    coeffs = G.sum_coefficients(7, s)
    Xs = G.block_sum(tts, coeffs)
    A = O.round_sum_rand(tts, coeffs, 4, 1, seed=77)
    B = O.round_rand(Xs, 4, 1, seed=77)
    for a, b in zip(A, B):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-11 * max(1, np.abs(b).max()))


def test_sum_rto_exact_small_workload():
    w = G.workload_small_sum()
    X = O.round_sum_rand(w["summands"], None, w["target"], w["oversample"],
                         seed=w["sketch_seed"])
    twoA = [2.0 * w["A"][0]] + [c.copy() for c in w["A"][1:]]
    assert O.rel_diff(X, twoA) <= 1e-12


# ---------------------------------------------------------------- Algorithms 1, 2

def test_orthogonalize_rl_right_orthogonal_and_equivalent():
    Y = tiny_tt(51, N=5, I=3, R=4)
    X = O.orthogonalize_rl(Y)
    for c in X[1:]:
        Hn = O.H(c)
        assert np.abs(Hn @ Hn.T - np.eye(Hn.shape[0])).max() < 1e-13
    np.testing.assert_allclose(O.full(X), O.full(Y), rtol=0, atol=1e-12 * np.abs(O.full(Y)).max())


@pytest.mark.parametrize("seed", RNG_SEEDS)
def test_round_svd_equals_dense_tt_svd(seed):
    Y = tiny_tt(seed, N=5, I=4, R=6, scale="nominal")
    X, ranks, _ = O.round_svd(Y, 0.0, 3)
    D = O.dense_tt_svd(O.full(Y), 3)
    assert ranks == O.ranks_of(D)
    np.testing.assert_allclose(O.full(X), O.full(D), rtol=0, atol=1e-12)


@pytest.mark.parametrize("eps0", [1e-1, 1e-3, 1e-8])
def test_round_svd_error_bound(eps0):
    # Algorithm 2 guarantees ||X - Y|| <= eps0 ||Y||; the tails add up
    X0, _, _ = G.perturbed_tt(5, 6, 5, 3, 1e-4)
    X, ranks, tails = O.round_svd(X0, eps0)
    err = O.rel_diff(X, X0)
    assert err <= eps0 * (1 + 1e-10)
    nrm = O.tt_norm(X0)
    assert (err * nrm) ** 2 == pytest.approx(sum(tails), rel=1e-6, abs=1e-30)


# ---------------------------------------------------------------- norms

def test_rel_diff_matches_dense():
    A = tiny_tt(61, N=4, I=3, R=3)
    B = tiny_tt(62, N=4, I=3, R=3)
    d = O.rel_diff(A, B)
    Fa, Fb = O.full(A), O.full(B)
    assert d == pytest.approx(np.linalg.norm(Fa - Fb) / np.linalg.norm(Fb), rel=1e-12)
    assert O.rel_diff(A, A) < 1e-14


# ---------------------------------------------------------------- paper behaviour

def test_perturbed_tt_behaviour():
    # section 4.1: with l above the rank of X1, the deterministic error is about
    # eps (relative); randomized errors are not smaller than deterministic/sqrt(N-1)
    N, I, R, eps = 6, 12, 4, 1e-6
    X, X1, X2 = G.perturbed_tt(123, N, I, R, eps)
    Xd, _, _ = O.round_svd(X, 0.0, 6)
    ed = O.rel_diff(Xd, X)
    scale = O.tt_norm(X2) / O.tt_norm(X)
    assert 0.05 * eps * scale < ed < 2 * eps * scale
    Xr = O.round_rand(X, 6, 0, seed=9)
    er = O.rel_diff(Xr, X)
    assert er >= ed / math.sqrt(N - 1)
    assert er < 1e3 * eps * scale


def test_hilbert_tt_similar_accuracy():
    # appendix C: deterministic and RtO reach very similar accuracy
    dims = [6, 8, 10, 12, 14, 16]
    ranks = [1, 4, 5, 6, 7, 8, 1]
    Y = G.hilbert_tt(dims, ranks)
    for r in [2, 3, 4]:
        Xd, _, _ = O.round_svd(Y, 0.0, r)
        Xr = O.round_rand(Y, r, 2, seed=3)
        ed, er = O.rel_diff(Xd, Y), O.rel_diff(Xr, Y)
        assert er >= ed / math.sqrt(5)
        assert er < 50 * ed + 1e-14


# ---------------------------------------------------------------- flop model

def test_flop_count_matches_table1_leading_order():
    # C_RtO = I (N-2) (4 R^2 l + 6 R l^2 + 4 l^3) at leading order (section 3.5)
    I, R, l = 100, 200, 60
    for N in [200, 2000]:
        dims, ranks = G.uniform_tt_shape(N, I, R)
        ell = [1] + [l] * (N - 1) + [1]
        f = O.rto_flops(dims, ranks, ell)
        model = I * (N - 2) * (4 * R * R * l + 6 * R * l * l + 4 * l ** 3)
        assert abs(f / model - 1) < 10.0 / N


# ---------------------------------------------------------------- conventions

def test_rto_qr_sign_convention():
    # reading of the QR normalisation: R = Q^T (Z_n W_n) has a non-negative diagonal
    Y = tiny_tt(71, N=5, I=4, R=5, scale="nominal")
    S, ell, _ = _sketch(12, Y, 3, 1)
    W = O.partial_contractions_rl(Y, S)
    X = O.rto_sweep(Y, W)
    # rebuild Z_n from the output: Z_1 = V(Y_1); Z_{n+1} = (Q_n^T Z_n) H(Y_{n+1})
    Z = O.V(Y[0])
    for n in range(1, 5):
        Q = O.V(X[n - 1])
        R = Q.T @ (Z @ W[n])
        assert np.all(np.diag(R) >= 0)
        assert np.abs(np.tril(R, -1)).max() < 1e-12 * np.abs(R).max()
        M = Q.T @ Z
        Z = (M @ O.H(Y[n])).reshape(-1, Y[n].shape[2])


def superdiagonal_tt(sigmas, N):
    """T = sum_k sigma_k e_k (x) ... (x) e_k: every unfolding has singular
    values exactly sigma (closed form)."""
    K = len(sigmas)
    cores = []
    for n in range(N):
        if n == 0:
            c = np.zeros((1, K, K))
            for k in range(K):
                c[0, k, k] = sigmas[k]
        elif n == N - 1:
            c = np.zeros((K, K, 1))
            for k in range(K):
                c[k, k, 0] = 1.0
        else:
            c = np.zeros((K, K, K))
            for k in range(K):
                c[k, k, k] = 1.0
        cores.append(c)
    return cores


def test_round_svd_eps_threshold_closed_form():
    # Algorithm 2 threshold: eps = ||Y|| eps0 / sqrt(N-1).  With singular values
    # (1,1,1,a) at every bond, N=5, eps0=1e-3: eps = 8.66e-4 < a = 1.2e-3, so
    # rank 4 is kept; a threshold without the sqrt(N-1) would cut to 3.
    a = 1.2e-3
    Y = superdiagonal_tt([1.0, 1.0, 1.0, a], 5)
    X, ranks, tails = O.round_svd(Y, 1e-3)
    assert ranks == [1, 4, 4, 4, 4, 1]
    X, ranks, tails = O.round_svd(Y, 2.0 * a * 2 / math.sqrt(3 + a * a))
    assert ranks == [1, 3, 3, 3, 3, 1]
    assert sum(tails) == pytest.approx(a * a, rel=1e-10)


def test_round_bf16_hand_values():
    # 8 significant bits: spacing 2^-7 on [1, 2); ties go to the even neighbour
    x = np.array([1.0, 1 + 2**-8, 1 + 3 * 2**-8, 1 + 2**-8 + 2**-20, -(1 + 2**-8 + 2**-20),
                  3.0, 0.0, 2**-130, 65504.0, 1 + 2**-7])
    want = np.array([1.0, 1.0, 1 + 2**-6, 1 + 2**-7, -(1 + 2**-7), 3.0, 0.0, 2**-130,
                     65536.0, 1 + 2**-7])
    np.testing.assert_array_equal(O.round_bf16(x), want)


def test_round_bf16_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-20, 20, 20000),
                        O.round_f32(rng.standard_normal(2000))])
    t = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(O.round_bf16(x), t)
    # two-step reading: the FP32 rounding comes first
    np.testing.assert_array_equal(O.round_bf16(x), O.round_bf16(O.round_f32(x)))


def test_rto_invariant_under_power_of_two_scaling_of_W():
    # the reduced-precision modes renormalise each W_n by a power of two; the
    # RtO output must not depend on it (Q of Z_n W_n is scale invariant)
    X = G.random_tt(77, [5, 6, 4, 5, 3], [1, 4, 6, 5, 3, 1])
    sk = O.make_sketch(78, O.dims_of(X), [1, 3, 4, 4, 3, 1])
    W = O.partial_contractions_rl(X, sk)
    Ws = [None] + [w * 2.0 ** (-17 * n) for n, w in enumerate(W) if n > 0]
    A = O.rto_sweep(X, W)
    B = O.rto_sweep(X, Ws)
    for a, b in zip(A, B):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-13)


# ---------------------------------------------------------------- adjoint oracle

def _adjoint_case(seed, N=5, I=4, R=5, ell=3):
    dims, ranks = G.uniform_tt_shape(N, I, R)
    Y = G.random_tt(seed, dims, ranks, scale="nominal")
    ellv, _ = O.plan_ranks(dims, ranks, ell, 0)
    S = O.make_sketch(seed + 1, dims, ellv)
    return Y, S, ell


def test_adjoint_oracle_forward_matches_numpy_oracle():
    torch = pytest.importorskip("torch")
    from oracle.tt_adjoint import rto_torch
    for seed in (3, 4):
        Y, S, ell = _adjoint_case(seed)
        ref = O.round_rand(Y, ell, 0, sketch=S, truncate=False)
        out = rto_torch([torch.tensor(c) for c in Y], [torch.tensor(c) for c in S])
        for a, b in zip(out, ref):
            np.testing.assert_allclose(a.numpy(), b, rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed", [5, 6])
def test_adjoint_oracle_matches_central_differences(seed):
    # directional derivative of sum_n <G_n, out_n(Y)> from the numpy forward
    pytest.importorskip("torch")
    from oracle.tt_adjoint import rto_vjp
    Y, S, ell = _adjoint_case(seed, N=4, I=5, R=6, ell=3)
    rng = np.random.default_rng(seed + 10)
    ref = O.round_rand(Y, ell, 0, sketch=S, truncate=False)
    Gc = [rng.standard_normal(c.shape) for c in ref]
    D = [rng.standard_normal(c.shape) for c in Y]

    def f(t):
        out = O.round_rand([y + t * d for y, d in zip(Y, D)], ell, 0, sketch=S, truncate=False)
        return sum(float(np.sum(g * o)) for g, o in zip(Gc, out))

    h = 1e-6
    fd = (f(h) - f(-h)) / (2 * h)
    grads = rto_vjp(Y, S, Gc)
    an = sum(float(np.sum(g * d)) for g, d in zip(grads, D))
    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_tt_inner_torch_matches_full_tensor():
    torch = pytest.importorskip("torch")
    from oracle.tt_adjoint import loss_round_minus_target, tt_inner_torch
    A = tiny_tt(7)
    B = tiny_tt(8)
    ip = float(tt_inner_torch([torch.tensor(c) for c in A], [torch.tensor(c) for c in B]))
    assert abs(ip - float(np.sum(O.full(A) * O.full(B)))) <= 1e-12 * max(1.0, abs(ip))
    ls = float(loss_round_minus_target([torch.tensor(c) for c in A], [torch.tensor(c) for c in B]))
    assert abs(ls - float(np.sum((O.full(A) - O.full(B)) ** 2))) <= 1e-10 * max(1.0, ls)


# ---------------------------------------------------------------- Algorithm 6

def _left_interface(cores):
    """V(X_{1:n}) of the first n cores by successive dense products,
    (I_1 ... I_n) x r_n."""
    M = cores[0].reshape(-1, cores[0].shape[2])
    for c in cores[1:]:
        M = (M @ c.reshape(c.shape[0], -1)).reshape(-1, c.shape[2])
    return M


@pytest.mark.parametrize("seed", RNG_SEEDS)
def test_partial_contractions_lr_brute_force(seed):
    # closed form W^L_n = Psi_n V(Y_{1:n}) with Psi_n = V(L_{1:n})^T
    X = tiny_tt(seed, N=5, I=3, R=4)
    L = G.random_tt(seed + 70, [3] * 5, [1, 2, 3, 3, 2, 1], scale="unit")
    W = O.partial_contractions_lr(X, L)
    for n in range(1, 5):
        want = _left_interface(L[:n]).T @ _left_interface(X[:n])
        np.testing.assert_allclose(W[n], want, rtol=1e-12, atol=1e-12)


def test_partial_contractions_lr_norm():
    # with both tensors equal, W_{N-1} contracted with the last cores is ||X||^2
    X = tiny_tt(4, N=6, I=3, R=3)
    W = O.partial_contractions_lr(X, X)
    last = O.H(X[-1])
    val = float(np.sum(W[5] * (last @ last.T)))
    assert val == pytest.approx(float(np.sum(O.full(X) ** 2)), rel=1e-12)


def test_plan_two_sided_ranks():
    ell, rho = O.plan_two_sided_ranks([10] * 8, [1] + [20] * 7 + [1], 10)
    assert ell == [1] + [10] * 7 + [1]
    assert rho == [1] + [15] * 6 + [10, 1]  # rho_7 capped by I_8 = 10
    ell, rho = O.plan_two_sided_ranks([100] * 4, [1, 200, 200, 200, 1], 60)
    assert ell == [1, 60, 60, 60, 1] and rho == [1, 90, 90, 90, 1]


@pytest.mark.parametrize("seed", RNG_SEEDS)
def test_two_sided_order_two_is_matrix_nystrom(seed):
    # N = 2: Algorithm 6 is the generalized Nystrom approximation of section 2.2,
    # Y Omega (Psi Y Omega)^+ Psi Y, with Psi = V(L_1)^T and Omega = H(R_2)^T
    dims, ranks = [9, 11], [1, 7, 1]
    Y = G.random_tt(seed, dims, ranks, scale="unit")
    ell, rho = O.plan_two_sided_ranks(dims, ranks, 4)
    Ls = O.make_sketch(10 + seed, dims, ell)
    Rs = O.make_sketch(20 + seed, dims, rho)
    X = O.round_two_sided(Y, 4, sketch_left=Ls, sketch_right=Rs)
    A = O.full(Y).reshape(9, 11)
    Psi = Ls[0].reshape(9, ell[1]).T
    Omega = Rs[1].reshape(rho[1], 11).T
    want = A @ Omega @ np.linalg.pinv(Psi @ A @ Omega, rcond=O.NYSTROM_RCOND) @ Psi @ A
    np.testing.assert_allclose(O.full(X).reshape(9, 11), want, rtol=0,
                               atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("seed", RNG_SEEDS)
def test_two_sided_equals_dense_bond_projectors(seed):
    # section 3.3: X is Y with the bond projector W^R_n (W^L_n W^R_n)^+ W^L_n
    # inserted at every bond; W^L_n, W^R_n formed densely from the sketches
    dims, ranks = [3, 4, 3, 4], [1, 4, 5, 4, 1]
    Y = G.random_tt(30 + seed, dims, ranks, scale="unit")
    ell, rho = O.plan_two_sided_ranks(dims, ranks, 2)
    Ls = O.make_sketch(40 + seed, dims, ell)
    Rs = O.make_sketch(50 + seed, dims, rho)
    X = O.round_two_sided(Y, 2, sketch_left=Ls, sketch_right=Rs)
    proj = []
    for n in range(1, 4):
        WL = _left_interface(Ls[:n]).T @ _left_interface(Y[:n])
        WR = O.full_with_left_rank(Y[n:]) @ O.full_with_left_rank(Rs[n:]).T
        proj.append(WR @ np.linalg.pinv(WL @ WR, rcond=O.NYSTROM_RCOND) @ WL)
    cores = [np.einsum("aib,bc->aic", Y[n], proj[n]) for n in range(3)] + [Y[3]]
    want = O.full(cores)
    np.testing.assert_allclose(O.full(X), want, rtol=0, atol=1e-12 * np.abs(want).max())
    assert O.ranks_of(X) == ell


def test_two_sided_exact_on_small_sum_workload():
    # generalized Nystrom is exact when every unfolding rank is at most l_n:
    # A + A (rank 10, formally 20) -> 2A, also with l_n above the rank
    w = G.workload_small_sum()
    twoA = [2.0 * w["A"][0]] + [c.copy() for c in w["A"][1:]]
    for target, tol in [(10, 1e-11), (12, 1e-9)]:
        X = O.round_two_sided(w["X"], target, seed_left=3, seed_right=4)
        assert O.rel_diff(X, twoA) <= tol, target
        assert O.ranks_of(X)[3] == target


def test_two_sided_error_lower_bound():
    # Eckart-Young at every bond: ||Y - X|| >= sqrt(sum_{k > l_n} s_k^2) of the
    # n-th unfolding, since X has rank l_n there
    Y = tiny_tt(8, N=5, I=3, R=5, scale="nominal")
    X = O.round_two_sided(Y, 2, seed_left=1, seed_right=2)
    T = O.full(Y)
    err = O.rel_diff(X, Y) * O.tt_norm(Y)
    for n in range(1, 5):
        s = np.linalg.svd(T.reshape(3 ** n, -1), compute_uv=False)
        assert err >= math.sqrt(float(np.sum(s[2:] ** 2))) * (1 - 1e-12)


# ---------------------------------------------------------------- tolerance-driven ranks

def test_truncate_rl_eps_threshold_closed_form():
    # singular values (1, 1, 1, a) at every bond of a left-orthogonal TT: the
    # threshold eps = ||X|| eps0 / sqrt(N-1) keeps a exactly when eps < a
    # (the closed form of the Algorithm 2 pin, from the right)
    a = 1.2e-3
    Y = superdiagonal_tt([1.0, 1.0, 1.0, a], 5)
    X = O.rto_sweep(Y, O.partial_contractions_rl(Y, Y))  # left-orthogonal, exact
    assert O.rel_diff(X, Y) < 1e-13
    Z, ranks, tails = O.truncate_rl_eps(X, 1e-3)
    assert ranks == [1, 4, 4, 4, 4, 1]
    Z, ranks, tails = O.truncate_rl_eps(X, 2.0 * a * 2 / math.sqrt(3 + a * a))
    assert ranks == [1, 3, 3, 3, 3, 1]
    assert sum(tails) == pytest.approx(a * a, rel=1e-10)
    assert O.rel_diff(Z, X) == pytest.approx(a / math.sqrt(3 + a * a), rel=1e-8)


@pytest.mark.parametrize("eps0", [1e-2, 1e-5])
def test_round_rand_eps_bound_and_dense_tt_svd(eps0):
    # X1 (rank 3) + 1e-6 X2 (rank 4), sketch rank 9 > 7: RtO is exact to
    # rounding, the tolerance truncation meets ||X - Xr|| <= eps0 ||Xr|| and
    # keeps the same ranks as the deterministic TT-SVD with the same eps0
    Y = G.near_low_rank_tt(7, [5] * 6, 3, 4, 1e-6)
    Xr = O.round_rand(Y, 9, 0, seed=1, truncate=False)
    assert O.rel_diff(Xr, Y) < 1e-12
    X, ranks, tails = O.round_rand_eps(Y, 9, eps0, seed=1)
    assert O.rel_diff(X, Xr) <= eps0 * (1 + 1e-12)
    assert math.sqrt(sum(tails)) == pytest.approx(O.rel_diff(X, Xr) * O.tt_norm(Xr), rel=1e-6)
    D, dranks, _ = O.round_svd(Y, eps0)
    assert ranks == dranks
    assert ranks == [1] + [3] * 5 + [1]
    assert O.rel_diff(X, D) < 1e-5
    # right-orthogonal cores 2..N
    for c in X[1:]:
        Hn = O.H(c)
        assert np.abs(Hn @ Hn.T - np.eye(Hn.shape[0])).max() < 1e-12


def test_round_rand_eps_zero_keeps_everything():
    Y = tiny_tt(3, N=4, I=3, R=3)
    X, ranks, tails = O.round_rand_eps(Y, 9, 0.0, seed=2)
    Xr = O.round_rand(Y, 9, 0, seed=2, truncate=False)
    assert ranks == O.ranks_of(Xr)
    assert O.rel_diff(X, Xr) < 1e-13


def test_round_sum_rand_eps_equals_assembled():
    A = G.random_tt(11, [4] * 5, [1, 2, 2, 2, 2, 1])
    B = G.random_tt(12, [4] * 5, [1, 2, 2, 2, 2, 1])
    S = G.block_sum([A, B, A], [1.0, 0.5, -2.0])
    X, ranks, _ = O.round_sum_rand_eps([A, B, A], [1.0, 0.5, -2.0], 8, 1e-10, seed=3)
    Z, zr, _ = O.round_rand_eps(S, 8, 1e-10, seed=3)
    assert ranks == zr == [1, 4, 4, 4, 4, 1]
    assert O.rel_diff(X, S) < 1e-12


# ---------------------------------------------------------------- Algorithm 4

def test_orthogonalize_rl_wide_panel_gauge():
    # I_N r_N < r_{N-1}: the last bond drops to I_N and the result is still
    # right-orthogonal and equal to the input
    Y = G.random_tt(5, [3, 4, 2], [1, 3, 5, 1])
    X = O.orthogonalize_rl(Y)
    assert O.ranks_of(X) == [1, 3, 2, 1]
    assert O.rel_diff(X, Y) < 1e-13
    for c in X[1:]:
        Hn = O.H(c)
        assert np.abs(Hn @ Hn.T - np.eye(Hn.shape[0])).max() < 1e-14


@pytest.mark.parametrize("seed", RNG_SEEDS)
def test_orth_rand_equals_rto_with_partial_contractions_as_omega(seed):
    # Omega_n = W_n = H(X_{n+1:N}) H(Rk_{n+1:N})^T of the right-orthogonalised
    # X turns Algorithm 4's sweep into Algorithm 5's on X, and Algorithm 5 is
    # invariant under the gauge change of Algorithm 1: the outputs agree core
    # by core
    Y = tiny_tt(seed, N=5, I=3, R=4)
    X = O.orthogonalize_rl(Y)
    dims, ranks = O.dims_of(X), O.ranks_of(X)
    ell, _ = O.plan_ranks(dims, ranks, 3, 0)
    Rk = O.make_sketch(seed + 9, dims, ell)
    W = O.partial_contractions_rl(X, Rk)
    a = O.round_orth_rand(Y, 3, 0, omegas=W)
    b = O.round_rand(Y, 3, 0, sketch=Rk)
    for x, y in zip(a, b):
        np.testing.assert_allclose(x, y, atol=1e-12)


@pytest.mark.parametrize("seed", RNG_SEEDS)
def test_orth_rand_equals_dense_range_finder(seed):
    # on the right-orthogonal X, V(X_n) Omega_n = T_n H(X_{n+1:N})^T Omega_n
    # with T_n the n-th sequential unfolding: the dense sequential range
    # finder with the sketch H(X_{n+1:N})^T Omega_n gives the same cores
    Y = tiny_tt(seed, N=4, I=3, R=3)
    X = O.orthogonalize_rl(Y)
    N = len(X)
    dims, ranks = O.dims_of(X), O.ranks_of(X)
    ell, _ = O.plan_ranks(dims, ranks, 2, 1)
    om = [None] + [O.gaussian_matrix(seed, n, ranks[n], ell[n]) for n in range(1, N)]
    out = O.round_orth_rand(Y, 2, 1, omegas=om, truncate=False)
    T = O.full(Y).reshape(dims[0], -1)
    for n in range(1, N):
        right = O.full_with_left_rank(X[n:])  # (R_n, I_{n+1} ... I_N)
        Q, _ = O.qr_pos(T @ right.T @ om[n])
        np.testing.assert_allclose(Q, O.V(out[n - 1]), atol=1e-11)
        T = (Q.T @ T).reshape(ell[n] * dims[n], -1)


def test_orth_rand_exact_on_small_sum_workload():
    w = G.workload_small_sum()
    twoA = [2.0 * w["A"][0]] + [c.copy() for c in w["A"][1:]]
    out = O.round_orth_rand(w["X"], w["target"], w["oversample"], seed=w["sketch_seed"])
    assert O.rel_diff(out, twoA) <= 1e-12
    for c in out[1:]:
        Hn = O.H(c)
        assert np.abs(Hn @ Hn.T - np.eye(Hn.shape[0])).max() < 1e-12


def test_gaussian_matrix_distribution():
    M = O.gaussian_matrix(7, 3, 300, 200)
    assert M.shape == (300, 200)
    assert abs(M.mean()) < 3e-4
    assert abs(M.var() * 300 * 200 - 1.0) < 2e-2
    np.testing.assert_array_equal(M, O.make_sketch(10, [60000], [1, 1])[0].reshape(300, 200))


# ---------------------------------------------------------------- TT-GMRES (section 4.2)

def _dense_gmres_residuals(A, P, f, m):
    # right-preconditioned GMRES on the dense system, modified Gram-Schmidt
    n = f.size
    beta = np.linalg.norm(f)
    Vd = np.zeros((n, m + 1))
    Hd = np.zeros((m + 1, m))
    Vd[:, 0] = f / beta
    res = [1.0]
    for k in range(m):
        w = A @ (P @ Vd[:, k])
        for j in range(k + 1):
            Hd[j, k] = Vd[:, j] @ w
            w = w - Hd[j, k] * Vd[:, j]
        Hd[k + 1, k] = np.linalg.norm(w)
        Vd[:, k + 1] = w / Hd[k + 1, k]
        e1 = np.zeros(k + 2)
        e1[0] = beta
        y, *_ = np.linalg.lstsq(Hd[:k + 2, :k + 1], e1, rcond=None)
        res.append(np.linalg.norm(e1 - Hd[:k + 2, :k + 1] @ y) / beta)
    return res


def test_tt_gmres_matches_dense_gmres_when_rounding_is_exact():
    # tiny problem, rounding tolerance at the rounding level and sketch rank
    # above every rank that appears: the TT iteration is GMRES itself
    op = G.parametric_operator(N=3, I_space=6, I_param=4)
    dims = op["dims"]
    A = O.kron_operator_dense(op["mats"], dims)
    P = np.kron(op["precond"], np.eye(int(np.prod(dims[1:]))))
    f = O.full(op["f"]).ravel()
    x, res, m = O.tt_gmres(op["mats"], op["f"], op["precond"], 24, 1e-14, 1e-10, 40, seed=5)
    dres = _dense_gmres_residuals(A, P, f, m)
    np.testing.assert_allclose(res, dres, rtol=1e-6, atol=1e-12)
    assert res[-1] <= 1e-10
    xd = O.full(x).ravel()
    assert np.linalg.norm(A @ xd - f) / np.linalg.norm(f) <= 1e-9


def test_tt_gmres_true_residual_meets_tolerance():
    # rounding tolerance well below the solver tolerance: the true residual
    # of the returned TT follows the estimate
    op = G.parametric_operator(N=4, I_space=10, I_param=5)
    dims = op["dims"]
    A = O.kron_operator_dense(op["mats"], dims)
    f = O.full(op["f"]).ravel()
    x, res, m = O.tt_gmres(op["mats"], op["f"], op["precond"], 30, 1e-10, 1e-7, 30, seed=9)
    assert res[-1] <= 1e-7
    xd = O.full(x).ravel()
    assert np.linalg.norm(A @ xd - f) / np.linalg.norm(f) <= 1e-6
