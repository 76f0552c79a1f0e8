"""GPU parity of Two-Sided-Randomization (Algorithm 6) through the C ABI with
the FP64 oracle on the same seeded inputs and the same sketches (both sides
draw them from the seeds with the counter-based generator).  The output is
not orthogonal and its gauge depends on the signs of singular vectors, so the
comparison is of the represented tensors: ||X_gpu - X_oracle|| / ||X_oracle||
by the oracle's orthogonalised difference."""
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


@pytest.mark.parametrize("case", [
    (3, 4, 5, 2),       # tiny
    (5, 7, 9, 4),       # ragged
    (6, 9, 12, 5),
    (4, 30, 40, 16),    # several GEMM tiles
    (3, 100, 200, 60),  # interior cores of the workload size (rho = 90)
    (5, 3, 20, 64),     # l and rho capped by the mode products at both ends
    (2, 11, 7, 4),      # N = 2: the matrix generalized Nystrom
])
def test_two_sided_matches_oracle(gpu_lib, case):
    N, I, R, t = case
    say(f"two-sided {case}")
    dims, ranks = G.uniform_tt_shape(N, I, R)
    Y = G.random_tt(90 + N, dims, ranks, scale="nominal")
    out = host(gpu_lib.round_two_sided(dev(Y), t, seed_left=5, seed_right=6))
    ref = O.round_two_sided(Y, t, seed_left=5, seed_right=6)
    assert O.ranks_of(out) == O.ranks_of(ref)
    assert O.rel_diff(out, ref) < 1e-10


def test_two_sided_exact_on_small_sum_workload(gpu_lib):
    # A + A (rank 10, formally 20): generalized Nystrom returns 2A, also with
    # l_n above the rank (the extra singular values fall under the cutoff)
    say("two-sided A + A")
    w = G.workload_small_sum()
    twoA = [2.0 * w["A"][0]] + [c.copy() for c in w["A"][1:]]
    for target, tol in [(10, 1e-11), (12, 1e-9)]:
        out = host(gpu_lib.round_two_sided(dev(w["X"]), target, seed_left=3, seed_right=4))
        assert O.rel_diff(out, twoA) <= tol, target


def test_two_sided_order_one_and_deterministic(gpu_lib):
    say("two-sided N=1, determinism")
    Y1 = [np.random.default_rng(0).standard_normal((1, 7, 1))]
    out = host(gpu_lib.round_two_sided(dev(Y1), 3))
    np.testing.assert_array_equal(out[0], Y1[0])
    dims, ranks = G.uniform_tt_shape(6, 20, 30)
    Y = dev(G.random_tt(7, dims, ranks, scale="nominal"))
    a = host(gpu_lib.round_two_sided(Y, 10, 1, 2))
    b = host(gpu_lib.round_two_sided(Y, 10, 1, 2))
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_two_sided_rejects_float32(gpu_lib):
    say("two-sided float32")
    dims, ranks = G.uniform_tt_shape(3, 5, 4)
    Y = [c.float() for c in dev(G.random_tt(1, dims, ranks, scale="unit"))]
    with pytest.raises((gpu_lib.TTError, ValueError)):
        gpu_lib.round_two_sided(Y, 2)


@pytest.mark.parametrize("eps", [1e-3, 1e-6])
@pytest.mark.parametrize("case", [
    (5, 40, 8, 40, 8),    # l equal to the strong rank
    (5, 40, 8, 40, 12),   # l above it: W^L W^R has small singular values
    (4, 30, 10, 30, 10),
])
def test_two_sided_near_low_rank_matches_oracle(gpu_lib, case, eps):
    # X1 + eps X2 (the kind of input of the paper's first experiment): the
    # products W^L_n W^R_n span several orders of magnitude, which the two
    # Jacobi passes resolve
    N, I, rl, rh, t = case
    say(f"two-sided near-low-rank {case} eps={eps}")
    Y = G.near_low_rank_tt(321, [I] * N, rl, rh, eps)
    out = host(gpu_lib.round_two_sided(dev(Y), t, seed_left=5, seed_right=6))
    ref = O.round_two_sided(Y, t, seed_left=5, seed_right=6)
    assert O.ranks_of(out) == O.ranks_of(ref)
    assert O.rel_diff(out, ref) < 1e-10
