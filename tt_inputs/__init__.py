"""Seeded synthetic TT inputs shared by the oracle, the tests and the benchmark.

This module only *draws and lays out* inputs; it holds none of the rounding
arithmetic.  Everything here is numpy on the host, deterministic in the seed.

Core layout everywhere: a TT of order N is a list of N float64 arrays, core n
having shape (r_{n-1}, I_n, r_n) in C order with r_0 = r_N = 1 (the TT format
of the paper's section 2.1).

Workload recipes (the synthetic stand-ins for the paper's experiments):

* ``random_tt(seed, dims, ranks, scale="nominal")`` -- every core iid
  N(0,1) / sqrt(I_n * r_nom), with r_nom the largest interior rank.
* ``random_tt(..., scale="def31")`` -- core n iid N(0, 1/(r_{n-1} I_n r_n)),
  the normalisation of Definition 3.1 (used by the perturbed-TT experiment of
  section 4.1).
* ``block_sum(tts, coeffs)`` -- the formal sum of TTs as block-diagonal cores
  (section 2.1), summand j scaled by coeffs[j] on its first core.
* ``hilbert_tt(dims, ranks)`` -- the Hilbert-type TT of appendix C.
"""
from __future__ import annotations

import numpy as np

INPUT_SEED_BASE = 1000
SKETCH_SEED_BASE = 2000
BATCH_SEED_BASE = 100000


def _check_shape(dims, ranks):
    N = len(dims)
    if len(ranks) != N + 1 or ranks[0] != 1 or ranks[-1] != 1:
        raise ValueError("ranks must have length N+1 with r_0 = r_N = 1")
    if any(int(d) < 1 for d in dims) or any(int(r) < 1 for r in ranks):
        raise ValueError("dims and ranks must be positive")


def random_tt(seed, dims, ranks, scale="nominal", dtype=np.float64):
    """Random Gaussian TT with C-ordered cores (r_{n-1}, I_n, r_n)."""
    dims = [int(d) for d in dims]
    ranks = [int(r) for r in ranks]
    _check_shape(dims, ranks)
    rng = np.random.default_rng(seed)
    r_nom = max(ranks[1:-1]) if len(ranks) > 2 else 1
    cores = []
    for n, I in enumerate(dims):
        shape = (ranks[n], I, ranks[n + 1])
        g = rng.standard_normal(shape)
        if scale == "nominal":
            g *= 1.0 / np.sqrt(I * r_nom)
        elif scale == "def31":
            g *= 1.0 / np.sqrt(ranks[n] * I * ranks[n + 1])
        elif scale == "unit":
            pass
        else:
            raise ValueError(scale)
        cores.append(np.ascontiguousarray(g, dtype=dtype))
    return cores


def block_sum(tts, coeffs=None):
    """Assemble the formal sum sum_j coeffs[j] * tts[j] as one TT.

    Section 2.1: interior cores are block diagonal in their two rank indices,
    the first core concatenates along its right rank, the last along its left
    rank.  The coefficient multiplies summand j's first core.
    """
    s = len(tts)
    if coeffs is None:
        coeffs = [1.0] * s
    N = len(tts[0])
    dims = [c.shape[1] for c in tts[0]]
    for t in tts:
        if [c.shape[1] for c in t] != dims:
            raise ValueError("summands must share mode sizes")
    if N == 1:
        return [sum(float(c) * t[0] for c, t in zip(coeffs, tts))]
    out = []
    for n in range(N):
        left = [t[n].shape[0] for t in tts]
        right = [t[n].shape[2] for t in tts]
        if n == 0:
            out.append(np.concatenate([coeffs[j] * tts[j][0] for j in range(s)], axis=2))
        elif n == N - 1:
            out.append(np.concatenate([tts[j][n] for j in range(s)], axis=0))
        else:
            core = np.zeros((sum(left), dims[n], sum(right)), dtype=tts[0][n].dtype)
            a = b = 0
            for j in range(s):
                core[a:a + left[j], :, b:b + right[j]] = tts[j][n]
                a += left[j]
                b += right[j]
            out.append(core)
    return [np.ascontiguousarray(c) for c in out]


def hilbert_tt(dims, ranks):
    """Hilbert-type TT (appendix C): core entries 1/(i1+i2+i3-1), 1-based."""
    dims = [int(d) for d in dims]
    ranks = [int(r) for r in ranks]
    _check_shape(dims, ranks)
    cores = []
    for n, I in enumerate(dims):
        a = np.arange(1, ranks[n] + 1)[:, None, None]
        i = np.arange(1, I + 1)[None, :, None]
        b = np.arange(1, ranks[n + 1] + 1)[None, None, :]
        cores.append(np.ascontiguousarray(1.0 / (a + i + b - 1), dtype=np.float64))
    return cores


def sum_coefficients(seed, s):
    """Summand coefficients c_j ~ U(-1, 1) (the GMRES-like sum workload)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=s)


def uniform_tt_shape(N, I, R):
    return [I] * N, [1] + [R] * (N - 1) + [1]


# ----------------------------------------------------------------------------
# The five workloads (sizes of the paper-derived configurations).
# ----------------------------------------------------------------------------

def workload_small_sum(k=0):
    """A: N=8, I=10, rank 10, cores N(0,1)/sqrt(10*10); X = A + A assembled
    (formal rank 20); round to rank 10 with a sketch of rank 10+5.
    The exact answer is 2A."""
    dims, ranks = uniform_tt_shape(8, 10, 10)
    A = random_tt(INPUT_SEED_BASE + k, dims, ranks, scale="nominal")
    X = block_sum([A, A])
    return dict(A=A, X=X, summands=[A, A], target=10, oversample=5,
                sketch_seed=SKETCH_SEED_BASE + k)


def workload_single_tt(k=1, N=30, I=100, R=200, target=50, oversample=10):
    """Single TT, N=30, I=100, rank 200, cores N(0,1)/sqrt(I*R); target rank
    50 through a sketch of rank 60."""
    dims, ranks = uniform_tt_shape(N, I, R)
    X = random_tt(INPUT_SEED_BASE + k, dims, ranks, scale="nominal")
    return dict(X=X, target=target, oversample=oversample,
                sketch_seed=SKETCH_SEED_BASE + k)


def workload_gmres_sum(k=2, s=20, N=16, I=128, R=20, target=60, oversample=10):
    """Sum of s=20 TTs, N=16, I=128, each rank 20, coefficients U(-1,1),
    formal rank 400; target 60 via a sketch of rank 70."""
    dims, ranks = uniform_tt_shape(N, I, R)
    summands = [random_tt(INPUT_SEED_BASE + 100 * k + j, dims, ranks, scale="nominal")
                for j in range(s)]
    coeffs = sum_coefficients(INPUT_SEED_BASE + 100 * k + 99, s)
    return dict(summands=summands, coeffs=coeffs, target=target,
                oversample=oversample, sketch_seed=SKETCH_SEED_BASE + k)


def perturbed_tt(seed, N, I, R, eps):
    """X = X1 + eps * X2 with X1, X2 random rank-R TTs normalised as in
    Definition 3.1 (the construction of section 4.1); formal rank 2R."""
    dims, ranks = uniform_tt_shape(N, I, R)
    X1 = random_tt(seed, dims, ranks, scale="def31")
    X2 = random_tt(seed + 1, dims, ranks, scale="def31")
    return block_sum([X1, X2], [1.0, eps]), X1, X2


def near_low_rank_tt(seed, dims, r_low, r_high, eps):
    """X = X1 + eps * X2: X1 a random TT of uniform rank r_low, X2 of rank
    r_high (cores N(0,1)/sqrt(I r), so that both have norm about 1/sqrt(r)),
    as one TT of formal rank r_low + r_high.  Rounding to a target >= r_low
    is then exact up to O(eps)."""
    N = len(dims)
    X1 = random_tt(seed, dims, [1] + [r_low] * (N - 1) + [1], scale="nominal")
    X2 = random_tt(seed + 1, dims, [1] + [r_high] * (N - 1) + [1], scale="nominal")
    return block_sum([X1, X2], [1.0, eps])


def batched_specs(seed=0, B=64):
    """Shapes of the ragged batch: per item N ~ U{8..24}, one I in
    {16,32,64,128,256}, rank R ~ U{8..128}, target R//2, oversample
    min(10, R - target)."""
    rng = np.random.default_rng(BATCH_SEED_BASE + seed)
    specs = []
    for b in range(B):
        N = int(rng.integers(8, 25))
        I = int(rng.choice([16, 32, 64, 128, 256]))
        R = int(rng.integers(8, 129))
        t = R // 2
        specs.append(dict(N=N, I=I, R=R, target=t, oversample=min(10, R - t),
                          input_seed=BATCH_SEED_BASE + b,
                          sketch_seed=SKETCH_SEED_BASE + 10000 + b))
    return specs


def parametric_operator(N=5, I_space=64, I_param=16, reaction=10.0):
    """A synthetic stand-in for the parametric diffusion system of section 4.2
    (its cookie-problem data are not available): the operator
    sum_{i=1}^{N} A_{i,1} x ... x A_{i,N} on I_space x I_param^(N-1) with
    A_{1,1} = K (the 1D finite-difference Laplacian on I_space interior
    points of (0, 1)), chi_i the indicator of the i-th of N-1 equal
    subintervals, A_{i,i} = diag(rho) with the
    parameter values rho linearly spaced in [1, 10], and identities
    elsewhere (None); A_{i,1} = reaction diag(chi_i) for i >= 2 (a reaction
    term on the i-th subinterval, weighted by the i-th parameter).  The right-hand
    side f is the rank-1 TT of all ones, and
    the right preconditioner is (sum_i A_{i,1})^{-1} on the first mode (the
    mean-based preconditioner of the section).  Returns dict(mats, f,
    precond, dims) with mats[i][n] a float64 matrix or None."""
    h = 1.0 / (I_space + 1)
    K = (np.diag(np.full(I_space, 2.0)) - np.diag(np.ones(I_space - 1), 1)
         - np.diag(np.ones(I_space - 1), -1)) / (h * h)
    dims = [I_space] + [I_param] * (N - 1)
    rho = np.linspace(1.0, 10.0, I_param)
    mats = [[None] * N for _ in range(N)]
    mats[0][0] = K
    edges = np.linspace(0, I_space, N).astype(int)
    for i in range(1, N):
        chi = np.zeros(I_space)
        chi[edges[i - 1]:edges[i]] = 1.0
        mats[i][0] = reaction * np.diag(chi)
        mats[i][i] = np.diag(rho)
    S = sum(mats[i][0] for i in range(N))
    precond = np.linalg.inv(S)
    f = [np.ones((1, d, 1)) for d in dims]
    return dict(mats=mats, f=f, precond=precond, dims=dims)


def workload_gmres(k=3):
    """The TT-GMRES workload: the parametric operator with N=5, 64 spatial
    points, 16 samples per parameter; sketch rank 60, rounding tolerance
    1e-9, solver tolerance 1e-8 (the section's), at most 40 iterations."""
    op = parametric_operator(N=5, I_space=64, I_param=16)
    return dict(op=op, max_rank=60, round_eps=1e-9, tol=1e-8, max_iter=40,
                seed=SKETCH_SEED_BASE + k)
