"""FP64 CPU oracle for randomized TT-rounding.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call this module.  The GPU
product path never touches it and shares no code with it.

Everything is plain numpy in float64; QR and SVD are LAPACK via numpy.linalg.
Functions follow the paper (Al Daas et al., "Randomized algorithms for
rounding in the Tensor-Train format") step by step in its notation:

* TT format, unfoldings H/V, sums of TTs ............ section 2.1 / 2.3
* OrthogonalizeRL ................................... Algorithm 1
* Orthogonalize-then-Randomize ...................... Algorithm 4
* deterministic TT-Rounding ......................... Algorithm 2
* PartialContractionsRL (the W_n chain) ............. Algorithm 3, eq. (RLContraction)
* random Gaussian TT sketch ......................... Definition 3.1
* Randomize-then-Orthogonalize ...................... Algorithm 5
* Two-Sided-Randomization (generalized Nystrom) ..... Algorithm 6, eq. (LnRn)
* rounding a sum, Randomize-then-Orthogonalize ...... Algorithm 7
* truncation of the left-orthogonal RtO output ...... section 3.2 (remark after
  Algorithm 5), run as the right-to-left mirror of Algorithm 2; to fixed ranks
  or to a tolerance (ranks not known in advance)

Readings taken where the paper is silent (each also listed in the design notes):

* Cores are C-ordered (r_{n-1}, I_n, r_n); V() and H() are C reshapes.  This is
  a row permutation of the paper's MATLAB-ordered V(); it changes neither R
  factors, orthonormality nor the represented tensor.
* Thin QR is normalised to diag(R) >= 0 (zero counts as +), which makes the
  RtO output unique when every sketch Y_n has full column rank.
* Sketch ranks: u_N = 1, u_n = min(l, I_{n+1} u_{n+1}); l_0 = 1,
  l_n = min(l, l_{n-1} I_n, u_n, R_n) with l = target + oversample;
  output ranks r_n = min(target, l_n).
* The sketch generator (the paper fixes only the distribution): SplitMix64
  (Steele, Lea, Flood 2014) evaluated at a counter, Box-Muller transform.
* When r_n < l_n somewhere, the left-orthogonal RtO output is truncated by a
  right-to-left sweep of SVDs (the mirror of the truncation loop of Algorithm 2, since the
  output is left- and not right-orthogonal).
* eps-truncation is absolute: keep the smallest k >= 1 with
  sqrt(sum_{j>k} s_j^2) <= eps0 ||Y|| / sqrt(N-1), capped by max_rank.
* Sum coefficients multiply each summand's first core.
* Two-Sided-Randomization: l_n as above with no oversampling, right sketch
  ranks rho_n = ceil(3 l_n / 2) capped by I_{n+1} ... I_N; the pseudo-inverse
  of W^L_n W^R_n drops singular values at or below 1e-6 of the largest.
* Reduced-precision modes are compared with this FP64 oracle run on the same
  inputs and on the same sketch values: the FP32 sketch is the FP64 draw
  rounded to nearest-even FP32, the BF16 sketch is that FP32 value rounded
  to nearest-even bfloat16 (round_f32, round_bf16).
"""
from __future__ import annotations

import math

import numpy as np

# ----------------------------------------------------------------------------
# TT basics (section 2.1)
# ----------------------------------------------------------------------------


def ranks_of(cores):
    return [1] + [int(c.shape[2]) for c in cores]


def dims_of(cores):
    return [int(c.shape[1]) for c in cores]


def H(core):
    """Horizontal unfolding: r_{n-1} x (I_n r_n)."""
    return core.reshape(core.shape[0], -1)


def V(core):
    """Vertical unfolding: (r_{n-1} I_n) x r_n."""
    return core.reshape(-1, core.shape[2])


def full(cores):
    """Dense tensor of a TT: entry = product of the slices (section 2.1)."""
    T = V(cores[0])  # (I_1, r_1)
    for c in cores[1:]:
        T = T @ H(c)  # (I_1..I_{n-1}, I_n r_n)
        T = T.reshape(-1, c.shape[2])
    return T.reshape(dims_of(cores))


def tt_add(A, B, alpha=1.0, beta=1.0):
    """alpha*A + beta*B as block-diagonal cores (section 2.1)."""
    N = len(A)
    if N == 1:
        return [alpha * A[0] + beta * B[0]]
    out = []
    for n in range(N):
        a, b = A[n], B[n]
        if n == 0:
            out.append(np.concatenate([alpha * a, beta * b], axis=2))
        elif n == N - 1:
            out.append(np.concatenate([a, b], axis=0))
        else:
            c = np.zeros((a.shape[0] + b.shape[0], a.shape[1], a.shape[2] + b.shape[2]))
            c[: a.shape[0], :, : a.shape[2]] = a
            c[a.shape[0]:, :, a.shape[2]:] = b
            out.append(c)
    return out


def tt_norm(X):
    """||X|| by a left-to-right Householder orthogonalisation: once cores
    1..N-1 are left-orthogonal the norm is the Frobenius norm of the last
    core (section 2.3, mirrored Algorithm 1)."""
    X = [np.array(c, dtype=np.float64) for c in X]
    for n in range(len(X) - 1):
        Q, R = np.linalg.qr(V(X[n]))
        nxt = R @ H(X[n + 1])
        X[n + 1] = nxt.reshape(R.shape[0], X[n + 1].shape[1], X[n + 1].shape[2])
    return float(np.linalg.norm(X[-1]))


def rel_diff(A, B):
    """||A - B|| / ||B|| through the orthogonalised difference TT (never the
    Gram expansion, which cancels to about 1e-8)."""
    return tt_norm(tt_add(A, B, 1.0, -1.0)) / tt_norm(B)


def inner(X, Y):
    """<X, Y> as Algorithm 3 run with the second tensor of rank R (appendix A):
    the chain W_1, then one more contraction with the first cores."""
    W = partial_contractions_rl(X, Y)
    if len(X) == 1:
        return float(np.sum(X[0] * Y[0]))
    Z = V(X[0]) @ W[1]
    return float((H(Z.reshape(1, X[0].shape[1], -1)) @ H(Y[0]).T)[0, 0])


# ----------------------------------------------------------------------------
# Sketch: Definition 3.1 with a counter-based SplitMix64 / Box-Muller generator
# ----------------------------------------------------------------------------

_GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_MASK = (1 << 64) - 1


def splitmix64_mix(z):
    """SplitMix64 output function on a uint64 numpy array (wrapping)."""
    z = np.asarray(z, dtype=np.uint64)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
    return z ^ (z >> np.uint64(31))


def splitmix64_stream(state, idx):
    """idx-th output (idx >= 1) of the SplitMix64 stream started at `state`:
    mix(state + idx * gamma) mod 2^64."""
    idx = np.asarray(idx, dtype=np.uint64)
    return splitmix64_mix(np.uint64(state) + idx * np.uint64(_GAMMA))


def sketch_core_key(seed, n):
    """Key of sketch core n (0-based): output n+1 of the stream seeded `seed`."""
    return int(splitmix64_stream(np.uint64(seed & _MASK), np.array([n + 1]))[0])


def gaussian_stream(key, count):
    """`count` standard normals from the stream keyed `key`: element k uses
    pair p = k // 2 built from stream outputs 2p+1 and 2p+2,
    u1 = (a >> 11 + 1) 2^-53 in (0, 1], u2 = (b >> 11) 2^-53 in [0, 1),
    z_{2p} = sqrt(-2 ln u1) cos(2 pi u2), z_{2p+1} = sqrt(-2 ln u1) sin(2 pi u2)."""
    npairs = (count + 1) // 2
    p = np.arange(npairs, dtype=np.uint64)
    a = splitmix64_stream(key, np.uint64(2) * p + np.uint64(1))
    b = splitmix64_stream(key, np.uint64(2) * p + np.uint64(2))
    u1 = ((a >> np.uint64(11)).astype(np.float64) + 1.0) * (2.0 ** -53)
    u2 = (b >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    rad = np.sqrt(-2.0 * np.log(u1))
    th = (2.0 * math.pi) * u2
    z = np.empty(2 * npairs)
    z[0::2] = rad * np.cos(th)
    z[1::2] = rad * np.sin(th)
    return z[:count]


def round_f32(x):
    """Nearest-even FP32 value of each entry, returned in float64."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(x):
    """Reading of the BF16 sketch: each FP64 value rounded to nearest-even
    FP32, then to nearest-even bfloat16 (8 significant bits), returned in
    float64 (finite inputs)."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    keep = (u >> np.uint64(16)) & np.uint64(1)          # lowest kept bit
    u = ((u + np.uint64(0x7FFF) + keep) >> np.uint64(16)) << np.uint64(16)
    return u.astype(np.uint32).view(np.float32).astype(np.float64).reshape(f.shape)


def make_sketch(seed, dims, sketch_ranks):
    """Random Gaussian TT (Definition 3.1): core n has shape
    (l_{n-1}, I_n, l_n) with iid N(0, 1/(l_{n-1} I_n l_n)) entries."""
    cores = []
    for n, I in enumerate(dims):
        shape = (int(sketch_ranks[n]), int(I), int(sketch_ranks[n + 1]))
        cnt = shape[0] * shape[1] * shape[2]
        z = gaussian_stream(sketch_core_key(seed, n), cnt)
        cores.append((z / math.sqrt(cnt)).reshape(shape))
    return cores


# ----------------------------------------------------------------------------
# Rank plan
# ----------------------------------------------------------------------------


def plan_ranks(dims, ranks, target, oversample):
    """Sketch ranks l_n and output ranks r_n (readings in the module header):
    the thin QR of the (l_{n-1} I_n) x l_n sketch needs l_n <= l_{n-1} I_n;
    the right factor limits l_n <= I_{n+1} ... I_N; l_n <= R_n avoids sketches
    wider than the unfolding's rank."""
    N = len(dims)
    if target < 1 or oversample < 0:
        raise ValueError("target >= 1 and oversample >= 0 required")
    lreq = target + oversample
    u = [1] * (N + 1)
    for n in range(N - 1, 0, -1):
        u[n] = min(lreq, dims[n] * u[n + 1])
    ell = [1] * (N + 1)
    for n in range(1, N):
        ell[n] = min(lreq, ell[n - 1] * dims[n - 1], u[n], ranks[n])
    out = [1] + [min(target, ell[n]) for n in range(1, N)] + [1]
    return ell, out


# ----------------------------------------------------------------------------
# Algorithm 3: right-to-left partial contractions
# ----------------------------------------------------------------------------


def partial_contractions_rl(X, Y):
    """W_n = H(X_{n+1:N}) H(Y_{n+1:N})^T for 1 <= n < N, returned as a list
    indexed by n (entry 0 unused).  W_{N-1} = H(X_N) H(Y_N)^T, then for
    n = N-1 .. 2:  V(Z_n) = V(X_n) W_n,  W_{n-1} = H(Z_n) H(Y_n)^T."""
    N = len(X)
    W = [None] * N
    if N < 2:
        return W
    W[N - 1] = H(X[N - 1]) @ H(Y[N - 1]).T
    for n in range(N - 1, 1, -1):  # 1-based core index n
        Xn, Yn = X[n - 1], Y[n - 1]
        Z = V(Xn) @ W[n]
        Z = Z.reshape(Xn.shape[0], Xn.shape[1], W[n].shape[1])
        W[n - 1] = H(Z) @ H(Yn).T
    return W


# ----------------------------------------------------------------------------
# Algorithm 5: Randomize-then-Orthogonalize
# ----------------------------------------------------------------------------


def qr_pos(A):
    """Thin Householder QR (LAPACK) with diag(R) >= 0."""
    Q, R = np.linalg.qr(A, mode="reduced")
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d, R * d[:, None]


def rto_sweep(Y, W):
    """Left-to-right pass of Algorithm 5 given the partial contractions W_n
    of Y with the sketch.  Returns the left-orthogonal TT X with ranks l_n
    (the column counts of W_n)."""
    N = len(Y)
    out = []
    X = np.array(Y[0], dtype=np.float64)
    for n in range(1, N):  # 1-based: n = 1 .. N-1
        Z = V(X)                      # l_{n-1} I_n x R_n
        Ys = Z @ W[n]                 # sketched matrix, l_{n-1} I_n x l_n
        Q, _ = qr_pos(Ys)
        ln = W[n].shape[1]
        out.append(Q.reshape(X.shape[0], X.shape[1], ln))
        M = Q.T @ Z                   # l_n x R_n
        Ynext = Y[n]
        X = (M @ H(Ynext)).reshape(ln, Ynext.shape[1], Ynext.shape[2])
    out.append(X)
    return out


def truncate_rl(X, out_ranks):
    """Truncate a left-orthogonal TT to ranks out_ranks by a right-to-left
    sweep: for n = N .. 2, SVD of H(X_n) (its singular values are those of
    the n-1 unfolding because cores 1..n-1 are left-orthogonal), keep
    r_{n-1} triplets, X_n <- V_k^T, X_{n-1} <- X_{n-1} x_3 (U_k S_k).
    Returns (cores, tails) with tails[n] = sum of discarded s_j^2 at bond n."""
    X = [np.array(c, dtype=np.float64) for c in X]
    N = len(X)
    tails = [0.0] * (N + 1)
    for n in range(N - 1, 0, -1):  # 0-based core index, left bond n
        Hn = H(X[n])
        U, S, Vt = np.linalg.svd(Hn, full_matrices=False)
        k = min(int(out_ranks[n]), S.shape[0])
        tails[n] = float(np.sum(S[k:] ** 2))
        X[n] = Vt[:k].reshape(k, X[n].shape[1], X[n].shape[2])
        P = U[:, :k] * S[:k]
        prev = X[n - 1]
        X[n - 1] = (V(prev) @ P).reshape(prev.shape[0], prev.shape[1], k)
    return X, tails


def round_rand(Y, target, oversample=0, seed=None, sketch=None, truncate=True):
    """Randomize-then-Orthogonalize rounding (Algorithm 5) of TT Y.

    The sketch is either drawn from `seed` (Definition 3.1, generator in the
    module header) or given.  With truncate and some r_n < l_n the left-
    orthogonal output is truncated by `truncate_rl`."""
    Y = [np.array(c, dtype=np.float64) for c in Y]
    N = len(Y)
    if N == 1:
        return [Y[0].copy()]
    dims, ranks = dims_of(Y), ranks_of(Y)
    ell, out_ranks = plan_ranks(dims, ranks, target, oversample)
    if sketch is None:
        sketch = make_sketch(seed, dims, ell)
    W = partial_contractions_rl(Y, sketch)
    X = rto_sweep(Y, W)
    if truncate and any(out_ranks[n] < ell[n] for n in range(N + 1)):
        X, _ = truncate_rl(X, out_ranks)
    return X


def truncate_rl_eps(X, eps0, max_rank=None):
    """Tolerance-driven truncation of a left-orthogonal TT (the section 3.2
    remark after Algorithm 5: choose the sketch ranks large, then run the
    truncation loop of Algorithm 2 with its threshold).  ||X|| is the
    Frobenius norm of the last core (the others are left-orthogonal); with
    eps = eps0 ||X|| / sqrt(N-1) (Algorithm 2), for n = N .. 2 the SVD of
    H(X_n) keeps the smallest k >= 1 with sqrt(sum_{j>k} s_j^2) <= eps
    (capped by max_rank), X_n <- V_k^T, X_{n-1} <- X_{n-1} x_3 (U_k S_k).
    Then ||X_out - X||^2 = sum of the discarded s_j^2 <= eps0^2 ||X||^2.
    Returns (cores, ranks, tails)."""
    X = [np.array(c, dtype=np.float64) for c in X]
    N = len(X)
    tails = [0.0] * (N + 1)
    if N == 1:
        return X, ranks_of(X), tails
    eps = eps0 * float(np.linalg.norm(X[-1])) / math.sqrt(N - 1)
    for n in range(N - 1, 0, -1):
        U, S, Vt = np.linalg.svd(H(X[n]), full_matrices=False)
        k = _trunc_rank(S, eps, max_rank)
        tails[n] = float(np.sum(S[k:] ** 2))
        X[n] = Vt[:k].reshape(k, X[n].shape[1], X[n].shape[2])
        prev = X[n - 1]
        X[n - 1] = (V(prev) @ (U[:, :k] * S[:k])).reshape(prev.shape[0], prev.shape[1], k)
    return X, ranks_of(X), tails


def round_rand_eps(Y, max_rank, eps0, seed=None, sketch=None):
    """Rounding to a tolerance with ranks not known in advance (section 3.2,
    remark after Algorithm 5): Randomize-then-Orthogonalize with sketch ranks
    from plan_ranks(target = max_rank, oversample = 0), then truncate_rl_eps.
    Returns (cores, ranks, tails)."""
    X = round_rand(Y, max_rank, 0, seed=seed, sketch=sketch, truncate=False)
    return truncate_rl_eps(X, eps0)


def round_sum_rand_eps(summands, coeffs, max_rank, eps0, seed=None, sketch=None):
    """The same for a sum of TTs (Algorithm 7, then truncate_rl_eps)."""
    X = round_sum_rand(summands, coeffs, max_rank, 0, seed=seed, sketch=sketch, truncate=False)
    return truncate_rl_eps(X, eps0)


# ----------------------------------------------------------------------------
# Algorithm 7: rounding a sum of TTs
# ----------------------------------------------------------------------------


def sum_plan(summands, target, oversample):
    dims = dims_of(summands[0])
    N = len(dims)
    formal = [1] + [sum(int(t[n].shape[2]) for t in summands) for n in range(N - 1)] + [1]
    return plan_ranks(dims, formal, target, oversample)


def round_sum_rand(summands, coeffs, target, oversample=0, seed=None, sketch=None,
                   truncate=True):
    """Algorithm 7.  One sketch for every summand; W^{(j)} per summand; the
    sweep uses the stacked [W^{(1)}; ...; W^{(s)}] and builds the next core
    summand by summand: X_{n+1}(:, i, block j) = M^{(j)} Y^{(j)}_{n+1}(:, i, :),
    and at n = N-1, X_N = sum_j M^{(j)} Y^{(j)}_N."""
    s = len(summands)
    if coeffs is None:
        coeffs = np.ones(s)
    Ys = [[np.array(c, dtype=np.float64) for c in t] for t in summands]
    N = len(Ys[0])
    if N == 1:
        return [sum(float(coeffs[j]) * Ys[j][0] for j in range(s))]
    dims = dims_of(Ys[0])
    ell, out_ranks = sum_plan(Ys, target, oversample)
    if sketch is None:
        sketch = make_sketch(seed, dims, ell)
    Ws = [partial_contractions_rl(t, sketch) for t in Ys]
    X = np.concatenate([float(coeffs[j]) * Ys[j][0] for j in range(s)], axis=2)
    out = []
    for n in range(1, N):
        Z = V(X)
        Wst = np.vstack([Ws[j][n] for j in range(s)])
        Q, _ = qr_pos(Z @ Wst)
        ln = ell[n]
        out.append(Q.reshape(X.shape[0], X.shape[1], ln))
        M = Q.T @ Z
        widths = [int(t[n - 1].shape[2]) for t in Ys]
        offs = np.concatenate([[0], np.cumsum(widths)])
        Mj = [M[:, offs[j]:offs[j + 1]] for j in range(s)]
        I1 = dims[n]
        if n < N - 1:
            blocks = [(Mj[j] @ H(Ys[j][n])).reshape(ln, I1, Ys[j][n].shape[2])
                      for j in range(s)]
            X = np.concatenate(blocks, axis=2)
        else:
            X = sum((Mj[j] @ H(Ys[j][n])) for j in range(s)).reshape(ln, I1, 1)
    out.append(X)
    if truncate and any(out_ranks[n] < ell[n] for n in range(N + 1)):
        out, _ = truncate_rl(out, out_ranks)
    return out


# ----------------------------------------------------------------------------
# Algorithms 1 and 2: deterministic TT-rounding
# ----------------------------------------------------------------------------


def orthogonalize_rl(Y):
    """Algorithm 1: for n = N .. 2, QR of H(X_n)^T, H(X_n) <- Q^T,
    X_{n-1} <- X_{n-1} x_3 R^T.  Returns a right-orthogonal TT.  When
    H(X_n)^T is wide (I_n r_n < r_{n-1} rows), Q is square and the bond rank
    drops to I_n r_n; Q is then the QR factor of the leading square block of
    H(X_n)^T (diag >= 0), R = Q^T H(X_n)^T."""
    X = [np.array(c, dtype=np.float64) for c in Y]
    for n in range(len(X) - 1, 0, -1):
        Ht = H(X[n]).T
        m, cc = Ht.shape
        if m >= cc:
            Q, R = qr_pos(Ht)
        else:
            Q, _ = qr_pos(Ht[:, :m])
            R = Q.T @ Ht
        k = Q.shape[1]
        X[n] = Q.T.reshape(k, X[n].shape[1], X[n].shape[2])
        prev = X[n - 1]
        X[n - 1] = (V(prev) @ R.T).reshape(prev.shape[0], prev.shape[1], k)
    return X


def gaussian_matrix(seed, n, rows, cols):
    """The Gaussian matrix Omega_n (rows x cols) of Algorithm 4: the
    Definition 3.1 generator for a single core of rows*cols entries keyed by
    seed + n, iid N(0, 1/(rows cols)), read row-major."""
    return make_sketch(int(seed) + int(n), [rows * cols], [1, 1])[0].reshape(rows, cols)


def round_orth_rand(Y, target, oversample=0, seed=None, omegas=None, truncate=True):
    """Orthogonalize-then-Randomize (Algorithm 4): OrthogonalizeRL (Algorithm 1),
    then for n = 1 .. N-1 with Z_n = V(X_n): Y_n = Z_n Omega_n, thin QR
    (diag(R) >= 0), V(X_n) <- Q, M_n = Q^T Z_n, H(X_{n+1}) = M_n H(X_{n+1}).
    Sketch ranks l_n from plan_ranks on the ranks after Algorithm 1; Omega_n
    (R_n x l_n) given or drawn by gaussian_matrix(seed, n, ...).  With
    truncate and some r_n < l_n the left-orthogonal result is truncated as
    round_rand's."""
    X = orthogonalize_rl(Y)
    N = len(X)
    if N == 1:
        return X
    dims, ranks = dims_of(X), ranks_of(X)
    ell, out_ranks = plan_ranks(dims, ranks, target, oversample)
    if omegas is None:
        omegas = [None] + [gaussian_matrix(seed, n, ranks[n], ell[n]) for n in range(1, N)]
    out = rto_sweep(X, omegas)
    if truncate and any(out_ranks[n] < ell[n] for n in range(N + 1)):
        out, _ = truncate_rl(out, out_ranks)
    return out


def _trunc_rank(S, eps_abs, max_rank):
    k = S.shape[0]
    if eps_abs > 0:
        tail2 = np.concatenate([np.cumsum((S ** 2)[::-1])[::-1], [0.0]])
        # smallest k >= 1 with sqrt(tail2[k]) <= eps_abs
        ok = np.nonzero(np.sqrt(tail2) <= eps_abs)[0]
        k = max(1, int(ok[0])) if ok.size else S.shape[0]
    if max_rank is not None and max_rank > 0:
        k = min(k, int(max_rank))
    return max(1, min(k, S.shape[0]))


def round_svd(Y, eps0=0.0, max_rank=None):
    """Algorithm 2 (deterministic TT-Rounding).  Returns (X, ranks, tails)."""
    N = len(Y)
    X = orthogonalize_rl(Y)
    if N == 1:
        return X, ranks_of(X), [0.0, 0.0]
    nrm = float(np.linalg.norm(X[0]))
    eps = eps0 * nrm / math.sqrt(N - 1)
    tails = [0.0] * (N + 1)
    for n in range(N - 1):
        Q, R = qr_pos(V(X[n]))
        U, S, Vt = np.linalg.svd(R, full_matrices=False)
        k = _trunc_rank(S, eps, max_rank)
        tails[n + 1] = float(np.sum(S[k:] ** 2))
        X[n] = (Q @ U[:, :k]).reshape(X[n].shape[0], X[n].shape[1], k)
        nxt = (S[:k, None] * Vt[:k]) @ H(X[n + 1])
        X[n + 1] = nxt.reshape(k, X[n + 1].shape[1], X[n + 1].shape[2])
    return X, ranks_of(X), tails


# ----------------------------------------------------------------------------
# Algorithm 6: Two-Sided-Randomization (generalized Nystrom, section 3.3)
# ----------------------------------------------------------------------------

# singular values of W^L_n W^R_n at or below this fraction of the largest are
# treated as zero in the pseudo-inverse
NYSTROM_RCOND = 1e-6


def plan_two_sided_ranks(dims, ranks, target):
    """Left sketch ranks l_n (the output ranks) and right sketch ranks rho_n.

    l_n follows plan_ranks with no oversampling.  rho_n = ceil(3 l_n / 2)
    (the choice the experiments of section 4 make for the right sketch,
    after the generalized Nystrom recommendation of section 2.2), capped by
    I_{n+1} ... I_N, the row count of Omega_n; rho_0 = rho_N = 1."""
    N = len(dims)
    ell, _ = plan_ranks(dims, ranks, target, 0)
    big = 1 << 40
    w = [1] * (N + 1)
    for n in range(N - 1, 0, -1):
        w[n] = min(big, int(dims[n]) * w[n + 1])
    rho = [1] * (N + 1)
    for n in range(1, N):
        rho[n] = min((3 * ell[n] + 1) // 2, w[n])
    return ell, rho


def partial_contractions_lr(X, Y):
    """Left-to-right partial contractions, the mirror of Algorithm 3:
    W_n = V(Y_{1:n})^T V(X_{1:n}) (r^Y_n x r^X_n) for 1 <= n < N, as a list
    indexed by n (entry 0 unused).  W_1 = V(Y_1)^T V(X_1), then for
    n = 2 .. N-1:  Z = W_{n-1} H(X_n) read as V(Z) (r^Y_{n-1} I_n x r^X_n),
    W_n = V(Y_n)^T V(Z).  With Y the left sketch L this is
    W^L_n = Psi_n V(X_{1:n})."""
    N = len(X)
    W = [None] * N
    if N < 2:
        return W
    W[1] = V(Y[0]).T @ V(X[0])
    for n in range(2, N):  # 1-based core index n
        Xn, Yn = X[n - 1], Y[n - 1]
        Z = (W[n - 1] @ H(Xn)).reshape(W[n - 1].shape[0] * Xn.shape[1], Xn.shape[2])
        W[n] = V(Yn).T @ Z
    return W


def nystrom_factors(WL, WR):
    """Equation (LnRn): with the SVD W^L W^R = U S V^T,
    L = W^R V (S^+)^(1/2) and R = (S^+)^(1/2) U^T W^L, where S^+ inverts the
    singular values above NYSTROM_RCOND times the largest and zeroes the
    rest.  Returns (L, R)."""
    C = WL @ WR
    U, S, Vt = np.linalg.svd(C, full_matrices=False)
    h = np.zeros_like(S)
    if S.size and S[0] > 0:
        keep = S > NYSTROM_RCOND * S[0]
        h[keep] = 1.0 / np.sqrt(S[keep])
    Lf = (WR @ Vt.T) * h[None, :]
    Rf = h[:, None] * (U.T @ WL)
    return Lf, Rf


def round_two_sided(Y, target, seed_left=None, seed_right=None, sketch_left=None,
                    sketch_right=None):
    """Two-Sided-Randomization rounding (Algorithm 6) of TT Y to ranks l_n.

    Sketches L (ranks l_n) and R (ranks rho_n) are drawn from seed_left and
    seed_right (Definition 3.1) or given.  W^L from the left, W^R from the
    right (Algorithm 3), the factors of equation (LnRn) at every bond, then
    every core independently: X_1 = V(Y_1) L_1, H(X_n) = R_{n-1} H(V(Y_n) L_n),
    H(X_N) = R_{N-1} H(Y_N)."""
    Y = [np.array(c, dtype=np.float64) for c in Y]
    N = len(Y)
    if N == 1:
        return [Y[0].copy()]
    dims, ranks = dims_of(Y), ranks_of(Y)
    ell, rho = plan_two_sided_ranks(dims, ranks, target)
    if sketch_left is None:
        sketch_left = make_sketch(seed_left, dims, ell)
    if sketch_right is None:
        sketch_right = make_sketch(seed_right, dims, rho)
    WL = partial_contractions_lr(Y, sketch_left)
    WR = partial_contractions_rl(Y, sketch_right)
    Lf, Rf = [None] * N, [None] * N
    for n in range(1, N):
        Lf[n], Rf[n] = nystrom_factors(WL[n], WR[n])
    X = [(V(Y[0]) @ Lf[1]).reshape(1, dims[0], ell[1])]
    for n in range(2, N):  # 1-based core index n
        T = (V(Y[n - 1]) @ Lf[n]).reshape(ranks[n - 1], dims[n - 1], ell[n])
        X.append((Rf[n - 1] @ H(T)).reshape(ell[n - 1], dims[n - 1], ell[n]))
    X.append((Rf[N - 1] @ H(Y[N - 1])).reshape(ell[N - 1], dims[N - 1], 1))
    return X


# ----------------------------------------------------------------------------
# Dense twins (tiny sizes only)
# ----------------------------------------------------------------------------


def dense_rto(T, sketch):
    """The sequential randomized range finder on unfoldings of the dense
    tensor T, which Algorithm 5 evaluates in factored form: with
    T_1 = T_(1) and Omega_n = H(sketch_{n+1:N})^T, for n = 1..N-1:
    Q_n = qr(T_n Omega_n), T_{n+1} = reshape(Q_n^T T_n); last core T_N."""
    dims = list(T.shape)
    N = len(dims)
    ell = [1] + [int(c.shape[2]) for c in sketch]
    out = []
    Tn = T.reshape(dims[0], -1)
    for n in range(1, N):
        tail = sketch[n:]
        Om = full_with_left_rank(tail)  # (l_n, I_{n+1}..I_N)
        Q, _ = qr_pos(Tn @ Om.T)
        out.append(Q.reshape(ell[n - 1], dims[n - 1], ell[n]))
        Tn = (Q.T @ Tn).reshape(ell[n] * dims[n], -1)
    out.append(Tn.reshape(ell[N - 1], dims[N - 1], 1))
    return out


def full_with_left_rank(cores):
    """H(C_{1:k}) for a train whose first core has left rank > 1:
    a (r_0) x (I_1 ... I_k) matrix."""
    T = H(cores[0])  # r0 x (I r1)
    r0 = cores[0].shape[0]
    T = T.reshape(-1, cores[0].shape[2])  # (r0 I) x r1
    for c in cores[1:]:
        T = (T @ H(c)).reshape(-1, c.shape[2])
    return T.reshape(r0, -1)


def dense_tt_svd(T, max_rank):
    """Sequential truncated SVDs of the unfoldings of the dense tensor T
    (TT-SVD) at fixed ranks: max_rank is an int (same cap at every bond) or a
    list of N+1 ranks."""
    dims = list(T.shape)
    N = len(dims)
    caps = list(max_rank) if hasattr(max_rank, "__len__") else [max_rank] * (N + 1)
    cores = []
    r = 1
    M = T.reshape(dims[0], -1)
    for n in range(N - 1):
        M = M.reshape(r * dims[n], -1)
        U, S, Vt = np.linalg.svd(M, full_matrices=False)
        k = min(int(caps[n + 1]), S.shape[0])
        cores.append(U[:, :k].reshape(r, dims[n], k))
        M = S[:k, None] * Vt[:k]
        r = k
    cores.append(M.reshape(r, dims[-1], 1))
    return cores


# ----------------------------------------------------------------------------
# Flop accounting (section 3.5 / appendix A, exact GEMM shapes)
# ----------------------------------------------------------------------------


def rto_flops(dims, ranks, ell):
    """Exact 2mnk GEMM flops of Algorithm 3 + Algorithm 5 (QR counted as
    Householder 4mn^2 - 4n^3/3, section 2.1)."""
    N = len(dims)
    f = 0.0
    # W chain
    f += 2.0 * ranks[N - 1] * dims[N - 1] * ell[N - 1]
    for n in range(N - 1, 1, -1):
        Rl, I, Rr = ranks[n - 1], dims[n - 1], ranks[n]
        f += 2.0 * Rl * I * Rr * ell[n]          # V(Y_n) W_n
        f += 2.0 * Rl * I * ell[n] * ell[n - 1]  # H(Z_n) H(R_n)^T
    for n in range(1, N):
        m = ell[n - 1] * dims[n - 1]
        f += 2.0 * m * ranks[n] * ell[n]           # Z_n W_n
        f += 4.0 * m * ell[n] ** 2 - 4.0 * ell[n] ** 3 / 3.0  # QR
        f += 2.0 * ell[n] * m * ranks[n]           # Q^T Z_n
        f += 2.0 * ell[n] * ranks[n] * dims[n] * ranks[n + 1]  # M_n H(Y_{n+1})
    return f


# ----------------------------------------------------------------------------
# Section 4.2: TT-GMRES with randomized rounding of the sums
# ----------------------------------------------------------------------------


def apply_mode_matrix(core, M):
    """core x_2 M: out[a, i, b] = sum_j M[i, j] core[a, j, b]."""
    return np.einsum("ij,ajb->aib", M, core)


def operator_terms(mats, X):
    """The N terms (A_{i,1} x ... x A_{i,N}) X of a Kronecker-sum operator
    applied to the TT X, each a TT with X's ranks (mats[i][n] None = I)."""
    return [[c if M is None else apply_mode_matrix(c, M) for M, c in zip(row, X)]
            for row in mats]


def tt_gmres(mats, f, precond, max_rank, round_eps, tol, max_iter, seed):
    """Right-preconditioned TT-GMRES (section 4.2) with every sum rounded by
    Algorithm 7 to the tolerance round_eps (round_sum_rand_eps, sketch rank
    max_rank).  x_0 = 0, beta = ||f||, V_1 = f / beta; step k:
      Y = (P x I x ... x I) V_k                     (P the preconditioner)
      W = round(sum_i (A_{i,1} x ... x A_{i,N}) Y)  (seed + 2k - 1)
      h_jk = <V_j, W>,  j = 1..k
      Z = round(W - sum_j h_jk V_j)                 (seed + 2k)
      h_{k+1,k} = ||Z||,  V_{k+1} = Z / h_{k+1,k}
    and the least-squares problem min ||beta e_1 - H y|| by Givens rotations;
    the residual estimate |g_{k+1}| / beta is recorded.  It stops when that
    falls to tol or after max_iter steps; then x = (P x I ..) round(sum_j y_j
    V_j) (seed + 2 m + 1).  Returns (x, residual history, iterations)."""
    f = [np.array(c, dtype=np.float64) for c in f]
    beta = math.sqrt(inner(f, f))
    V = [[f[0] / beta] + [c.copy() for c in f[1:]]]
    Hm = np.zeros((max_iter + 1, max_iter))
    cs, sn = np.zeros(max_iter), np.zeros(max_iter)
    g = np.zeros(max_iter + 1)
    g[0] = beta
    res = [1.0]
    m = 0
    for k in range(1, max_iter + 1):
        Vk = V[k - 1]
        Y = [apply_mode_matrix(Vk[0], precond)] + Vk[1:]
        terms = operator_terms(mats, Y)
        W, _, _ = round_sum_rand_eps(terms, None, max_rank, round_eps, seed=seed + 2 * k - 1)
        h = [inner(V[j], W) for j in range(k)]
        Z, _, _ = round_sum_rand_eps([W] + V, [1.0] + [-x for x in h], max_rank, round_eps,
                                     seed=seed + 2 * k)
        hz = float(np.linalg.norm(Z[0]))
        V.append([Z[0] / hz] + Z[1:])
        col = np.array(h + [hz])
        for j in range(k - 1):  # previous rotations
            a, b = col[j], col[j + 1]
            col[j], col[j + 1] = cs[j] * a + sn[j] * b, -sn[j] * a + cs[j] * b
        r = math.hypot(col[k - 1], col[k])
        cs[k - 1], sn[k - 1] = col[k - 1] / r, col[k] / r
        col[k - 1], col[k] = r, 0.0
        Hm[:k + 1, k - 1] = col
        g[k] = -sn[k - 1] * g[k - 1]
        g[k - 1] = cs[k - 1] * g[k - 1]
        res.append(abs(g[k]) / beta)
        m = k
        if res[-1] <= tol:
            break
    y = np.linalg.solve(np.triu(Hm[:m, :m]), g[:m])
    U, _, _ = round_sum_rand_eps(V[:m], list(y), max_rank, round_eps, seed=seed + 2 * m + 1)
    x = [apply_mode_matrix(U[0], precond)] + U[1:]
    return x, res, m


def kron_operator_dense(mats, dims):
    """The dense matrix sum_i A_{i,1} x ... x A_{i,N} (C order of the modes),
    for checks on tiny problems."""
    tot = 0.0
    for row in mats:
        K = np.ones((1, 1))
        for M, d in zip(row, dims):
            K = np.kron(K, np.eye(d) if M is None else M)
        tot = tot + K
    return tot
