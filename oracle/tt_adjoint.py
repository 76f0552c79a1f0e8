"""FP64 CPU oracle of the adjoint of Randomize-then-Orthogonalize.

TEST INFRASTRUCTURE ONLY (same rules as tt_oracle): used by tests/ to check
the library's hand-written reverse pass.  It shares no code with the HIP
library.

The forward map is written once more in plain torch float64 operations on
the CPU (partial contractions of Algorithm 3, then the sweep of Algorithm 5
with the thin QR normalised to diag(R) >= 0, no truncation); its gradient
is torch's reverse-mode differentiation of those operations, including the
QR backward of torch.linalg.qr.  The forward is pinned against the numpy
oracle and the gradient against central finite differences of the numpy
oracle (tests/test_oracle_pins.py).
"""
from __future__ import annotations

import numpy as np
import torch


def _H(c):
    return c.reshape(c.shape[0], -1)


def _V(c):
    return c.reshape(-1, c.shape[2])


def rto_torch(Y, S):
    """Randomize-then-Orthogonalize (Algorithms 3 and 5) of the TT Y (list of
    torch float64 cores) with the sketch TT S; returns the output cores."""
    N = len(Y)
    if N == 1:
        return [Y[0]]
    W = [None] * N
    W[N - 1] = _H(Y[N - 1]) @ _H(S[N - 1]).T
    for n in range(N - 1, 1, -1):          # core n is Y[n-1]
        Zc = _V(Y[n - 1]) @ W[n]
        W[n - 1] = Zc.reshape(Y[n - 1].shape[0], -1) @ _H(S[n - 1]).T
    X = Y[0]
    out = []
    for n in range(1, N):
        Z = _V(X)
        Q, R = torch.linalg.qr(Z @ W[n])
        d = torch.sign(torch.diagonal(R))
        d = torch.where(d == 0, torch.ones_like(d), d)
        Q = Q * d
        out.append(Q.reshape(X.shape[0], X.shape[1], -1))
        M = Q.T @ Z
        X = (M @ _H(Y[n])).reshape(M.shape[0], Y[n].shape[1], Y[n].shape[2])
    out.append(X)
    return out


def rto_vjp(Y, S, gout):
    """Gradient of sum_n <gout_n, out_n> with respect to the cores of Y (all
    numpy arrays in, numpy float64 arrays out)."""
    Yt = [torch.tensor(np.asarray(c, dtype=np.float64), requires_grad=True) for c in Y]
    St = [torch.tensor(np.asarray(c, dtype=np.float64)) for c in S]
    out = rto_torch(Yt, St)
    loss = sum((o * torch.tensor(np.asarray(g, dtype=np.float64))).sum()
               for o, g in zip(out, gout))
    grads = torch.autograd.grad(loss, Yt)
    return [g.detach().numpy() for g in grads]


def tt_inner_torch(A, B):
    """<A, B> of two TTs with the same mode sizes (torch, left to right)."""
    P = torch.ones((1, 1), dtype=A[0].dtype, device=A[0].device)
    for a, b in zip(A, B):
        # P (ra x rb), a (ra, I, ra'), b (rb, I, rb') -> (ra' x rb')
        T = (P.T @ _H(a)).reshape(b.shape[0], a.shape[1], a.shape[2])   # (rb, I, ra')
        P = _V(T).T @ _V(b)
    return P.reshape(())


def loss_round_minus_target(X_out, T):
    """||X_out - T||_F^2 for two TTs (torch)."""
    return tt_inner_torch(X_out, X_out) - 2.0 * tt_inner_torch(X_out, T) + tt_inner_torch(T, T)
