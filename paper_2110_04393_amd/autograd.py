"""torch.autograd bindings of randomized TT-rounding.

The forward pass is tt_round_rand, the backward pass the library's
hand-written adjoint tt_round_rand_backward (no torch arithmetic: torch only
hands over device buffers and the stream).  The sketch is fixed by the seed
and is not differentiated; roundings that truncate are not supported.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from .api import (_DTYPE, _PREC, STORAGE, _check_cores, _shape_of, _stream_handle, _workspace,
                  plan, round_rand)


def round_rand_backward(cores, grad_out, target_rank: int, oversample: int = 0, seed: int = 0,
                        prec: str = "f64", stream=None):
    """Vector-Jacobian product of round_rand: gradients with respect to the
    input cores given cotangents of the output cores."""
    _check_cores(cores)
    if cores[0].dtype != STORAGE[prec]:
        raise ValueError(f"prec {prec!r} needs {STORAGE[prec]} cores")
    dims, ranks = _shape_of(cores)
    N = len(dims)
    _, out_r = plan(dims, ranks, target_rank, oversample)
    go = []
    for n in range(N):
        shape = (out_r[n], dims[n], out_r[n + 1])
        g = grad_out[n]
        if g is None:
            g = torch.zeros(shape, dtype=cores[0].dtype, device=cores[0].device)
        if tuple(g.shape) != shape:
            raise ValueError(f"grad_out[{n}] has shape {tuple(g.shape)}, expected {shape}")
        go.append(g.to(cores[0].dtype).contiguous())
    gi = [torch.empty_like(c) for c in cores]
    b = ctypes.c_size_t(0)
    L.check(L.lib().tt_round_rand_backward_workspace(N, L.i64_array(dims), L.i64_array(ranks),
                                                     int(target_rank), int(oversample),
                                                     _PREC[prec], ctypes.byref(b)))
    ws = _workspace(b.value, cores[0].device)
    L.check(L.lib().tt_round_rand_backward(
        N, L.i64_array(dims), L.i64_array(ranks), L.ptr_array([c.data_ptr() for c in cores]),
        _DTYPE[cores[0].dtype], int(target_rank), int(oversample), int(seed) & ((1 << 64) - 1),
        _PREC[prec], L.ptr_array([g.data_ptr() for g in go]),
        L.ptr_array([g.data_ptr() for g in gi]), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
        _stream_handle(stream)))
    return gi


class _RoundRand(torch.autograd.Function):
    @staticmethod
    def forward(ctx, target_rank, oversample, seed, prec, *cores):
        cores = [c.contiguous() for c in cores]
        out = round_rand(cores, target_rank, oversample, seed=seed, prec=prec)
        ctx.save_for_backward(*cores)
        ctx.cfg = (target_rank, oversample, seed, prec)
        return tuple(out)

    @staticmethod
    def backward(ctx, *grads):
        cores = list(ctx.saved_tensors)
        target_rank, oversample, seed, prec = ctx.cfg
        gi = round_rand_backward(cores, list(grads), target_rank, oversample, seed, prec)
        return (None, None, None, None, *gi)


def round_rand_ad(cores, target_rank: int, oversample: int = 0, seed: int = 0,
                  prec: str = "f64"):
    """Differentiable randomized rounding (no truncation): returns the output
    cores; gradients flow to the input cores through the library adjoint."""
    return list(_RoundRand.apply(int(target_rank), int(oversample), int(seed), prec, *cores))
