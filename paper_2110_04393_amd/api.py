"""Python binding of libttround: torch tensors in, torch tensors out.

Torch only provides device memory and the stream; every arithmetic step runs
in the library's HIP kernels.  Cores are lists of C-contiguous device tensors
of shape (r_{n-1}, I_n, r_n).
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import _lib as L

_PREC = {"f64": L.TT_PREC_F64, "f32": L.TT_PREC_F32, "bf16": L.TT_PREC_MIXED_BF16}
_DTYPE = {torch.float64: L.TT_F64, torch.float32: L.TT_F32, torch.bfloat16: L.TT_BF16}
# storage type of the cores in each arithmetic mode
STORAGE = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.float32}


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes_void(s.cuda_stream)


def ctypes_void(v):
    import ctypes
    return ctypes.c_void_p(int(v))


def _shape_of(cores):
    dims = [int(c.shape[1]) for c in cores]
    ranks = [1] + [int(c.shape[2]) for c in cores]
    return dims, ranks


def _check_cores(cores, what="cores"):
    if len(cores) == 0:
        raise ValueError(f"{what}: empty TT")
    dt = cores[0].dtype
    dev = cores[0].device
    prev = 1
    for n, c in enumerate(cores):
        if c.dim() != 3:
            raise ValueError(f"{what}[{n}] must be 3-D (r_prev, I, r_next)")
        if not c.is_cuda:
            raise ValueError(f"{what}[{n}] must be a device tensor")
        if c.dtype != dt or c.device != dev:
            raise ValueError(f"{what}: mixed dtypes/devices")
        if not c.is_contiguous():
            raise ValueError(f"{what}[{n}] must be contiguous")
        if int(c.shape[0]) != prev:
            raise ValueError(f"{what}[{n}]: left rank {c.shape[0]} != {prev}")
        prev = int(c.shape[2])
    if prev != 1:
        raise ValueError(f"{what}: last rank must be 1")
    if dt not in (torch.float64, torch.float32):
        raise ValueError(f"{what}: dtype must be float64 or float32")


def version() -> int:
    return L.lib().tt_version()


def plan(dims: Sequence[int], ranks: Sequence[int], target_rank: int, oversample: int = 0):
    """Sketch ranks l_n and output ranks r_n (host only)."""
    N = len(dims)
    sr = L.i64_array([0] * (N + 1))
    orr = L.i64_array([0] * (N + 1))
    L.check(L.lib().tt_round_rand_plan(N, L.i64_array(dims), L.i64_array(ranks),
                                       int(target_rank), int(oversample), sr, orr))
    return [sr[i] for i in range(N + 1)], [orr[i] for i in range(N + 1)]


def round_rand_workspace(dims, ranks, target_rank, oversample=0, prec="f64") -> int:
    import ctypes
    b = ctypes.c_size_t(0)
    L.check(L.lib().tt_round_rand_workspace(len(dims), L.i64_array(dims), L.i64_array(ranks),
                                            int(target_rank), int(oversample), _PREC[prec],
                                            ctypes.byref(b)))
    return int(b.value)


def sum_round_workspace(dims, ranks_list, target_rank, oversample=0, prec="f64") -> int:
    import ctypes
    b = ctypes.c_size_t(0)
    flat = [r for rr in ranks_list for r in rr]
    L.check(L.lib().tt_sum_round_workspace(len(ranks_list), len(dims), L.i64_array(dims),
                                           L.i64_array(flat), int(target_rank), int(oversample),
                                           _PREC[prec], ctypes.byref(b)))
    return int(b.value)


def _workspace(nbytes, device):
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def make_sketch(seed: int, dims, sketch_ranks, dtype=torch.float64, device="cuda", stream=None):
    """Random Gaussian TT of Definition 3.1 drawn on the device."""
    N = len(dims)
    cores = [torch.empty((int(sketch_ranks[n]), int(dims[n]), int(sketch_ranks[n + 1])),
                         dtype=dtype, device=device) for n in range(N)]
    L.check(L.lib().tt_make_sketch(int(seed) & ((1 << 64) - 1), N, L.i64_array(dims),
                                   L.i64_array(sketch_ranks), _DTYPE[dtype],
                                   L.ptr_array([c.data_ptr() for c in cores]),
                                   _stream_handle(stream)))
    return cores


def partial_contractions_rl(X, Y, prec="f64", stream=None):
    """W_n = H(X_{n+1:N}) H(Y_{n+1:N})^T, n = 1..N-1 (Algorithm 3); returns a
    list indexed by n with entry 0 = None.  X and Y in the storage type of
    `prec` (float64 for "f64", float32 for "f32" and "bf16")."""
    import ctypes
    _check_cores(X, "X")
    _check_cores(Y, "Y")
    dims, rx = _shape_of(X)
    dy, ry = _shape_of(Y)
    if dims != dy:
        raise ValueError("X and Y must share mode sizes")
    if X[0].dtype != STORAGE[prec] or Y[0].dtype != STORAGE[prec]:
        raise ValueError(f"prec {prec!r} needs {STORAGE[prec]} cores")
    N = len(dims)
    dev = X[0].device
    W = [None] + [torch.empty((rx[n], ry[n]), dtype=STORAGE[prec], device=dev)
                  for n in range(1, N)]
    b = ctypes.c_size_t(0)
    L.check(L.lib().tt_partial_contractions_rl_workspace(N, L.i64_array(dims), L.i64_array(rx),
                                                         L.i64_array(ry), _PREC[prec],
                                                         ctypes.byref(b)))
    ws = _workspace(b.value, dev)
    L.check(L.lib().tt_partial_contractions_rl(
        N, L.i64_array(dims), L.i64_array(rx), L.ptr_array([c.data_ptr() for c in X]),
        L.i64_array(ry), L.ptr_array([c.data_ptr() for c in Y]), _PREC[prec],
        L.ptr_array([w.data_ptr() for w in W[1:]]), ctypes.c_void_p(ws.data_ptr()),
        ws.numel(), _stream_handle(stream)))
    return W


class RoundPlan:
    """Pre-sized outputs and workspace for repeated roundings of one shape
    (the timed benchmark loop allocates nothing)."""

    def __init__(self, dims, ranks, target_rank, oversample=0, prec="f64", device="cuda",
                 dtype=None, summand_ranks=None):
        if prec not in _PREC:
            raise ValueError(f"unknown prec {prec!r}")
        if dtype is None:
            dtype = STORAGE[prec]
        self.dims = [int(d) for d in dims]
        self.N = len(self.dims)
        self.target = int(target_rank)
        self.oversample = int(oversample)
        self.prec = prec
        self.dtype = dtype
        self.device = torch.device(device)
        self.summand_ranks = summand_ranks
        if summand_ranks is not None:
            formal = [1] + [sum(r[n] for r in summand_ranks) for n in range(1, self.N)] + [1]
            self.ranks = formal
            self.ws_bytes = sum_round_workspace(self.dims, summand_ranks, self.target,
                                                self.oversample, prec)
        else:
            self.ranks = [int(r) for r in ranks]
            self.ws_bytes = round_rand_workspace(self.dims, self.ranks, self.target,
                                                 self.oversample, prec)
        self.sketch_ranks, self.out_ranks = plan(self.dims, self.ranks, self.target,
                                                 self.oversample)
        self.workspace = _workspace(self.ws_bytes, self.device)
        self.out = [torch.empty((self.out_ranks[n], self.dims[n], self.out_ranks[n + 1]),
                                dtype=dtype, device=self.device) for n in range(self.N)]
        self._out_ptrs = L.ptr_array([c.data_ptr() for c in self.out])
        self._dims = L.i64_array(self.dims)

    def run(self, cores, seed=0, sketch=None, stream=None):
        import ctypes
        _check_cores(cores)
        dims, ranks = _shape_of(cores)
        if dims != self.dims or ranks != self.ranks:
            raise ValueError("cores do not match the plan's shape")
        st = _stream_handle(stream)
        ptrs = L.ptr_array([c.data_ptr() for c in cores])
        ws = ctypes.c_void_p(self.workspace.data_ptr())
        if sketch is None:
            L.check(L.lib().tt_round_rand(self.N, self._dims, L.i64_array(ranks), ptrs,
                                          _DTYPE[cores[0].dtype], self.target, self.oversample,
                                          int(seed) & ((1 << 64) - 1), _PREC[self.prec],
                                          self._out_ptrs, ws, self.workspace.numel(), st))
        else:
            _check_cores(sketch, "sketch")
            _, sr = _shape_of(sketch)
            L.check(L.lib().tt_round_rand_with_sketch(
                self.N, self._dims, L.i64_array(ranks), ptrs, _DTYPE[cores[0].dtype],
                self.target, self.oversample, L.i64_array(sr),
                L.ptr_array([c.data_ptr() for c in sketch]), _PREC[self.prec], self._out_ptrs,
                ws, self.workspace.numel(), st))
        return self.out

    def run_sum(self, summands, coeffs=None, seed=0, stream=None):
        import ctypes
        s = len(summands)
        flat_ranks, ptrs = [], []
        for t in summands:
            _check_cores(t)
            d, r = _shape_of(t)
            if d != self.dims:
                raise ValueError("summand mode sizes differ from the plan")
            flat_ranks += r
            ptrs += [c.data_ptr() for c in t]
        if self.summand_ranks is None or [list(map(int, r)) for r in self.summand_ranks] != \
                [_shape_of(t)[1] for t in summands]:
            raise ValueError("summand ranks differ from the plan")
        cf = None
        if coeffs is not None:
            cf = (ctypes.c_double * s)(*[float(c) for c in coeffs])
        L.check(L.lib().tt_sum_round(s, self.N, self._dims, L.i64_array(flat_ranks),
                                     L.ptr_array(ptrs), cf, _DTYPE[summands[0][0].dtype],
                                     self.target, self.oversample, int(seed) & ((1 << 64) - 1),
                                     _PREC[self.prec], self._out_ptrs,
                                     ctypes.c_void_p(self.workspace.data_ptr()),
                                     self.workspace.numel(), _stream_handle(stream)))
        return self.out


def round_svd(cores, eps0: float = 0.0, max_rank: int = 0, prec: str = "f64", stream=None):
    """Deterministic TT-rounding (Algorithms 1 and 2).  Returns the output
    cores at their actual ranks (views of freshly allocated buffers)."""
    import ctypes
    _check_cores(cores)
    if prec not in ("f64", "f32"):
        raise ValueError("round_svd supports prec 'f64' and 'f32'")
    if cores[0].dtype != STORAGE[prec]:
        raise ValueError(f"prec {prec!r} needs {STORAGE[prec]} cores")
    dims, ranks = _shape_of(cores)
    N = len(dims)
    bound = L.i64_array([0] * (N + 1))
    L.check(L.lib().tt_round_svd_plan(N, L.i64_array(dims), L.i64_array(ranks), int(max_rank),
                                      bound))
    b = ctypes.c_size_t(0)
    L.check(L.lib().tt_round_svd_workspace(N, L.i64_array(dims), L.i64_array(ranks),
                                           int(max_rank), _PREC[prec], ctypes.byref(b)))
    dev = cores[0].device
    ws = _workspace(b.value, dev)
    bufs = [torch.empty(bound[n] * dims[n] * bound[n + 1], dtype=cores[0].dtype, device=dev)
            for n in range(N)]
    out_r = L.i64_array([0] * (N + 1))
    L.check(L.lib().tt_round_svd(N, L.i64_array(dims), L.i64_array(ranks),
                                 L.ptr_array([c.data_ptr() for c in cores]), _DTYPE[cores[0].dtype],
                                 float(eps0), int(max_rank), _PREC[prec],
                                 L.ptr_array([x.data_ptr() for x in bufs]), out_r,
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                 _stream_handle(stream)))
    r = [out_r[n] for n in range(N + 1)]
    return [bufs[n][: r[n] * dims[n] * r[n + 1]].view(r[n], dims[n], r[n + 1]) for n in range(N)]


def two_sided_plan(dims, ranks, target_rank: int):
    """Left ranks l_n (the output ranks) and right sketch ranks rho_n of
    tt_round_two_sided (host only)."""
    N = len(dims)
    lr, rr = L.i64_array([0] * (N + 1)), L.i64_array([0] * (N + 1))
    L.check(L.lib().tt_round_two_sided_plan(N, L.i64_array(dims), L.i64_array(ranks),
                                            int(target_rank), lr, rr))
    return [lr[n] for n in range(N + 1)], [rr[n] for n in range(N + 1)]


class TwoSidedPlan:
    """Pre-sized outputs and workspace for repeated Two-Sided-Randomization
    roundings (Algorithm 6) of one FP64 shape."""

    def __init__(self, dims, ranks, target_rank, device="cuda"):
        import ctypes
        self.dims = [int(d) for d in dims]
        self.ranks = [int(r) for r in ranks]
        self.N = len(self.dims)
        self.target = int(target_rank)
        self.device = torch.device(device)
        self.left_ranks, self.right_ranks = two_sided_plan(self.dims, self.ranks, self.target)
        b = ctypes.c_size_t(0)
        L.check(L.lib().tt_round_two_sided_workspace(self.N, L.i64_array(self.dims),
                                                     L.i64_array(self.ranks), self.target,
                                                     ctypes.byref(b)))
        self.ws_bytes = int(b.value)
        self.workspace = _workspace(self.ws_bytes, self.device)
        lr = self.left_ranks
        self.out = [torch.empty((lr[n], self.dims[n], lr[n + 1]), dtype=torch.float64,
                                device=self.device) for n in range(self.N)]
        self._out_ptrs = L.ptr_array([c.data_ptr() for c in self.out])
        self._dims = L.i64_array(self.dims)
        self._ranks = L.i64_array(self.ranks)

    def run(self, cores, seed_left=0, seed_right=1, stream=None):
        import ctypes
        _check_cores(cores)
        dims, ranks = _shape_of(cores)
        if dims != self.dims or ranks != self.ranks:
            raise ValueError("cores do not match the plan's shape")
        if cores[0].dtype != torch.float64:
            raise ValueError("two-sided rounding takes float64 cores")
        L.check(L.lib().tt_round_two_sided(
            self.N, self._dims, self._ranks, L.ptr_array([c.data_ptr() for c in cores]),
            _DTYPE[cores[0].dtype], self.target, int(seed_left) & ((1 << 64) - 1),
            int(seed_right) & ((1 << 64) - 1), self._out_ptrs,
            ctypes.c_void_p(self.workspace.data_ptr()), self.ws_bytes, _stream_handle(stream)))
        return self.out


def round_two_sided(cores, target_rank: int, seed_left: int = 0, seed_right: int = 1,
                    stream=None):
    """Two-Sided-Randomization rounding (Algorithm 6) of an FP64 TT; returns
    new output cores (clones) at ranks l_n."""
    _check_cores(cores)
    dims, ranks = _shape_of(cores)
    p = TwoSidedPlan(dims, ranks, target_rank, cores[0].device)
    return [c.clone() for c in p.run(cores, seed_left, seed_right, stream=stream)]


def round_rand(cores, target_rank: int, oversample: int = 0, seed: int = 0, prec: str = "f64",
               sketch: Optional[list] = None, stream=None):
    """Randomize-then-Orthogonalize rounding (Algorithm 5) of a TT; returns
    new output cores (clones)."""
    _check_cores(cores)
    dims, ranks = _shape_of(cores)
    p = RoundPlan(dims, ranks, target_rank, oversample, prec, cores[0].device)
    return [c.clone() for c in p.run(cores, seed=seed, sketch=sketch, stream=stream)]


def _narrowed(out, dims, ranks):
    """Views of the caller-sized output buffers at the ranks the library
    chose (each core written C-contiguous from the start of its buffer)."""
    return [out[n].view(-1)[:ranks[n] * dims[n] * ranks[n + 1]].view(ranks[n], dims[n],
                                                                     ranks[n + 1])
            for n in range(len(dims))]


def round_rand_eps(cores, max_rank: int, eps0: float, seed: int = 0, prec: str = "f64",
                   stream=None):
    """Rounding to the tolerance eps0 with sketch ranks up to max_rank
    (tt_round_rand_eps; section 3.2, remark after Algorithm 5).  Returns the
    output cores at the chosen ranks."""
    import ctypes
    _check_cores(cores)
    if prec not in _PREC:
        raise ValueError(f"unknown prec {prec!r}")
    dims, ranks = _shape_of(cores)
    N = len(dims)
    sr, _ = plan(dims, ranks, max_rank, 0)
    b = ctypes.c_size_t(0)
    L.check(L.lib().tt_round_rand_eps_workspace(N, L.i64_array(dims), L.i64_array(ranks),
                                                int(max_rank), _PREC[prec], ctypes.byref(b)))
    dev = cores[0].device
    ws = _workspace(b.value, dev)
    out = [torch.empty((sr[n], dims[n], sr[n + 1]), dtype=cores[0].dtype, device=dev)
           for n in range(N)]
    got = L.i64_array([0] * (N + 1))
    L.check(L.lib().tt_round_rand_eps(
        N, L.i64_array(dims), L.i64_array(ranks), L.ptr_array([c.data_ptr() for c in cores]),
        _DTYPE[cores[0].dtype], int(max_rank), float(eps0), int(seed) & ((1 << 64) - 1),
        _PREC[prec], L.ptr_array([c.data_ptr() for c in out]), got,
        ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream)))
    return _narrowed(out, dims, [got[i] for i in range(N + 1)])


def sum_round_eps(summands, coeffs, max_rank: int, eps0: float, seed: int = 0,
                  prec: str = "f64", stream=None):
    """Rounding of sum_j coeffs[j] * summands[j] to the tolerance eps0
    (tt_sum_round_eps).  Returns the output cores at the chosen ranks."""
    import ctypes
    if prec not in _PREC:
        raise ValueError(f"unknown prec {prec!r}")
    s = len(summands)
    dims, _ = _shape_of(summands[0])
    N = len(dims)
    flat_ranks, ptrs = [], []
    for t in summands:
        _check_cores(t)
        d, r = _shape_of(t)
        if d != dims:
            raise ValueError("summands must share mode sizes")
        flat_ranks += r
        ptrs += [c.data_ptr() for c in t]
    formal = [1] + [sum(_shape_of(t)[1][n] for t in summands) for n in range(1, N)] + [1]
    sr, _ = plan(dims, formal, max_rank, 0)
    b = ctypes.c_size_t(0)
    L.check(L.lib().tt_sum_round_eps_workspace(s, N, L.i64_array(dims), L.i64_array(flat_ranks),
                                               int(max_rank), _PREC[prec], ctypes.byref(b)))
    dev = summands[0][0].device
    ws = _workspace(b.value, dev)
    out = [torch.empty((sr[n], dims[n], sr[n + 1]), dtype=summands[0][0].dtype, device=dev)
           for n in range(N)]
    cf = None
    if coeffs is not None:
        cf = (ctypes.c_double * s)(*[float(c) for c in coeffs])
    got = L.i64_array([0] * (N + 1))
    L.check(L.lib().tt_sum_round_eps(
        s, N, L.i64_array(dims), L.i64_array(flat_ranks), L.ptr_array(ptrs), cf,
        _DTYPE[summands[0][0].dtype], int(max_rank), float(eps0), int(seed) & ((1 << 64) - 1),
        _PREC[prec], L.ptr_array([c.data_ptr() for c in out]), got,
        ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream)))
    return _narrowed(out, dims, [got[i] for i in range(N + 1)])


def orth_rand_plan(dims, ranks, target_rank: int, oversample: int = 0):
    """Sketch and out ranks of Orthogonalize-then-Randomize (host only)."""
    N = len(dims)
    sr = L.i64_array([0] * (N + 1))
    orr = L.i64_array([0] * (N + 1))
    L.check(L.lib().tt_round_orth_rand_plan(N, L.i64_array(dims), L.i64_array(ranks),
                                            int(target_rank), int(oversample), sr, orr))
    return [sr[i] for i in range(N + 1)], [orr[i] for i in range(N + 1)]


def round_orth_rand(cores, target_rank: int, oversample: int = 0, seed: int = 0,
                    prec: str = "f64", stream=None):
    """Orthogonalize-then-Randomize rounding (Algorithm 4, tt_round_orth_rand);
    returns new output cores."""
    import ctypes
    _check_cores(cores)
    if prec not in ("f64", "f32"):
        raise ValueError("tt_round_orth_rand takes prec 'f64' or 'f32'")
    dims, ranks = _shape_of(cores)
    N = len(dims)
    _, out_ranks = orth_rand_plan(dims, ranks, target_rank, oversample)
    b = ctypes.c_size_t(0)
    L.check(L.lib().tt_round_orth_rand_workspace(N, L.i64_array(dims), L.i64_array(ranks),
                                                 int(target_rank), int(oversample), _PREC[prec],
                                                 ctypes.byref(b)))
    dev = cores[0].device
    ws = _workspace(b.value, dev)
    out = [torch.empty((out_ranks[n], dims[n], out_ranks[n + 1]), dtype=cores[0].dtype,
                       device=dev) for n in range(N)]
    L.check(L.lib().tt_round_orth_rand(
        N, L.i64_array(dims), L.i64_array(ranks), L.ptr_array([c.data_ptr() for c in cores]),
        _DTYPE[cores[0].dtype], int(target_rank), int(oversample), int(seed) & ((1 << 64) - 1),
        _PREC[prec], L.ptr_array([c.data_ptr() for c in out]), ctypes.c_void_p(ws.data_ptr()),
        ws.numel(), _stream_handle(stream)))
    return out


def gmres(mats, f_cores, precond=None, max_rank: int = 60, round_eps: float = 1e-9,
          tol: float = 1e-8, max_iter: int = 40, seed: int = 0, stream=None):
    """TT-GMRES (tt_gmres; section 4.2) for sum_t A_{t,1} x ... x A_{t,N}
    applied to x equal to f.  mats[t][n]: device FP64 I_n x I_n matrices or
    None (identity); precond: device I_1 x I_1 or None.  Returns
    (x cores at their ranks, residual estimates, iterations)."""
    import ctypes
    _check_cores(f_cores, "f")
    dims, fr = _shape_of(f_cores)
    N, T = len(dims), len(mats)
    dev = f_cores[0].device
    flat = []
    for row in mats:
        if len(row) != N:
            raise ValueError("every operator term needs N matrices (None = identity)")
        flat += [0 if M is None else M.data_ptr() for M in row]
    b = ctypes.c_size_t(0)
    L.check(L.lib().tt_gmres_workspace(N, L.i64_array(dims), T, L.i64_array(fr), int(max_rank),
                                       int(max_iter), ctypes.byref(b)))
    ws = _workspace(b.value, dev)
    out = [torch.empty((int(max_rank) ** 2 * d,), dtype=torch.float64, device=dev) for d in dims]
    xr = L.i64_array([0] * (N + 1))
    res = (ctypes.c_double * (int(max_iter) + 1))()
    it = ctypes.c_int32(0)
    L.check(L.lib().tt_gmres(
        N, L.i64_array(dims), T, L.ptr_array(flat),
        ctypes.c_void_p(precond.data_ptr() if precond is not None else 0), L.i64_array(fr),
        L.ptr_array([c.data_ptr() for c in f_cores]), _DTYPE[f_cores[0].dtype], int(max_rank),
        float(round_eps), float(tol), int(max_iter), int(seed) & ((1 << 64) - 1),
        L.ptr_array([c.data_ptr() for c in out]), xr, res, ctypes.byref(it),
        ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream)))
    ranks = [xr[i] for i in range(N + 1)]
    x = [out[n][:ranks[n] * dims[n] * ranks[n + 1]].view(ranks[n], dims[n], ranks[n + 1])
         for n in range(N)]
    return x, [res[i] for i in range(it.value + 1)], it.value


def round_rand_noalloc(cores, target_rank: int, oversample: int = 0, seed: int = 0,
                       prec: str = "f64", out=None, stream=None):
    """Randomize-then-Orthogonalize rounding through tt_round_rand_noalloc
    (workspace in the library's fixed device array, nothing allocated by
    the call).  `out`: preallocated output cores at the plan's out ranks
    (allocated here when omitted); returns them."""
    _check_cores(cores)
    if prec not in _PREC:
        raise ValueError(f"unknown prec {prec!r}")
    dims, ranks = _shape_of(cores)
    N = len(dims)
    _, out_ranks = plan(dims, ranks, target_rank, oversample)
    if out is None:
        out = [torch.empty((out_ranks[n], dims[n], out_ranks[n + 1]), dtype=cores[0].dtype,
                           device=cores[0].device) for n in range(N)]
    for n, c in enumerate(out):
        if tuple(c.shape) != (out_ranks[n], dims[n], out_ranks[n + 1]) or not c.is_contiguous():
            raise ValueError("output cores do not match the plan's out ranks")
    L.check(L.lib().tt_round_rand_noalloc(
        N, L.i64_array(dims), L.i64_array(ranks), L.ptr_array([c.data_ptr() for c in cores]),
        _DTYPE[cores[0].dtype], int(target_rank), int(oversample), int(seed) & ((1 << 64) - 1),
        _PREC[prec], L.ptr_array([c.data_ptr() for c in out]), _stream_handle(stream)))
    return out


def sum_round(summands, coeffs, target_rank: int, oversample: int = 0, seed: int = 0,
              prec: str = "f64", stream=None):
    """Rounding of sum_j coeffs[j] * summands[j] (Algorithm 7)."""
    dims, _ = _shape_of(summands[0])
    p = RoundPlan(dims, None, target_rank, oversample, prec, summands[0][0].device,
                  summand_ranks=[_shape_of(t)[1] for t in summands])
    return [c.clone() for c in p.run_sum(summands, coeffs, seed=seed, stream=stream)]


class BatchPlan:
    """Many independent roundings in lock step (tt_batch_*): one grouped
    launch per step of the method, optionally one hipGraph for the whole
    batch and autotuned GEMM tiles.  Inputs are the device cores given at
    construction (read at every run); outputs are preallocated."""

    def __init__(self, tts, targets, oversamples, seeds, prec="f32", graph=True, autotune=True,
                 stream=None):
        import ctypes
        if prec not in _PREC:
            raise ValueError(f"unknown prec {prec!r}")
        B = len(tts)
        if not (len(targets) == len(oversamples) == len(seeds) == B):
            raise ValueError("targets, oversamples and seeds need one entry per TT")
        self.prec = prec
        self.tts = [list(t) for t in tts]
        for t in self.tts:
            _check_cores(t)
            if t[0].dtype != STORAGE[prec]:
                raise ValueError(f"prec {prec!r} needs {STORAGE[prec]} cores")
        dev = self.tts[0][0].device
        orders, dims, ranks = [], [], []
        self.out = []
        for t, tr, ov in zip(self.tts, targets, oversamples):
            d, r = _shape_of(t)
            orders.append(len(d))
            dims += d
            ranks += r
            _, outr = plan(d, r, tr, ov)
            self.out.append([torch.empty((outr[n], d[n], outr[n + 1]), dtype=STORAGE[prec],
                                         device=dev) for n in range(len(d))])
        self._orders = (ctypes.c_int32 * B)(*orders)
        self._dims = L.i64_array(dims)
        self._ranks = L.i64_array(ranks)
        self._targets = L.i64_array(targets)
        self._over = L.i64_array(oversamples)
        self._seeds = (ctypes.c_uint64 * B)(*[int(s) & ((1 << 64) - 1) for s in seeds])
        b = ctypes.c_size_t(0)
        L.check(L.lib().tt_batch_workspace(B, self._orders, self._dims, self._ranks, self._targets,
                                           self._over, _PREC[prec], ctypes.byref(b)))
        self.ws_bytes = int(b.value)
        self.workspace = _workspace(self.ws_bytes, dev)
        flags = (L.TT_BATCH_GRAPH if graph else 0) | (L.TT_BATCH_AUTOTUNE if autotune else 0)
        self._cores = L.ptr_array([c.data_ptr() for t in self.tts for c in t])
        self._outp = L.ptr_array([c.data_ptr() for t in self.out for c in t])
        h = ctypes.c_void_p(0)
        L.check(L.lib().tt_batch_create(B, self._orders, self._dims, self._ranks, self._targets,
                                        self._over, self._seeds, _DTYPE[STORAGE[prec]],
                                        _PREC[prec], self._cores, self._outp,
                                        ctypes.c_void_p(self.workspace.data_ptr()),
                                        self.workspace.numel(), flags, _stream_handle(stream),
                                        ctypes.byref(h)))
        self._h = h

    def run(self, stream=None):
        L.check(L.lib().tt_batch_run(self._h, _stream_handle(stream)))
        return self.out

    def info(self):
        import ctypes
        la, gg = ctypes.c_int32(0), ctypes.c_int32(0)
        vc = (ctypes.c_int32 * 4)()
        L.check(L.lib().tt_batch_info(self._h, ctypes.byref(la), ctypes.byref(gg), vc))
        names = ("32x64", "64x32", "64x64", "128x128")
        return {"launches_per_run": la.value, "grouped_gemms": gg.value,
                "tile_variants": dict(zip(names, (vc[0], vc[1], vc[2], vc[3])))}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.lib().tt_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
