"""Host-only checks of the C ABI: the library loads, exports every function
include/tt_round.h declares, plans ranks like the oracle and rejects bad
arguments before touching the GPU."""
import ctypes
import random

import pytest

import oracle as O
import paper_2110_04393_amd as tt
from paper_2110_04393_amd import _lib as L


def test_library_exports_every_header_function():
    lib = tt.lib()
    names = tt.header_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert tt.version() >= 100


def test_plan_matches_oracle():
    rng = random.Random(0)
    for _ in range(200):
        N = rng.randint(1, 9)
        dims = [rng.randint(1, 7) for _ in range(N)]
        ranks = [1] + [rng.randint(1, 12) for _ in range(N - 1)] + [1]
        t, p = rng.randint(1, 10), rng.randint(0, 6)
        assert tt.plan(dims, ranks, t, p) == tuple(O.plan_ranks(dims, ranks, t, p))


def test_workspace_queries_positive():
    assert tt.round_rand_workspace([100] * 30, [1] + [200] * 29 + [1], 50, 10) > 0
    assert tt.sum_round_workspace([128] * 16, [[1] + [20] * 15 + [1]] * 20, 60, 10) > 0


@pytest.mark.parametrize("dims,ranks,t,p", [
    ([3, 3], [1, 2, 2], 1, 0),        # last rank != 1
    ([3, 0, 3], [1, 2, 2, 1], 1, 0),  # zero mode size
    ([3, 3], [1, 2, 1], 0, 0),        # target < 1
    ([3, 3], [1, 2, 1], 1, -1),       # oversample < 0
])
def test_plan_rejects_bad_arguments(dims, ranks, t, p):
    with pytest.raises(tt.TTError) as e:
        tt.plan(dims, ranks, t, p)
    assert e.value.status == L.TT_EINVAL
    assert len(str(e.value)) > 10


def test_unsupported_sketch_rank():
    with pytest.raises(tt.TTError) as e:
        tt.round_rand_workspace([100] * 5, [1, 200, 200, 200, 200, 1], 150, 10)
    assert e.value.status == L.TT_EUNSUPPORTED


def _call_round(ws_bytes, dtype=L.TT_F64, prec=L.TT_PREC_F64, target=2):
    # fake (never dereferenced) device pointers: validation fails before any launch
    N = 3
    dims, ranks = [4, 4, 4], [1, 3, 3, 1]
    fake = [0x1000 * (i + 1) for i in range(N)]
    outs = [0x9000 * (i + 1) for i in range(N)]
    st = L.lib().tt_round_rand(N, L.i64_array(dims), L.i64_array(ranks), L.ptr_array(fake),
                               dtype, target, 0, 7, prec, L.ptr_array(outs),
                               ctypes.c_void_p(0x100000), ws_bytes, None)
    return st, L.lib().tt_last_error().decode()


def test_round_rejects_small_workspace_before_launch():
    st, msg = _call_round(0)
    assert st == L.TT_ENOMEM and "workspace" in msg


def test_round_rejects_unknown_precision():
    st, msg = _call_round(1 << 30, prec=7)
    assert st == L.TT_EINVAL


def test_round_rejects_null_cores():
    N = 2
    st = L.lib().tt_round_rand(N, L.i64_array([3, 3]), L.i64_array([1, 2, 1]), None, 0, 1, 0, 0,
                               0, L.ptr_array([1, 2]), None, 0, None)
    assert st == L.TT_EINVAL


def test_sketch_rejects_bad_shape():
    st = L.lib().tt_make_sketch(1, 2, L.i64_array([3, 3]), L.i64_array([1, 2, 2]), 0,
                                L.ptr_array([1, 2]), None)
    assert st == L.TT_EINVAL


def test_round_svd_plan_bounds_oracle_ranks():
    import oracle as O
    import tt_inputs as G
    for dims, ranks, k in [([5, 6, 4, 5, 3, 4], [1, 5, 8, 8, 6, 4, 1], 4),
                           ([3, 4, 5, 3], [1, 3, 8, 6, 1], 0),
                           ([7, 9], [1, 7, 1], 2)]:
        N = len(dims)
        out = L.i64_array([0] * (N + 1))
        L.check(L.lib().tt_round_svd_plan(N, L.i64_array(dims), L.i64_array(ranks), k, out))
        bound = [out[i] for i in range(N + 1)]
        Y = G.random_tt(3, dims, ranks)
        _, rr, _ = O.round_svd(Y, 0.0, k if k > 0 else None)
        assert bound[0] == bound[N] == 1
        assert all(r <= b for r, b in zip(rr, bound)), (rr, bound)
        if k > 0:
            assert rr == bound  # fixed rank: the bound is attained


def test_round_svd_rejects_bad_arguments():
    dims, ranks = [4, 4, 4], [1, 2, 2, 1]
    ptrs = L.ptr_array([1, 1, 1])
    outr = L.i64_array([0] * 4)
    lib = L.lib()
    st = lib.tt_round_svd(3, L.i64_array(dims), L.i64_array(ranks), ptrs, L.TT_F64, -1.0, 0,
                          L.TT_PREC_F64, ptrs, outr, None, 0, None)
    assert st == L.TT_EINVAL
    st = lib.tt_round_svd(3, L.i64_array(dims), L.i64_array(ranks), ptrs, L.TT_F32, 0.0, 0,
                          L.TT_PREC_F64, ptrs, outr, None, 0, None)
    assert st == L.TT_EINVAL
    b = L.c_size(0)
    import ctypes
    st = lib.tt_round_svd_workspace(3, L.i64_array(dims), L.i64_array(ranks), 0,
                                    L.TT_PREC_MIXED_BF16, ctypes.byref(b))
    assert st == L.TT_EUNSUPPORTED
    # a bond wider than the small-panel limit
    st = lib.tt_round_svd_workspace(3, L.i64_array([200, 200, 200]),
                                    L.i64_array([1, 150, 150, 1]), 0, L.TT_PREC_F64,
                                    ctypes.byref(b))
    assert st == L.TT_EUNSUPPORTED


def test_two_sided_plan_matches_oracle():
    rng = random.Random(7)
    for _ in range(200):
        N = rng.randint(2, 7)
        dims = [rng.randint(1, 12) for _ in range(N)]
        ranks = [1] + [rng.randint(1, 30) for _ in range(N - 1)] + [1]
        t = rng.randint(1, 40)
        assert tt.two_sided_plan(dims, ranks, t) == tuple(O.plan_two_sided_ranks(dims, ranks, t))


def test_two_sided_workspace_and_limits():
    b = ctypes.c_size_t(0)
    dims, ranks = [100] * 4, [1, 200, 200, 200, 1]
    L.check(L.lib().tt_round_two_sided_workspace(4, L.i64_array(dims), L.i64_array(ranks), 60,
                                                 ctypes.byref(b)))
    assert b.value > 0
    # target 70 gives rho = 105 > 96
    rc = L.lib().tt_round_two_sided_workspace(4, L.i64_array(dims), L.i64_array(ranks), 70,
                                              ctypes.byref(b))
    assert rc == -5
    rc = L.lib().tt_round_two_sided(4, L.i64_array(dims), L.i64_array(ranks),
                                    L.ptr_array([1, 2, 3, 4]), 1, 60, 0, 1,
                                    L.ptr_array([5, 6, 7, 8]), None, 0, None)
    assert rc == -5  # FP32 cores are refused before any launch


def test_orth_rand_plan_and_workspace():
    # ranks after Algorithm 1 (the last bond drops to I_N = 7), then the
    # plan of tt_round_rand on them; the queries run without a GPU
    dims, ranks = [9, 8, 7], [1, 9, 12, 1]
    rr = [1, 9, 7, 1]
    assert tt.orth_rand_plan(dims, ranks, 4, 2) == tuple(O.plan_ranks(dims, rr, 4, 2))
    for prec in (L.TT_PREC_F64, L.TT_PREC_F32):
        b = ctypes.c_size_t(0)
        L.check(L.lib().tt_round_orth_rand_workspace(3, L.i64_array(dims), L.i64_array(ranks), 4,
                                                     2, prec, ctypes.byref(b)))
        assert b.value > 0
    b = ctypes.c_size_t(0)
    st = L.lib().tt_round_orth_rand_workspace(3, L.i64_array(dims), L.i64_array(ranks), 4, 2,
                                              L.TT_PREC_MIXED_BF16, ctypes.byref(b))
    assert st == L.TT_EUNSUPPORTED


def test_eps_workspace_queries():
    for prec in (L.TT_PREC_F64, L.TT_PREC_F32):
        b = ctypes.c_size_t(0)
        L.check(L.lib().tt_round_rand_eps_workspace(30, L.i64_array([100] * 30),
                                                    L.i64_array([1] + [200] * 29 + [1]), 60, prec,
                                                    ctypes.byref(b)))
        fixed = tt.round_rand_workspace([100] * 30, [1] + [200] * 29 + [1], 60, 0,
                                        "f64" if prec == L.TT_PREC_F64 else "f32")
        assert b.value >= fixed > 0
        L.check(L.lib().tt_sum_round_eps_workspace(2, 4, L.i64_array([5] * 4),
                                                   L.i64_array([1, 3, 3, 3, 1] * 2), 5, prec,
                                                   ctypes.byref(b)))
        assert b.value > 0


def test_gmres_workspace_and_argument_checks():
    dims = [64, 16, 16, 16, 16]
    b = ctypes.c_size_t(0)
    L.check(L.lib().tt_gmres_workspace(5, L.i64_array(dims), 5, L.i64_array([1] * 6), 60, 40,
                                       ctypes.byref(b)))
    assert b.value > 0
    # max_iter beyond the limit and max_rank beyond the sketch-rank limit
    assert L.lib().tt_gmres_workspace(5, L.i64_array(dims), 5, L.i64_array([1] * 6), 60, 64,
                                      ctypes.byref(b)) == L.TT_EUNSUPPORTED
    assert L.lib().tt_gmres_workspace(5, L.i64_array(dims), 5, L.i64_array([1] * 6), 200, 10,
                                      ctypes.byref(b)) == L.TT_EUNSUPPORTED
