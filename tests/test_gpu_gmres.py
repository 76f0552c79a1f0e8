"""TT-GMRES (tt_gmres, section 4.2) against the oracle's tt_gmres on the same
operator, right-hand side and sketch seeds: the same number of steps, the
residual estimates within 1e-6 relative (1e-3 for those within three
orders of the rounding tolerance), and the solutions within 1e-8
(every rounding agrees with the oracle's to about 1e-14; the iteration
carries those differences along).  On a tiny problem the true residual of
the returned TT is checked against the dense operator."""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_gpu(gpu_lib, op, **kw):
    mats = [[None if M is None else dev(M) for M in row] for row in op["mats"]]
    f = [dev(c) for c in op["f"]]
    x, res, it = gpu_lib.gmres(mats, f, dev(op["precond"]), **kw)
    torch.cuda.synchronize()
    return [c.cpu().numpy() for c in x], res, it


def test_gmres_tiny_matches_oracle_and_dense(gpu_lib):
    say("TT-GMRES tiny problem")
    op = G.parametric_operator(N=3, I_space=6, I_param=4)
    x, res, it = run_gpu(gpu_lib, op, max_rank=24, round_eps=1e-14, tol=1e-10, max_iter=40,
                         seed=5)
    xo, reso, ito = O.tt_gmres(op["mats"], op["f"], op["precond"], 24, 1e-14, 1e-10, 40, seed=5)
    print(f"steps gpu {it} oracle {ito}; final residual estimate {res[-1]:.3e}")
    assert it == ito
    np.testing.assert_allclose(res, reso, rtol=1e-6, atol=1e-13)
    assert O.rel_diff(x, xo) < 1e-8
    A = O.kron_operator_dense(op["mats"], op["dims"])
    f = O.full(op["f"]).ravel()
    assert np.linalg.norm(A @ O.full(x).ravel() - f) / np.linalg.norm(f) <= 1e-9


@pytest.mark.timeout(600)
def test_gmres_workload_matches_oracle(gpu_lib):
    # N=5, 64 spatial points, 16 samples per parameter, sketch rank 60,
    # rounding 1e-9, tolerance 1e-8
    say("TT-GMRES workload")
    w = G.workload_gmres()
    op = w["op"]
    x, res, it = run_gpu(gpu_lib, op, max_rank=w["max_rank"], round_eps=w["round_eps"],
                         tol=w["tol"], max_iter=w["max_iter"], seed=w["seed"])
    xo, reso, ito = O.tt_gmres(op["mats"], op["f"], op["precond"], w["max_rank"], w["round_eps"],
                               w["tol"], w["max_iter"], seed=w["seed"])
    err = O.rel_diff(x, xo)
    print(f"steps gpu {it} oracle {ito}; residual {res[-1]:.3e}; ranks {O.ranks_of(x)}; "
          f"x rel diff {err:.3e}")
    assert it == ito
    assert res[-1] <= w["tol"]
    # residual estimates agree to 1e-6 while they are far above the rounding
    # tolerance; near it (the last steps, 1e-8 against round_eps 1e-9) the
    # roundings' own differences show in them (measured 5e-5)
    res, reso = np.array(res), np.array(reso)
    far = reso >= 1e3 * w["round_eps"]
    np.testing.assert_allclose(res[far], reso[far], rtol=1e-6)
    np.testing.assert_allclose(res, reso, rtol=1e-3)
    assert err < 1e-8
