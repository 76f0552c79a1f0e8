"""Randomized TT-rounding on MI355X (gfx950): HIP kernels behind a C ABI.

Import the binding with ``import paper_2110_04393_amd as tt``; it needs the
built ``libttround.so`` (``python -m paper_2110_04393_amd.build``).
"""
from ._lib import TTError, header_functions, lib  # noqa: F401
from .api import (STORAGE, BatchPlan, RoundPlan, TwoSidedPlan, gmres, make_sketch,  # noqa: F401
                  orth_rand_plan, partial_contractions_rl, plan, round_orth_rand, round_rand,
                  round_rand_eps,
                  round_rand_noalloc, round_rand_workspace, round_svd, sum_round_eps,
                  round_two_sided, sum_round, sum_round_workspace, two_sided_plan, version)
from .autograd import round_rand_ad, round_rand_backward  # noqa: F401,E402
