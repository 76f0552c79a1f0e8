"""FP64 CPU oracle for randomized TT-rounding -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
import this package.  It shares no code with the HIP library.
"""
from .tt_oracle import *  # noqa: F401,F403
