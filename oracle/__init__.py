"""FP64 CPU oracle for the detection hot path -- test infrastructure only.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package; the product path never does.
"""
from .pd_oracle import *  # noqa: F401,F403
from . import pd_oracle  # noqa: F401
