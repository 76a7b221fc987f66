"""CPU oracle for the all-pairs CCM hot path -- test infrastructure only.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg may
import this package.  The GPU library never does.
"""
from .ccm_oracle import *  # noqa: F401,F403
from . import ccm_oracle  # noqa: F401
