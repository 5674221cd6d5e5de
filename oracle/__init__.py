"""CPU oracle of the propagation hot path (test infrastructure only).

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may import
this package.  The GPU product path never does.
"""
from .oracle import *  # noqa: F401,F403
