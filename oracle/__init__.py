"""CPU FP64 oracle for blocked randomized QR with column pivoting.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the GPU library; only seeded input matrices are common to both.
"""
from . import philox, rqrcp  # noqa: F401
