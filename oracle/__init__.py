"""FP64 CPU oracle for the articulated-NeRF deform-and-query path.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  It shares no
code with the HIP library; see ``oracle.c`` for the arithmetic and the paper
passage each function follows.

Parity status per function (what pins it is in ``tests/test_oracle_*.py``):
  march, skin weights / LBS, deform (root set), hash encode, MLP, composite,
  all backward passes: pinned.
  learned root initialiser forward: pinned against a float64 matmul chain.
"""
from .oracle import *  # noqa: F401,F403
