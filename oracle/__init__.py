"""CPU FP64 oracle for TR-ALS (Yu & Li, "Practical Alternating Least Squares
for Tensor Ring Decomposition", arXiv 2210.11362).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` use it.  It shares no code with the HIP path
and imports nothing from it; its only shared dependency is the seeded input
generator package ``workloads`` (random draws, no ALS arithmetic).

Every routine follows the paper's definitions in plain numpy/LAPACK FP64 with
no blocking or fusion.  Functions are pinned by the ``-m "not gpu"`` tests
against brute force, closed forms and textbook reductions.  Parity status of
each function is listed in ``oracle/tr_oracle.py``'s header.
"""
from .tr_oracle import *  # noqa: F401,F403
