"""Plain FP64 CPU oracle of C4v CTMRG (standard eigh variant and the QR variant).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this package:
only the tests, the smoke check of the entry module and the CPU-baseline leg of
the benchmark use it.  It shares no code, headers, tables or helpers with the
HIP library; it reads only the seeded inputs from ``synth.inputs``.

Every function cites the passage of arXiv:2505.00494 (Zhang, Yang, Corboz,
"Accelerating two-dimensional tensor network contractions using
QR-decompositions") that it follows.  Contractions are written as einsum /
matmul with no blocking or fusion; LAPACK (numpy.linalg) supplies eigh and QR.
"""
