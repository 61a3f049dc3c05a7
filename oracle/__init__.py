"""CPU oracle for approximate selected inversion — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct float64 implementations of every step the GPU
library computes, written from the paper (Sections 2.1-2.6) and independent of
the GPU path: the two share no code, headers, tables or helpers. Only the
tests, the smoke check and the CPU-baseline leg of the benchmark may import
this package; the product path never does.

Modules:
  core        ctypes front end of csrc/oracle.c: pattern S, SelInv (with a
              NaN-sentinel mode), NInv on S and on its own pattern, Mix, SPAI,
              rank-k correction on S; the diagonal, err_1 and trace sums; the
              dominant eigenpairs of E = A^-1 - X (error_eigenpairs) and the
              per-mode acceptance test of Algorithm 1 (accept_modes); the
              factor solve and products the eigen step applies; the DAG levels
              and a per-block check of the SelInv recursion
  dense       dense numpy references for tiny inputs (masked Takahashi
              recursion, Neumann series, SPAI) and a dense threshold ILDL with
              Bunch-Kaufman pivots that pins the host factorization; the
              numeric phase of the factorization on a given pattern and
              pivot sequence (masked Crout recurrence)
  mlp         float64 forward/backward of the learned per-entry correction
              with bf16 quantisation points, and the feature definitions
"""
from . import core  # noqa: F401
