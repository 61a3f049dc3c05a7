"""CPU oracle for approximate selected inversion — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct float64 implementations of every step the GPU
library computes, written from the paper (Sections 2.1-2.6) and independent of
the GPU path: the two share no code, headers, tables or helpers. Only the
tests, the smoke check and the CPU-baseline leg of the benchmark may import
this package; the product path never does.

Modules:
  core        ctypes front end of csrc/oracle.c: pattern S, SelInv, NInv, Mix,
              SPAI, rank-k correction on S; diagonal and err_1 helpers
  dense       dense numpy references for tiny inputs (masked Takahashi
              recursion, Neumann series, SPAI) and a dense threshold ILDL with
              Bunch-Kaufman pivots that pins the host factorization; the
              numeric phase of the factorization on a given pattern and
              pivot sequence (masked Crout recurrence)
  spectral    dominant eigenpairs of E_inv = A^-1 - A^inv and the acceptance
              test of Algorithm 1
  mlp         float64 forward/backward of the learned per-entry correction
              with bf16 quantisation points, and the feature definitions
"""
from . import core  # noqa: F401
