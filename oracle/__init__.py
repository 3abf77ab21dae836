"""Checker: a plain, slow FP64 CPU implementation of the method (test infrastructure).

This package is test infrastructure.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it; the GPU solver path never
calls it and shares no code with it.

Contents (each function cites the passage of the paper it follows):
  fem      -- structured Q2-P1disc mesh (Q1 pressure as an option), dof
              numbering, steady monolithic ALE residual and its exact
              Jacobian (complex-step differentiation)
  transfer -- natural-injection prolongation, equation-aware restriction,
              Galerkin coarse operators
  patches  -- Schwarz patches split along the fluid/solid interface
  solver   -- dense LU, restricted additive Schwarz Richardson smoother,
              V-cycle, right-preconditioned FGMRES(m) with CGS2
  problem  -- the level hierarchy of one seeded system
"""
