"""MI355X (gfx950) implementation of the non-equilibrium Monte Carlo estimator
of Renyi-entropy increments (Bulgarelli & Panero, arXiv:2304.03311).

Submodules:
  ee        -- ctypes binding of the C ABI (include/ee.h) and the Job owner
  build     -- in-tree hipcc build of libee.so
  workloads -- seeded synthetic job sets of the benchmark configurations
  analysis  -- host assembly of S_2(l) and the entropic c-function
"""
__all__ = ["ee", "build", "workloads", "analysis"]
