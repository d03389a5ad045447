"""Independent plain FP64 CPU oracle for the SBP-SAT overset right-hand side and
the multi-rate Adams-Bashforth integrator.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import or run anything in this package.  It
shares no code with the GPU product path (no kernels, headers, tables, helpers,
pre- or post-processing); the only common input is the seeded problem
description from the ``workloads`` package, which holds none of the method's
arithmetic.

Parts and the paper passages they follow:
  sbp.py        SBP first-derivative operators (section "The Compressible
                Navier-Stokes Equations on Overset Meshes"; Appendix on the
                spatial order of accuracy)
  coeffs.py     AB coefficients, eq. (vandermonde) and eq. (ext_ab)
  overset.py    blanking, runs, receivers, donor search, Lagrange weights
                (section "SAT-Based Interpolation")
  orc.c         right-hand side, SAT penalty eq. (int), donor data, metrics,
                timestep eq. (ts_inv)-(ts_overall)
  integrate.py  RK bootstrap, SRAB, MRAB Steps 1-7 (section "Multi-rate
                Adams-Bashforth Integration")
  system.py     ties the parts together for one overset problem

Parity-unpinned parts (pinned only by GPU == oracle, freestream and the
spectrum sign test): the exact isothermal-wall and far-field SAT forms, which
the paper takes from references it does not reproduce.
"""
from .system import OracleSystem, load_library  # noqa: F401
