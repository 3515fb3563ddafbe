"""FP64 CPU oracle for the SSFM march of the coupled SHG equations.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call or
link this package; only tests/, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP path: the two sides have
separate beam builders, propagators, right-hand sides and reductions, and meet
only in the seeded inputs of the `workloads` module.

Contents
  ssfm     forward march, Strang split N/2 - L - N/2 with RK4 half-steps
           (Sec. 3 split-step Fourier method, Eqs. 11-15; Appendix A)
  adjoint  reverse-mode derivative of exactly that discrete march
  beams    focused Gaussian input beam (Sec. 2.1, Eqs. 5-6)
  pins     closed forms and quadratures that pin the oracle to the physics
           (Boyd-Kleinman focusing function, Eq. 17; plane-wave laws)
  thermal  steady-state heat equation (Sec. 2.2, finite differences of
           Sec. 3.2) by a sparse direct solve, the heat source of the fields,
           and the self-consistent field <-> temperature loop (Sec. 4 flowchart)
"""
from . import ssfm, beams, pins, adjoint, thermal  # noqa: F401
