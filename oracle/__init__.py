"""FP64 CPU oracle for the nodal DG Euler hot path -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, deliberately unoptimized restatement of the
method, used only by the tests, by the smoke check and by the CPU-baseline
leg of the benchmark.  The product path (the HIP library and its Python
binding) never imports it and shares no code with it.

What it computes, and from where:

* physics: the compressible Euler system and the ideal-gas law (Section 2.1,
  Eqs. 1-2; the flux is the standard one, with pressure only on the diagonal
  momentum entries), the rest state and pass-through ghost (Section 2.2,
  Eq. 3), the reflective wall (Section 2.3, Eq. 4, applied as a mirror about
  the face normal), the mouthpiece inflow (Section 2.4, pulse p1 and
  Eqs. 5-7);
* discretization: the Galerkin weak form on each tetrahedron (Appendix A,
  Eqs. 8-12) in nodal, strong form, with the local Lax-Friedrichs numerical
  flux (Section 1.1) and a five-stage fourth-order low-storage Runge-Kutta
  integrator for the ODE system dc/dt = f(c) (Appendix A, Eq. 12).

Operators are built from monomials with exact rational integrals, which is a
different route from the orthonormal-basis construction used by the library.

Functions without an independent pin say "parity unpinned" in their docstring.
"""
from . import nodes, operators, mesh, euler, timestep, norms  # noqa: F401
# (probes, mlp and quadrature are imported by name where used)
