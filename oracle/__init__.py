"""Plain FP64 CPU oracle for the variational Stokes step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product path
(the HIP library and its Python binding) never imports, links or calls it,
and this package never imports the product.  The two share no code: the
only common module is ``cases`` (seeded input generators, no arithmetic of
the method).

What it computes (paper: "A Simple Finite Difference Method for
Time-Dependent, Variable Coefficient Stokes Flow on Irregular Domains"):

  grid.py       staggered MAC layout with stresses (Section 5, Figs. 1-2)
  fractions.py  volume fractions W_L, W_F of the sample control volumes
                (Section 5, Figs. 3-4) by an exact simplex integrator
  operators.py  centred difference operators G and D (Section 5)
  system.py     body force, coefficients, null-space elimination (Section 8
                "Null Space Elimination"), the SPD (stress, pressure) system
                and its right-hand side (eq. stokesmixedsystemspd and the
                prescribed-velocity terms of Section 6), direct and CG
                solves, velocity recovery, and the full (u, tau, p) KKT
                system (eq. stokesmixedsystem) for cross-checks; the
                prescribed-traction terms of Section 6.1
  cg.py         plain Jacobi-preconditioned CG (the CPU timing baseline)
  advect.py     the fractional step of Section 10: semi-Lagrangian velocity
                and level-set advection around the Stokes step
  schwarz.py    brick-local additive Schwarz / block symmetric Gauss-Seidel
                preconditioners and textbook PCG with them
  learned.py    the learned preconditioner's network, loss and flexible CG

Every function is FP64 and unoptimised on purpose.
"""
from . import grid, fractions, operators, system, cg, advect, schwarz  # noqa: F401
