"""CPU FP64 oracle for preconditioned orbital minimization (test infrastructure).

This package is test infrastructure.  Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import, call or execute anything here.
The GPU library never imports it and shares no code with it; the only module
both sides use is the seeded input generator, which holds none of the method's
arithmetic.

Modules follow the paper (Lu & Yang, "Preconditioning orbital minimization
method for planewave discretization"):
  hamiltonian  Section 4.1 discretization: dense H, FFT apply, spectra.
  omm          Section 2.1: E_omm (eq. omm), gradient, Hessian, Algorithm 1 with
               an exact quartic line search.
  poles        Section 3.1, eq. (dFOP): pole expansion of the Fermi projector.
  gmres        Section 3.1, eq. (lst): restarted GMRES rough solves.
  precond      Section 3.1-3.2: Fermi-pole preconditioner with the shifted-
               Laplacian inner preconditioner.
  metrics      Section 4 (distance d) and subspace angle.

Every function works in float64 / complex128.
"""
