"""CPU FP64 oracle for the spin-1 Bogoliubov-de Gennes (BdG) excitation problem.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the GPU library is checked against.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import it; the GPU library never
imports, links or calls it, and it never calls the GPU library.  It shares no
code with the GPU path: its only inputs are the seeded arrays of ``workloads``.

Everything is numpy / scipy in float64 / complex128 and follows the paper
(Li, Li, Xie, Zhang, "An efficient Fourier spectral algorithm for the
Bogoliubov-de Gennes excitation eigenvalue problem", arXiv 2506.08308):

  spectral   grid, wavenumbers and the Fourier pseudo-spectral Laplacian (Section 3.1)
  spin       spin-1 matrices, spin vector, GPE right-hand sides, energy (Section 1)
  groundstate projected, preconditioned normalized gradient flow for the ground state
             (Euler-Lagrange problem of Section 1)
  bdg        operators A, B and the BdG / linear-response forms (Sections 2.1, 3.1)
  branch     exact scalar branch decompositions and the uniform-state dispersion
             (Section 2.3 structure, derived closed forms)
  lrep       block subspace iteration with bi-orthogonal Gram-Schmidt and
             Rayleigh-Ritz projection (Section 3.2)
  grad       Hellmann-Feynman gradients with the ground-state sensitivity

Parity status of each function is stated in its module header; a function
without an independent pin says "parity unpinned".
"""
from . import spectral, spin, groundstate, bdg, branch, lrep, grad, kohn, modes, complexgs  # noqa: F401
