"""CPU FP64 oracle of the periodic higher-order finite-difference OF-DFT hot path.

TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import anything from here.  The GPU library shares no
code, headers, tables or helpers with this package, and the product path never
falls back to it.

Every function is a plain, direct statement of what the method computes,
following the paper (arXiv:1412.8250): the finite-difference Laplacian and its
weights (Section 4), the periodic Poisson problem for the electrostatic
potential (Section 3.3), the complex shifted (Helmholtz) equations of the local
kernel reformulation (Section 3.1), the exchange-correlation and Thomas-Fermi
potentials (Sections 2 and 3.3), the constrained non-linear conjugate-gradient
density update (Appendix C, Algorithm 1), Anderson mixing (Appendix D) and the
fixed-point iteration (Section 3.3).  Floating point is FP64 throughout.

Modules:
  fd        weights, exact discrete symbol, stencil apply (C)
  poisson   right-hand side, exact spectral solve, textbook CG (C)
  helmholtz exact spectral shifted solve, textbook COCG (C)
  multishift multi-shift COCG: one Krylov sequence for the shifts of one right-hand side
  xc        Thomas-Fermi and Perdew-Zunger LDA energy densities / potentials
  kernel    K_00 shifts/weights table and kernel-potential assembly
  anderson  Anderson mixing
  density   the density update U(v): Algorithm 1 with Brent line search
  scf       one fixed-point step
"""
