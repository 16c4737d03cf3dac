"""FP64 CPU oracle for the 3D FFT, the pseudo-spectral Navier-Stokes step and the
learned sub-grid closure.

TEST INFRASTRUCTURE.  This package is the plain, slow, obviously-correct reference
the GPU library is held to.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the GPU library never calls it and it
imports nothing from the GPU library.  It shares only the seeded input
generators (package ``synth``), which hold none of the method's arithmetic.

Modules:
  fft     3D r2c / c2r transforms (C, FP64, own mixed-radix FFT) and wavenumbers
  ns      curl, nonlinear term, 2/3 mask, projection, IF-RK2 and explicit RK steps
  diag    energy, dissipation, shell spectrum, divergence, Parseval, CFL step
  init    initial fields from the seeded noise
  mlp     closure network forward / backward / Adam in FP64
  les     spectral box filter, sub-grid stress, gradient features, LES right-hand side
"""
