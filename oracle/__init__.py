"""Plain FP64 CPU oracle for the FFT/Picard classical-DFT method of Knepley et al.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The product path (the HIP library and
its Python binding) never calls into it, and the two share no code: the oracle
follows the paper step by step in NumPy/SciPy, using library FFTs, spherical
Bessel functions, a root bracketer and a quadrature routine as its primitives.

Modules
  bulk      Appendix A: Percus-Yevick bulk hard-sphere mu and P, MSA Gamma; the
            BMCSL bulk of the White Bear functional.
  spectra   Appendix B weight spectra, the bulk-fluid kernel transform, k ordering.
  fmt       eq. (Phi): the anti-symmetrized Rosenfeld free-energy density and its
            first derivatives; Rosenfeld's original and the White Bear forms in its
            place; complex-step Hessian-vector products.
  residual  One residual evaluation G(rho): eqs. (nDef), (conv), (muHS),
            (potentialSolution), (muESexpansion), (rhoEquation).
  picard    Picard iteration with the quadratic line search and the n3 bound.
  brute     Real-space circulant convolution for tiny grids (pins the FFT path).
  adjoint   Implicit-adjoint gradient of an observable through the fixed point.
  screening RFD screening operator (ball average with a varying radius), O(N^2).

Parity-pinning status of each function is stated in its module header.
"""
