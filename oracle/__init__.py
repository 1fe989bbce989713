"""CPU oracle for the convolution-quadrature (CQ) Fokker-Planck solver.

TEST INFRASTRUCTURE ONLY. Plain, slow, fp64 numpy/scipy code written from the
paper (Sun, Nie & Deng, "Fast algorithms for convolution quadrature of
Riemann-Liouville fractional derivative"). Only the tests, the smoke check and
the benchmark's CPU-baseline leg may import it; the product path
(paper_1901_05128_amd) never does, and shares no code with it.

Modules
  weights      CQ weights: Taylor coefficients of the BE and BDF2 generating
               functions (eqs. 3.3-3.4 and 3.11-3.12).
  quadrature   Gauss-Jacobi rules and the fast sum-of-geometric-sequences
               weight approximations (eqs. 3.6, 3.14-3.16, real-part remark).
  grid         Finite-difference Dirichlet Laplacian A_h = -Delta_h.
  stepper      Direct BE (4.1) and BDF2 (4.7) schemes, fast BE (4.3) and fast
               BDF2 (4.8) schemes, all on the nodal grid.
  modal        The same schemes for one Laplacian eigenmode (2x2 recurrences),
               used to check full-size GPU runs mode by mode.
  mittag_leffler  E_alpha(-x) from its spectral integral, for closed-form pins.
  adjoint      Gradient of a loss of G^N with respect to G^0, alpha_1, alpha_2
               and m: the discrete adjoint of the schemes above (an extension,
               not in the paper).
"""
