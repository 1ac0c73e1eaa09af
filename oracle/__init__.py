"""FP64 CPU oracle for the 2-D TE domain-integral-equation solver.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path
(the HIP library and its Python binding) never calls into it and shares no
code with it: not the Green tensor, not the lag table, not the FFT, not the
Krylov method.  Inputs come from the separate ``synth`` generators.

Contents (each function cites the passage of Zouros & Budko it follows):

* ``operator``   -- the collocation/midpoint matrix of the E-block of the TE
                    system (Section 4, eq. A11 and the element formulas after it),
                    written element by element; a direct O(N^2) product; dense
                    assembly; LU solves; the regularizer A(chi') (Section 3,
                    eqs. InverseSymbol / Regularization).
* ``spectral``   -- the homogeneous-object eigenvalue map (Section 5,
                    eqs. EigenvaluesA .. EigenvaluesArA), the lossless segment
                    image, the essential-spectrum segment (eq. EssentialSpectrum),
                    dense-eigenvector deflation (Section 4, eq.
                    DeflatingPrecondtioner).
* ``systems``    -- the TM operator (Section 2 eq. MatrixSolutionTM, Section 4's [A33]
                    formulas with chi_e) and the full three-component TE system
                    (E1, E2, H3) with magnetic contrast (Section 4 eq. lin_system; the
                    coupling blocks from Section 3's compact kernels K13..K33).
* ``planning``   -- Section 5's deflation radius (the mapped segments [1, eps(x)]) and
                    its memory planner with the fair-memory rule.
* ``mie``        -- textbook Bessel/Hankel series of the TE (H-polarised) plane
                    wave on a homogeneous circular cylinder; the paper only names
                    it as its accuracy reference (Section 4, grid rule).
* ``unet``       -- the learned warm start (not in the paper): the U-Net that
                    proposes GMRES initial guesses, its loss gradient and the Adam
                    update, in plain PyTorch CPU float64 with the library's
                    bfloat16 rounding points.

Every function is pinned by CPU tests against something other than itself
(finite differences, quadrature, closed forms, brute force, exact invariants).
"""
