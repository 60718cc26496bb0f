"""CPU FP64 oracle for the BRAS mass-inverse approximation inside PCG.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package: only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library (no kernels, headers, tables or helpers) and never imports it.

Everything here is written from the paper ("Broken-space Additive Schwarz
Mass Inverse Approximations and (Block) Preconditioning", Krzysik, Southworth,
Wimmer), in plain, slow, obviously checkable NumPy/SciPy in float64:

  mesh      structured simplicial meshes on the unit square / cube and the
            counter-based SplitMix64 vertex jitter (Section 3 uses simplicial
            meshes of the unit square and cube).
  poly      polynomials on reference simplices with exact monomial integrals.
  fe        reference elements: Lagrange (GLL "spectral" variant), first-kind
            Nedelec (N1curl) and Raviart-Thomas (RT), their reference mass
            matrices (Section 2.4, eq. piola_mass_pullbacks).
  dofmap    entity numbering, the broken-to-conforming map pi, the
            multiplicities d_i (Section 2.2 and Fig. P_example).
  assembly  element mass matrices, the assembled M = P^T M_br P
            (eq. M_PMbrP), diag(M), and the explicitly assembled BRAS matrix
            D^-1 (sum_K P_K^T M_K^-1 P_K) D^-1 (eqs. mhatinvbras_def and
            mass_and_bras_element_sums).
  pcg       textbook preconditioned conjugate gradients with the paper's
            stopping rule (Section 3).
  stationary damped fixed point, Chebyshev iteration and the power iteration
            for lambda_max (Section 3).
  spectral  dense eigen-checks used as pins: kappa-hat (eq. spectral-kappa),
            Lemma bras_exact_inverse_correction, Cor. bras_lambda_min,
            Thm. bras_lambda_max_projector, Cor. bras_piola_metric_contrast.
  gradient  adjoint gradient of 0.5||M(rho)^-1 b - x*||^2 and finite
            differences by difference solves.
  reduced   emulation of FP32 / BF16 rounding of stored inverses.

Functions whose result has no independent pin say "parity unpinned" in their
docstring.
"""
