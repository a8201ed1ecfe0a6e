"""CPU FP64 oracle for the kernel-compensated Yee-scheme Maxwell eigenproblem.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package: only the tests, the smoke check of the package entry point and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP path;
both take their inputs from the `workloads` module, which holds no arithmetic of
the method.

Contents
--------
yee       explicit sparse matrices of Section 2.1 and Section 3: the circulant
          difference/average matrices D1, D0 (eq (2.5)), the blocks D_i
          (eq (2.6)), the curl A and divergence B (eq (2.7)), the
          inverse-permittivity matrices (eqs (3.3), (3.4), (3.8)), the penalty
          rule (eq (2.26)) and the compensated operator A M A^H + gamma B^H B
          (eq (2.13)).
kspace    the same operator expressed on k-space coefficients x = F3^H H
          (Prop 2.8, eq (2.30)) by conjugating the sparse operator with the
          unitary DFT, the diagonal-block preconditioner (eqs (2.31)-(2.32)), the
          transverse-projection preconditioner from its pseudo-inverse definition
          (not part of the paper: Johnson & Joannopoulos 2001) and a direct DFT
          by its definition (Lemma 2.1).
eigs      smallest strictly positive eigenvalues of the compensated operator
          (dense LAPACK for small n, shift-invert ARPACK otherwise), with the
          k = 0 constant-field null space removed (Prop 2.5).
nn        direct-summation 3D convolution with circular padding and its
          gradients (learned preconditioner), in FP64.
train     the training quantities of the learned preconditioner (not part of the
          paper): perturbed iterates and their residuals, exact corrections by a
          sparse direct solve, the scale-free misfit from its definition.
block     the dense block steps of the LOBPCG iteration (Section 4): Gram matrices of
          the search space and the Rayleigh-Ritz update with the residuals of
          eq (4.3), from their definitions.

Parity unpinned: none of the functions above is unpinned; the pins are listed
in the test modules tests/test_oracle_*.py.
"""
