"""CPU FP64 oracle for the Bloch-periodic Maxwell eigenvalue method of Boerm, Koehl and
Talebi, "Computing Maxwell eigenmodes with Bloch boundary conditions" (arXiv 2304.00337).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately unoptimised
reference written from the paper.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it.  The GPU library never calls it and shares
no code with it.

Modules and the paper passages they follow:
  fem          -- Section 3: Bloch edge and nodal bases, Galerkin matrices A, M, lifting L
  closed_form  -- discrete plane-wave spectrum for constant epsilon (derived from Section 3)
  dense        -- the plain definition: smallest non-zero eigenpairs of A e = lambda M e
  multigrid    -- Section 5: bisection hierarchy, Galerkin coarse matrices, node-patch
                  block Gauss-Seidel with the stabilised 4x4 solve, nodal multigrid
  householder  -- Section 4: generalized Householder factorisation in the M inner product
  pinvit       -- Section 4 and Section 7: block preconditioned inverse iteration with the
                  null-space elimination, Ritz step and throw-away vectors
  extrapolation-- Section 6: Rayleigh-quotient extrapolation across Bloch parameters
  throwaway    -- Section 7: observed convergence rates against the number of throw-away
                  vectors, and the block inverse-iteration rate lambda_i / lambda_{p+1}

Parity status of each function is stated in its docstring ("pinned by ..." or
"parity unpinned").
"""
