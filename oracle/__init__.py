"""Sequential FP64 CPU oracle for the multifrontal factor and solve.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct definition that the HIP
path is checked against.  Only the test suite, the package smoke check and the benchmark's CPU
baseline leg may import it; the product path never calls it and has no CPU fallback.  It shares
no code with the HIP path (no kernels, headers, helpers, tables or pre/post-processing) and never
imports it.

Modules
  tree      nested-dissection elimination tree, Foata levels, pivot / contribution-block sets,
            front index lists and extend-add maps (Sec. 2.4, Table 3, Sec. 3.3)
  factor    multifrontal partial LU in the paper's division -> multiplication -> subtraction
            order (Table 2, Sec. 2.2)
  solve     forward / backward substitution over the same tree, plain and transposed
  dense     assembled global matrix, dense unpivoted LU of the permuted matrix, brute-force solve
  foata     Foata-normal-form checks of the front-level trace (Sec. 3.3)
  residual  element-by-element residual, relative residual and normwise backward error
  adjoint   gradients of a least-squares loss through the solve (dense and multifrontal)

Parity status: every function is pinned by tests against closed forms, brute force or library
routines (tests/test_oracle_*.py); none is "parity unpinned".
"""
