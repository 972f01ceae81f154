"""FP64 CPU oracle for the RI-PNOF7 hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check
(__graft_entry__.smoke) and the CPU-baseline leg of the benchmark import this
package.
The product path (the HIP library and its Python binding) never imports,
links or executes anything here, and nothing here imports the product.

Modules:
  pnof7_ri  -- the plain definition of every hot-path step, in FP64 numpy.
  brute     -- independent checks: explicit four-index integrals with the
               conventional algorithm (Table 1), a closed-shell HF route,
               and an antisymmetrised-geminal-product expectation value.
  on_opt    -- ON optimisation at fixed orbitals (gamma variables, scipy L-BFGS).
  mlp       -- the warm-start network: features, forward, backward, Adam.
  orbital   -- orbital optimisation by iterative diagonalisation of F^lambda
               and the outer/inner loop of Fig. 1.
  metric    -- b from the three-centre integrals and the metric: pivoted
               symmetric factorisation, block eigenvalue correction, solve.
"""
from . import pnof7_ri, brute  # noqa: F401
