"""CPU oracle for CA-BCD / CA-BDCD ridge regression.

TEST INFRASTRUCTURE ONLY.  Only `tests/`, the smoke check in
`__graft_entry__` and the CPU-baseline leg of `bench.py` may import anything
under this package.  The HIP library never imports, links or calls it, and it
imports nothing from the HIP library.

* `sampler` - the block sampler specification (SplitMix64 + Lemire + Floyd).
* `bcd`     - plain FP64 Alg. 1-4 in numpy/scipy, plus the objectives, the Gram
              definition, the closed-form ridge solution, the full residuals
              of the stopping test and the runs stopped by it.
* `exact`   - Alg. 1-4 in exact rational arithmetic for tiny inputs.
"""

from .sampler import (mix64, splitmix64_output, iteration_key, sample_block,
                      sample_blocks)
from .bcd import (NotSPDError, primal_bcd, dual_bcd, primal_objective,
                  dual_objective, ridge_closed_form, gram, primal_residual,
                  dual_residual, primal_bcd_tol, dual_bcd_tol)
