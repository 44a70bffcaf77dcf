"""FP64 CPU oracle for the phaseless AFQMC walker update.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The product path (the HIP
library and its Python binding) never imports, links or calls it, and this
package imports nothing from the product path.  Its only shared dependency is
the seeded input generator ``afqmc_synth``, which holds none of the method's
arithmetic.

Everything here is plain numpy in float64 / complex128: batched matrix
products, ``np.linalg`` determinants, inverses and eigendecompositions, and
explicit loops where the algorithm is sequential.  There is no blocking,
fusion or reordering beyond the formulas cited in each function.
"""
from .afqmc import (  # noqa: F401
    Oracle,
    Options,
    WalkerState,
    philox4x64_10,
    words_to_uniform,
    gaussian_fields,
    comb_uniform,
    comb_parents,
    mgs_orthonormalize,
    taylor_apply,
    modified_cholesky,
)
from .stats import reblock, cs_difference  # noqa: F401
