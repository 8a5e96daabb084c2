"""Plain CPU FP64 oracle of fast randomized PCA for sparse data (Alg. 2, 5, 6), of the
basic randomized PCA it accelerates (Alg. 1, 4) and of eigSVDs (Alg. 3).

TEST INFRASTRUCTURE. This package is the slow, obviously-correct reference that the GPU
path is checked against. Only the tests, the smoke check and the benchmark's CPU-baseline
leg may import it; the product path never calls it, and it shares no code with the HIP
library (it reads the same seeded synthetic inputs only).

Pins (tests that tie each function to the paper or to mathematics, not to itself) live in
tests/test_oracle_*.py. Every function here is pinned; none is "parity unpinned".
"""
from .adjoint import svd_adjoint_values  # noqa: F401
from .eigsvds import eigsvds  # noqa: F401
from .frpca import check_args, frpca, pass_schedule, products, randomized_svd, sign_convention  # noqa: F401
from .linalg import eig_asc, eigsvd, lu_pl  # noqa: F401
from .rpca import rpca  # noqa: F401
from .philox import gaussian, philox4x32_10, uint32_stream  # noqa: F401
from .sparse import csc_mirror, csr_matmul, csr_tmatmul, transpose  # noqa: F401
