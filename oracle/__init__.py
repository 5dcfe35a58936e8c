"""Plain FP64 CPU oracle for the star-M truncated tensor SVD.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check of the package entry
file and the CPU-baseline leg of the benchmark use it.  It shares no code
with the HIP path (no kernels, headers, helpers or constant tables).

Every function follows one passage of the paper (Hussain et al., "High-
Performance star-M SVD for Big Data Compression"):

* mode-k product and the star-M product ......... Section 2.1
* full t-SVDM ................................... Section 2.2, Algorithm 1
* t-SVDM-II rank selection ...................... Section 2.2, Algorithm 2
* t-SVDM-I (uniform rank) ....................... Section 3.3
* Eckart-Young optimality for orthogonal M ...... Section 2.3
* compression accounting (inferred) ............. Section 4 (printed ratios)
* adjoint of the truncation loss ................ not in the paper (derived)

Parity status of each function is listed in the module docstring of
`oracle.tsvdm` and pinned by the CPU tests.
"""
from .tsvdm import *  # noqa: F401,F403
from .tsvdm import __all__  # noqa: F401
