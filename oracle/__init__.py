"""CPU FP64 oracle for the randomized truncated SVD (rSVD).

TEST INFRASTRUCTURE ONLY. This package is the plain, slow, obviously correct
reference that the HIP path is checked against. Only the test suite, the
smoke check of the build entry module and the ``cpu_baseline`` leg of the
benchmark may import it. The product library never calls into it, and it
shares no code with the HIP path (no kernels, headers, helpers or tables).

What it computes follows the section "Randomized matrix decompositions" of
arXiv:2307.15572 (Tichai et al.), which applies Halko et al.'s randomized
SVD: a random projection Z = V P, an orthonormal basis Q of Z from a QR
decomposition, the projection Y = Q^T V, a thin SVD Y = L_Y Sigma R^T and the
lift L = Q L_Y (Fig. 1, steps 1-3; Eq. 1), with oversampling p = l - R_SVD,
truncation to the rank R_SVD, the relative rank R% and the compression ratio
of Eq. 2.

Additions beyond the paper, each stated where it is implemented:
  * q power (subspace) iterations with a QR after every product with A or
    A^T (Halko et al., randomized subspace iteration). q = 0 is exactly the
    paper's method.
  * A counter-based Gaussian test matrix (Philox4x64-10 + Box-Muller), so the
    GPU path can draw the same random projection independently.
  * Rank rules by relative threshold and by Frobenius tail, the adaptive
    range finder and the a-posteriori error estimate, and a small MLP that
    predicts (rank, oversampling, q).
  * The symmetric-channel form A ~ Q (Q^T A Q) Q^T (symmetric.py), the basis
    transform on thin factors and the report of one decomposition truncated
    at several R% (transform.py).

Parity status per function is listed in each module's header.
"""

from .philox import philox4x64_10, gaussian_omega, box_muller  # noqa: F401
from .method import (  # noqa: F401
    RsvdResult,
    orth,
    rsvd,
    select_rank,
    residual,
    compression_eq2,
    compression_sym,
    relative_rank_percent,
    sign_normalize,
)
from .adaptive import rsvd_adaptive, FLAG_ADAPT_LIMIT, POSTERIOR_FACTOR  # noqa: F401
from . import mlp  # noqa: F401
from .symmetric import rsvd_sym  # noqa: F401
from .transform import factor_transform, truncation_report  # noqa: F401
