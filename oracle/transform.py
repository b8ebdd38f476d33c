"""Basis transformation of a decomposed channel matrix on its thin factors,
and the report of one decomposition truncated at several ranks, FP64 CPU
oracle.

TEST INFRASTRUCTURE ONLY (see the package header).

factor_transform: section "Low-rank interactions" of arXiv:2307.15572 notes
that a basis change mediated by a unitary U, Vbar = U^dagger V U, can act on
the thin factors of V = L Sigma R^T alone. For real U (U^dagger = U^T):

    Vbar = U^T L Sigma R^T U = (U^T L) Sigma (U^T R)^T,

so Lbar = U^T L and Rbar = U^T R, two products of U^T with N x k factors
instead of two N x N x N products. When U has orthonormal columns (N x N',
N' <= N; square U is the unitary case), Lbar and Rbar keep orthonormal
columns and Sigma is unchanged: the result is again an SVD.

truncation_report: the results of the paper are swept over the relative rank
R% (sections "Randomized matrix decompositions" and "Medium-mass nuclei");
one decomposition computed at the largest R% serves every smaller one by
keeping its leading R_SVD = ceil(R% N / 100) triplets. For each: the residual
||V - L_k Sigma_k R_k^T||_F / ||V||_F, R% and the compression ratios of Eq. 2
(as printed, and with one stored factor).

Library primitive: numpy's matrix product.

Pins (tests/test_oracle_transform.py): the factor form equals U^T (L Sigma
R^T) U computed densely for a non-symmetric U; orthonormal columns and
Sigma preserved; identity and permutation matrices; the truncation report
against Pythagoras (residual^2 = 1 - sum_{j<=k} s_j^2 / ||V||_F^2 for an
exact SVD) and Eq. 2's printed values.
"""

import numpy as np

from .method import compression_eq2, compression_sym, percent_rank, relative_rank_percent, residual


def factor_transform(Ub, L, R=None):
    """(U^T L, U^T R) for U (N x N'), L and R (N x k); R may be None."""
    Ub = np.asarray(Ub, dtype=np.float64)
    Lb = Ub.T @ np.asarray(L, dtype=np.float64)
    Rb = None if R is None else Ub.T @ np.asarray(R, dtype=np.float64)
    return Lb, Rb


def truncation_report(A, U, s, V, percents):
    """For each R% in percents: k = ceil(R% min(m, n) / 100) (at most len(s)),
    the residual of the leading k triplets, R% = 100 k / min(m, n) and both
    compression ratios. Returns a list of dicts."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    out = []
    for pct in percents:
        k = min(percent_rank(pct, m, n), len(s))
        e = residual(A, U[:, :k], s[:k], V[:, :k])
        out.append({"percent": float(pct), "rank": k, "residual": e,
                    "rel_percent": relative_rank_percent(k, m, n),
                    "c_eq2": compression_eq2(k, m, n), "c_sym": compression_sym(k, m, n)})
    return out

