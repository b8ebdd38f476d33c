"""Randomized decomposition of a symmetric channel matrix in the form
A ~ Q B Q^T with B = Q^T A Q, FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper decomposes each partial-wave channel matrix V on its own (section
"Low-rank interactions": the symmetry-adapted basis keeps the interaction
block diagonal in the conserved quantum numbers), and its method projects
V onto the sketch basis from one side only, Y = Q^T V (section "Randomized
matrix decompositions", Fig. 1). The channel matrices of a Hermitian
interaction are symmetric, V = V^T, so both factors can be taken in the
same basis: V ~ Q (Q^T V Q) Q^T. This is Halko, Martinsson and Tropp (SIAM
Review 2011), section 5.3 ("Hermitian matrices", direct decomposition), with
||V - Q B Q^T|| <= 2 ||V - Q Q^T V|| and B only l x l instead of l x N.

Steps (the same P, q and QR schedule as oracle.method.rsvd, which the
symmetric case shares up to the final basis Q):
  step 1  Z = V P; Q = orth(Z); q times: Q = orth(V Q); Q = orth(V Q)
  form    C = V Q (one more product with V); B = Q^T C (l x l);
          B <- (B + B^T) / 2 (B is symmetric in exact arithmetic; the
          average removes the rounding asymmetry)
  SVD     B = L_B Sigma R_B^T (singular values of B = |eigenvalues|)
  lift    L = Q L_B, R = Q R_B (for a positive semidefinite V, L = R up to
          rounding; a negative eigenvalue gives R_j = -L_j)
  then    sign rule, rank rule, R%, Eq. 2 and the residual exactly as
          oracle.method.rsvd.

Library primitives used as steps: numpy's matrix product, LAPACK's Householder
QR (oracle.method.orth) and LAPACK's SVD of the l x l matrix.

Pins (tests/test_oracle_symmetric.py): l = N reproduces the exact singular
values of V (numpy's SVD of V itself); constructed PSD spectra converge;
Cauchy interlacing (sigma_j(Q^T V Q) <= sigma_j(V)) and the bound by the
one-sided projection's values (sigma_j(Q^T V Q) <= sigma_j(Q^T V)); exact
low rank; an indefinite matrix gives |eigenvalues| with R_j = sign(lambda_j)
L_j; power-of-two scaling is exact; with k = l the residual obeys
||V - Q B Q^T||_F^2 = ||V||_F^2 - ||B||_F^2.
"""

import numpy as np

from .method import (
    FLAG_FULL_SVD,
    RANK_FIXED,
    RANK_PERCENT,
    RsvdResult,
    compression_eq2,
    compression_sym,
    orth,
    percent_rank,
    relative_rank_percent,
    residual,
    select_rank,
    sign_normalize,
)
from .philox import gaussian_omega


def rsvd_sym(A, k, p, q, seed=0, channel=0, omega=None, rank_mode=RANK_FIXED, rank_param=None,
             k_cap=None, want_residual=True):
    """Randomized decomposition A ~ Q (Q^T A Q) Q^T of a symmetric A (n x n).

    Parameters as oracle.method.rsvd (A must be symmetric; it is used for
    A^T). Returns an RsvdResult whose U and V are L = Q L_B and R = Q R_B.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if m != n:
        raise ValueError("the symmetric form needs a square matrix")
    if rank_mode == RANK_PERCENT:
        k = percent_rank(rank_param, m, n)
        rank_mode, rank_param = RANK_FIXED, k
    if rank_mode == RANK_FIXED and rank_param is None:
        rank_param = k
    l = min(k + p, n)
    flags = FLAG_FULL_SVD if l == n else 0
    if k_cap is None:
        k_cap = l

    # step 1 and the power iterations (A stands for A^T)
    P = gaussian_omega(n, l, seed, channel) if omega is None else np.asarray(omega, np.float64)
    Q = orth(A @ P)
    for _ in range(q):
        Q = orth(A @ Q)
        Q = orth(A @ Q)
    # the l x l core in the sketch basis, symmetrized
    C = A @ Q
    B = Q.T @ C
    B = 0.5 * (B + B.T)
    L_B, s_all, R_Bt = np.linalg.svd(B)
    L = Q @ L_B
    R = Q @ R_Bt.T
    L, R = sign_normalize(L, R)

    fro2 = float(np.sum(A * A))
    p_cap = 0 if l == n else p
    rank, f2 = select_rank(s_all, rank_mode, rank_param, l, p_cap, k_cap, fro2_A=fro2)
    flags |= f2
    U_k, s_k, V_k = L[:, :rank], s_all[:rank], R[:, :rank]
    e = residual(A, U_k, s_k, V_k) if want_residual else float("nan")
    return RsvdResult(
        s=s_k, U=U_k, V=V_k, s_all=s_all, U_all=L, V_all=R, Q=Q, rank=rank, l=l,
        residual=e, rel_percent=relative_rank_percent(rank, m, n),
        c_eq2=compression_eq2(rank, m, n), c_sym=compression_sym(rank, m, n),
        flags=flags, extra={"fro2": fro2, "B": B},
    )
