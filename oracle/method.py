"""Randomized truncated SVD, FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY (see the package header).

Follows the section "Randomized matrix decompositions" of arXiv:2307.15572
and its Fig. 1, in the paper's notation (V is the input matrix, P the random
projection, R_SVD the kept rank, l = R_SVD + p):

  step 1  Z = V P; QR decomposition Z = Q X (only Q is kept)
  step 2  Y = Q^T V; thin SVD Y = L_Y Sigma R^T
  step 3  L = Q L_Y
  then    keep the R_SVD leading singular triplets (Eq. 1 orders the singular
          values decreasingly), report R% = 100 R_SVD / N and the compression
          ratio of Eq. 2.

Readings where the paper is silent (all listed in the design notes):
  * q >= 0 power iterations between step 1 and step 2 (Halko et al.,
    randomized subspace iteration): Z' = V^T Q -> QR -> Z = V Q' -> QR, with
    a QR after every product. q = 0 is the paper's method exactly.
  * Symmetric input: the caller asserts V == V^T and V is used for V^T.
  * l = min(R_SVD + p, m, n); if l = min(m, n) the result is an exact SVD.
  * Signs: each pair (L_j, R_j) is flipped so that the entry of largest
    magnitude of L_j is positive (the lowest index wins ties).
  * Rank rules: fixed R_SVD; percent (R_SVD = ceil(R% * min(m, n) / 100));
    relative threshold (R_SVD = #{j : s_j >= tau * s_1}, at most l - p
    unless l = min(m, n), where every value is exact);
    Frobenius tail (smallest R_SVD whose discarded energy, including what
    the sketch missed, is at most tau * ||V||_F).
  * Eq. 2 is reported as printed, C = m n / ((m + n) R_SVD + R_SVD), which is
    N^2 / (2 N R_SVD + R_SVD) for square V, and in the form that matches the
    paper's own worked values (C ~ 100 at R% = 1), C_sym = N^2/(N R_SVD + R_SVD).

Library primitives used as steps: numpy's matrix product, LAPACK's
Householder QR (numpy.linalg.qr; signs fixed so diag(X) >= 0) and LAPACK's
SVD (numpy.linalg.svd) for the small l x n matrix. Nothing is blocked, fused
or reordered beyond the steps above.

Pins (tests/test_oracle_*.py): matrices with constructed singular values,
exact results when l = min(m, n), exactly low-rank inputs, interlacing,
Pythagoras for the projection, power-of-two scaling, orthonormality, the
Halko et al. average-error theorem for q = 0 over many seeds, and the
values printed with Eq. 2.
"""

from dataclasses import dataclass, field
import math

import numpy as np

from .philox import gaussian_omega

# Rank rules
RANK_FIXED = "fixed"
RANK_PERCENT = "percent"
RANK_REL_THRESHOLD = "rel_threshold"
RANK_FROB_TAIL = "frob_tail"

# Result flags (same meaning as the library's result flags)
FLAG_FULL_SVD = 1
FLAG_RANK_CAPPED = 2


@dataclass
class RsvdResult:
    s: np.ndarray          # kept singular values, decreasing (rank,)
    U: np.ndarray          # left singular vectors L (m x rank)
    V: np.ndarray          # right singular vectors R (n x rank)
    s_all: np.ndarray      # all l singular values of Y = Q^T V
    U_all: np.ndarray      # m x l
    V_all: np.ndarray      # n x l
    Q: np.ndarray          # final orthonormal basis (m x l)
    rank: int
    l: int
    residual: float        # ||V - L_k S_k R_k^T||_F / ||V||_F (nan if not asked)
    rel_percent: float
    c_eq2: float
    c_sym: float
    flags: int = 0
    extra: dict = field(default_factory=dict)


def orth(Z):
    """Q factor of the thin Householder QR Z = Q X, signs fixed so diag(X) >= 0."""
    Q, X = np.linalg.qr(Z, mode="reduced")
    d = np.sign(np.diag(X))
    d[d == 0] = 1.0
    return Q * d[None, :]


def sign_normalize(U, V):
    """Flip (U_j, V_j) together so the largest-magnitude entry of U_j is > 0."""
    U = U.copy()
    V = V.copy()
    if U.shape[0] == 0:
        return U, V
    idx = np.argmax(np.abs(U), axis=0)  # first index of the maximum
    sgn = np.sign(U[idx, np.arange(U.shape[1])])
    sgn[sgn == 0] = 1.0
    return U * sgn[None, :], V * sgn[None, :]


def relative_rank_percent(rank, m, n):
    """R% = 100 R_SVD / N, with N = min(m, n) for a non-square matrix."""
    return 100.0 * rank / min(m, n)


def compression_eq2(rank, m, n):
    """Eq. 2 as printed: N^2 / (2 N R_SVD + R_SVD); m n / ((m + n) R + R) if m != n."""
    return (m * n) / ((m + n) * rank + rank) if rank > 0 else math.inf


def compression_sym(rank, m, n):
    """Storage ratio with one factor stored: N^2 / (N R_SVD + R_SVD)."""
    return (m * n) / (max(m, n) * rank + rank) if rank > 0 else math.inf


def percent_rank(percent, m, n):
    """R_SVD = ceil(R% * min(m, n) / 100), with a 1e-12 relative guard so that
    a product that is an integer in exact arithmetic is not rounded up."""
    x = percent * min(m, n) / 100.0
    return int(math.ceil(x * (1.0 - 1e-12)))


def select_rank(s_all, mode, param, l, p, k_cap, fro2_A=None):
    """Rank rule. Returns (rank, flags)."""
    flags = 0
    if mode == RANK_FIXED:
        k = int(param)
    elif mode == RANK_PERCENT:
        raise ValueError("percent rank is resolved at plan time; pass it as fixed")
    elif mode == RANK_REL_THRESHOLD:
        tau = float(param)
        # an all-zero projection has no value above the threshold (k = 1 below)
        k = int(np.count_nonzero(s_all >= tau * s_all[0])) if len(s_all) and s_all[0] > 0 else 0
        cap = max(l - p, 1)
        if k > cap:
            k = cap
            flags |= FLAG_RANK_CAPPED
    elif mode == RANK_FROB_TAIL:
        tau = float(param)
        # discarded energy = sum_{j>k} s_j^2 + (||V||_F^2 - ||Y||_F^2)
        missed = max(fro2_A - float(np.sum(s_all ** 2)), 0.0)
        tail = np.concatenate([np.cumsum((s_all ** 2)[::-1])[::-1], [0.0]])  # tail[k] = sum_{j>=k}
        k = len(s_all)
        for kk in range(0, len(s_all) + 1):
            if math.sqrt(tail[kk] + missed) <= tau * math.sqrt(fro2_A):
                k = kk
                break
        cap = max(l - p, 1)
        if k > cap:
            k = cap
            flags |= FLAG_RANK_CAPPED
    else:
        raise ValueError(mode)
    k = max(1, min(k, l))
    if k > k_cap:
        k = k_cap
        flags |= FLAG_RANK_CAPPED
    return k, flags


def residual(A, U, s, V):
    """e = ||A - U diag(s) V^T||_F / ||A||_F, evaluated entrywise in FP64."""
    E = A - (U * s[None, :]) @ V.T
    return float(np.sqrt(np.sum(E * E)) / np.sqrt(np.sum(A * A)))


def rsvd(A, k, p, q, seed=0, channel=0, symmetric=False, omega=None,
         rank_mode=RANK_FIXED, rank_param=None, k_cap=None, want_residual=True):
    """Randomized SVD of A (m x n, FP64) following the paper's three steps.

    k: target rank R_SVD used to size l = min(k + p, m, n). For the fixed rule
    it is also the kept rank; for the other rules rank_param holds R% or tau.
    omega: optional n x l test matrix; default is the Philox/Box-Muller stream
    keyed by (seed, channel).
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if rank_mode == RANK_PERCENT:
        k = percent_rank(rank_param, m, n)
        rank_mode, rank_param = RANK_FIXED, k
    if rank_mode == RANK_FIXED and rank_param is None:
        rank_param = k
    l = min(k + p, m, n)
    flags = FLAG_FULL_SVD if l == min(m, n) else 0
    if k_cap is None:
        k_cap = l
    At = A if symmetric else A.T

    # step 1: random projection and QR
    P = gaussian_omega(n, l, seed, channel) if omega is None else np.asarray(omega, np.float64)
    Z = A @ P
    Q = orth(Z)
    # power (subspace) iterations, QR after every product
    for _ in range(q):
        Q = orth(At @ Q)
        Q = orth(A @ Q)
    # step 2: projection and thin SVD
    Y = Q.T @ A
    L_Y, s_all, Rt = np.linalg.svd(Y, full_matrices=False)
    # step 3: lift
    L = Q @ L_Y
    R = Rt.T
    L, R = sign_normalize(L, R)

    fro2 = float(np.sum(A * A))
    # the l - p cap protects unconverged trailing values; an exact SVD has none
    p_cap = 0 if l == min(m, n) else p
    rank, f2 = select_rank(s_all, rank_mode, rank_param, l, p_cap, k_cap, fro2_A=fro2)
    flags |= f2
    U_k, s_k, V_k = L[:, :rank], s_all[:rank], R[:, :rank]
    e = residual(A, U_k, s_k, V_k) if want_residual else float("nan")
    return RsvdResult(
        s=s_k, U=U_k, V=V_k, s_all=s_all, U_all=L, V_all=R, Q=Q, rank=rank, l=l,
        residual=e, rel_percent=relative_rank_percent(rank, m, n),
        c_eq2=compression_eq2(rank, m, n), c_sym=compression_sym(rank, m, n),
        flags=flags, extra={"fro2": fro2},
    )
