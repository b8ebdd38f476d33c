"""Adaptive randomized range finder with a posterior error estimate, FP64 CPU
oracle.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper fixes l = R_SVD + p before the projection (section "Randomized
matrix decompositions"); when the rank is chosen by a threshold the right l is
not known in advance. This routine grows the orthonormal basis Q of the range
of V block by block until the threshold rank is resolved, then finishes with
the paper's steps 2 and 3 on the final basis (projection Y = Q^T V, thin SVD,
lift L = Q L_Y).

Growth step (blocked form of the adaptive range finder of Halko, Martinsson
and Tropp, SIAM Rev. 2011, with the power scheme and Frobenius indicator of
the blocked randQB algorithm of Martinsson and Voronin 2016 / Yu, Gu and Li
2018):

  W   = (I - Q Q^T) V P_i      P_i: the next b columns of the projection P
                               (the same Philox stream as the fixed method,
                               so the columns of P never depend on l)
  est = 10 sqrt(2/pi) max_j ||W_j||
        bounds ||(I - Q Q^T) V||_2 except with probability 10^-b
        (Halko et al., section 4.3)
  stop (threshold rule) when est <= tau * s1 and the threshold rank of the
        current projection is at most l - p; s1 is a lower bound of the
        largest singular value of Y (the largest row norm of Y)
  else:
  Q_i = orth(W), re-orthonormalized once against Q: Q_i = orth(Q_i - Q Q^T Q_i)
  q times (power scheme on the deflated matrix (I - Q Q^T) V):
        Q_i' = orth(V^T Q_i);  Q_i = orth((I - Q Q^T) V Q_i') (+ the same
        re-orthonormalization)
  Y_i = Q_i^T V;  Q = [Q, Q_i], Y = [Y; Y_i];  l += b
  stop (Frobenius rule) when ||V||_F^2 - ||Y||_F^2 <= tau^2 ||V||_F^2 and the
        Frobenius-tail rank is at most l - p

A stop is accepted only after the small SVD of the current Y confirms that
the rank rule keeps at most l - p values; otherwise growth continues. Growth
ends at l_max with FLAG_ADAPT_LIMIT.

Library primitives: numpy's matrix product, LAPACK Householder QR (orth) and
SVD; nothing is blocked or fused beyond the steps above.
"""

import math

import numpy as np

from .method import (FLAG_FULL_SVD, FLAG_RANK_CAPPED, RANK_FROB_TAIL, RANK_REL_THRESHOLD,
                     RsvdResult, compression_eq2, compression_sym, orth,
                     relative_rank_percent, residual, select_rank, sign_normalize)
from .philox import gaussian_omega

FLAG_ADAPT_LIMIT = 64

# Halko et al. (2011), Eq. (4.3): ||(I - QQ^T) A|| <= 10 sqrt(2/pi) max_i ||(I - QQ^T) A w_i||
POSTERIOR_FACTOR = 10.0 * math.sqrt(2.0 / math.pi)


def _deflate(Q, X):
    """(I - Q Q^T) X."""
    if Q.shape[1] == 0:
        return X
    return X - Q @ (Q.T @ X)


def _orth_against(Q, W):
    """Orthonormal basis of W, orthogonal to Q: orth, then once more against Q."""
    Qi = orth(W)
    return orth(_deflate(Q, Qi))


def _wanted_rank(s_all, mode, tau, fro2, fro2_Y):
    """Rank the rule asks for before any cap (0 for an all-zero projection)."""
    if len(s_all) == 0 or s_all[0] == 0.0:
        return 0
    if mode == RANK_REL_THRESHOLD:
        return int(np.count_nonzero(s_all >= tau * s_all[0]))
    missed = max(fro2 - float(np.sum(s_all ** 2)), 0.0)
    tail = np.concatenate([np.cumsum((s_all ** 2)[::-1])[::-1], [0.0]])
    for kk in range(len(s_all) + 1):
        if math.sqrt(tail[kk] + missed) <= tau * math.sqrt(fro2):
            return kk
    return len(s_all)


def rsvd_adaptive(A, tau, p, q, block=64, seed=0, channel=0, symmetric=False, l_max=None,
                  rank_mode=RANK_REL_THRESHOLD, k_cap=None, want_residual=True):
    """Adaptive randomized SVD of A (m x n FP64) for a threshold rank rule.

    tau: relative threshold (rel_threshold: keep s_j >= tau s_1; frob_tail:
    discarded energy <= tau ||A||_F). p: columns kept beyond the rank; q:
    power steps per block; block: columns added per growth step.
    Returns an RsvdResult; extra holds est (the last posterior estimate, or
    the Frobenius indicator sqrt(||A||_F^2 - ||Y||_F^2) for frob_tail),
    blocks, fro2_Y and the history of (l, est).
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    mn = min(m, n)
    l_max = mn if l_max is None else min(int(l_max), mn)
    if rank_mode not in (RANK_REL_THRESHOLD, RANK_FROB_TAIL):
        raise ValueError("the adaptive finder serves the threshold rules")
    At = A if symmetric else A.T
    fro2 = float(np.sum(A * A))
    Q = np.zeros((m, 0))
    Y = np.zeros((0, n))
    l = 0
    s1_lb = 0.0
    fro2_Y = 0.0
    flags = 0
    est = math.inf
    history = []
    blocks = 0
    final = None

    def finish(l):
        L_Y, s_all, Rt = np.linalg.svd(Y, full_matrices=False)
        return L_Y, s_all, Rt

    while True:
        b = min(block, l_max - l)
        if b <= 0:
            flags |= FLAG_ADAPT_LIMIT
            final = finish(l)
            break
        P = gaussian_omega(n, b, seed, channel, col0=l)
        W = _deflate(Q, A @ P)
        if rank_mode == RANK_REL_THRESHOLD and l > 0:
            est = POSTERIOR_FACTOR * float(np.max(np.sqrt(np.sum(W * W, axis=0))))
            history.append((l, est))
            if est <= tau * s1_lb:
                cand = finish(l)
                if _wanted_rank(cand[1], rank_mode, tau, fro2, fro2_Y) <= l - p:
                    final = cand
                    break
        Qi = _orth_against(Q, W)
        for _ in range(q):
            Qh = orth(At @ Qi)
            Qi = _orth_against(Q, _deflate(Q, A @ Qh))
        Yi = (At @ Qi).T
        Q = np.concatenate([Q, Qi], axis=1)
        Y = np.concatenate([Y, Yi], axis=0)
        l += b
        blocks += 1
        s1_lb = max(s1_lb, float(np.max(np.sqrt(np.sum(Yi * Yi, axis=1)))))
        fro2_Y += float(np.sum(Yi * Yi))
        if rank_mode == RANK_FROB_TAIL:
            est = math.sqrt(max(fro2 - fro2_Y, 0.0))
            history.append((l, est))
            if est <= tau * math.sqrt(fro2):
                cand = finish(l)
                if _wanted_rank(cand[1], rank_mode, tau, fro2, fro2_Y) <= l - p:
                    final = cand
                    break

    L_Y, s_all, Rt = final
    if l == mn:
        flags |= FLAG_FULL_SVD
    if k_cap is None:
        k_cap = l
    L = Q @ L_Y
    R = Rt.T
    L, R = sign_normalize(L, R)
    rank, f2 = select_rank(s_all, rank_mode, tau, l, 0 if l == mn else p, k_cap, fro2_A=fro2)
    flags |= f2
    U_k, s_k, V_k = L[:, :rank], s_all[:rank], R[:, :rank]
    e = residual(A, U_k, s_k, V_k) if want_residual else float("nan")
    return RsvdResult(
        s=s_k, U=U_k, V=V_k, s_all=s_all, U_all=L, V_all=R, Q=Q, rank=rank, l=l,
        residual=e, rel_percent=relative_rank_percent(rank, m, n),
        c_eq2=compression_eq2(rank, m, n), c_sym=compression_sym(rank, m, n),
        flags=flags,
        extra={"fro2": fro2, "est": est, "blocks": blocks, "fro2_Y": fro2_Y,
               "history": history, "Y": Y},
    )


FLAG_POSTERIOR_FAIL = 256
FLAG_UNCONVERGED = 512
CONVERGED_RATIO = 1e-8


def posterior_judge(A, Q, s_all, rank, q, tau, r, seed=0, channel=0, rel_threshold=True):
    """A-posteriori judge of a fixed-l run with final basis Q (m x l) and
    computed values s_all (l, decreasing), kept rank `rank`:

      est = 10 sqrt(2/pi) max_j ||(I - Q Q^T) A P_r e_j||, P_r = columns
            l .. l + r - 1 of the projection stream (Halko et al., section 4.3)
      UNCONVERGED     when (s_l / s_k)^(4q + 2) > 1e-8 (k = rank), the
                      subspace-iteration factor of the kept values
      POSTERIOR_FAIL  (relative threshold) when est > tau s_1

    An exact decomposition (l = min(m, n)) is never flagged. Returns
    (est, flags)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    l = Q.shape[1]
    P = gaussian_omega(n, l + r, seed, channel)[:, l:]
    W = _deflate(Q, A @ P)
    est = POSTERIOR_FACTOR * float(np.sqrt(np.max(np.sum(W * W, axis=0))))
    flags = 0
    if l < min(m, n):
        k = rank
        if 1 <= k < l and s_all[k - 1] > 0:
            if not (s_all[l - 1] / s_all[k - 1]) ** (4 * q + 2) <= CONVERGED_RATIO:
                flags |= FLAG_UNCONVERGED
        if rel_threshold and not est <= tau * s_all[0]:
            flags |= FLAG_POSTERIOR_FAIL
    return est, flags
