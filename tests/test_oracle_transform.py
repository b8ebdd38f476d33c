"""Pins of the factor-space basis transform and the truncation report
(oracle/transform.py): the dense definition U^T V U, invariants of an
orthogonal change of basis, special matrices, Pythagoras and Eq. 2."""

import math

import numpy as np

import synth
from oracle.method import rsvd
from oracle.transform import factor_transform, truncation_report


def _factors(N, k, tag):
    rng = np.random.default_rng(tag)
    L = synth.haar_columns(N, k, rng)
    R = synth.haar_columns(N, k, rng)
    s = 10.0 ** (-np.arange(k) / 4.0)
    return L, s, R


def test_matches_dense_transform_nonsymmetric_basis():
    # Vbar = U^T (L S R^T) U computed as two N x N x N products; a factor form
    # that used U instead of U^T, or swapped L and R, fails for this U
    N, k = 90, 12
    L, s, R = _factors(N, k, 301)
    Ub = synth.haar_columns(N, N, np.random.default_rng(302))
    assert np.abs(Ub - Ub.T).max() > 0.1
    V = (L * s) @ R.T
    dense = Ub.T @ V @ Ub
    Lb, Rb = factor_transform(Ub, L, R)
    assert np.abs((Lb * s) @ Rb.T - dense).max() <= 1e-14 * 50


def test_orthonormality_and_sigma_preserved():
    N, k = 120, 10
    L, s, R = _factors(N, k, 303)
    Ub = synth.haar_columns(N, N, np.random.default_rng(304))
    Lb, Rb = factor_transform(Ub, L, R)
    eye = np.eye(k)
    assert np.abs(Lb.T @ Lb - eye).max() <= 1e-14 * 20
    assert np.abs(Rb.T @ Rb - eye).max() <= 1e-14 * 20
    got = np.linalg.svd((Lb * s) @ Rb.T, compute_uv=False)[:k]
    assert np.abs(got - s).max() <= 1e-14 * 20


def test_rectangular_basis_with_orthonormal_columns():
    # U: N x N' (N' < N), Vbar is N' x N'
    N, Np, k = 100, 60, 8
    L, s, R = _factors(N, k, 305)
    Ub = synth.haar_columns(N, Np, np.random.default_rng(306))
    Lb, Rb = factor_transform(Ub, L, R)
    assert Lb.shape == (Np, k) and Rb.shape == (Np, k)
    assert np.abs((Lb * s) @ Rb.T - Ub.T @ ((L * s) @ R.T) @ Ub).max() <= 1e-14 * 50


def test_identity_and_permutation():
    N, k = 40, 5
    L, s, R = _factors(N, k, 307)
    Lb, Rb = factor_transform(np.eye(N), L, R)
    assert np.array_equal(Lb, L) and np.array_equal(Rb, R)
    perm = np.random.default_rng(308).permutation(N)
    Pm = np.eye(N)[:, perm]  # column j of U is e_perm[j]: row j of U^T L is row perm[j] of L
    Lp, Rp = factor_transform(Pm, L, None)
    assert Rp is None and np.array_equal(Lp, L[perm])


def test_truncation_report_pythagoras_and_eq2():
    # an exact SVD (l = N): residual^2 = 1 - sum_{j<=k} s_j^2 / ||A||_F^2
    N = 450
    A, sig = synth.paper_channel(N)
    r = rsvd(A, k=N, p=0, q=0, seed=1, symmetric=True)
    rep = truncation_report(A, r.U_all, r.s_all, r.V_all, (0.2, 0.5, 1.0, 10.0))
    fro2 = np.sum(A * A)
    for row in rep:
        k = row["rank"]
        assert k == math.ceil(row["percent"] * N / 100 - 1e-9)
        e2 = 1.0 - np.sum(sig[:k] ** 2) / fro2
        assert abs(row["residual"] ** 2 - e2) <= 1e-12
        assert row["c_eq2"] == N * N / (2 * N * k + k)
        assert row["c_sym"] == N * N / (N * k + k)
    # 0.2 % of 450 = 0.9 -> R_SVD = 1; 1 % -> 4.5 -> 5
    assert [row["rank"] for row in rep] == [1, 3, 5, 45]
