"""Pins for the oracle's randomized SVD against closed forms, constructed
spectra and theorems (not against its own library calls)."""

import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import method as orsvd
from oracle.method import rsvd, compression_eq2, compression_sym, percent_rank

U_EPS = np.finfo(np.float64).eps / 2  # unit roundoff
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def _ortho_err(X):
    return np.abs(X.T @ X - np.eye(X.shape[1])).max()


def test_full_rank_sketch_is_exact_svd():
    # l = min(m, n): the method is an exact SVD, so the constructed sigma come back
    m, n = 60, 40
    sig = synth.spectrum_pow10(n, 0.25)
    A = synth.general(m, n, sig, tag=101)
    r = rsvd(A, k=35, p=10, q=0, seed=1)
    assert r.l == n and r.flags & orsvd.FLAG_FULL_SVD
    assert np.all(np.abs(r.s - sig[:35]) <= 1e-13 * sig[0])
    recon = (r.U_all * r.s_all) @ r.V_all.T
    assert np.abs(recon - A).max() <= 1e-14 * np.abs(A).max() * 10


def test_constructed_spectrum_converged_general():
    # (sigma_{l+1}/sigma_k)^(4q+2) = 10^(-31*10/16) ~ 1e-19: sigma exact to 1e-12
    m, n = 300, 200
    sig = synth.spectrum_pow10(n, 1 / 16)
    A = synth.general(m, n, sig, tag=102)
    r = rsvd(A, k=20, p=30, q=2, seed=5)
    rel = np.abs(r.s - sig[:20]) / sig[:20]
    assert rel.max() <= 1e-12
    # with q = 0 the same sketch is far from converged: the q loop is doing work
    r0 = rsvd(A, k=20, p=30, q=0, seed=5)
    assert (np.abs(r0.s - sig[:20]) / sig[:20]).max() > 1e-8


def test_power_iteration_uses_transpose_for_general_input():
    # for a square general matrix (U != V), a loop that multiplied by A where
    # A^T belongs would converge to the wrong subspace; the oracle's loop
    # reaches the constructed values and the wrong one visibly does not
    n = 150
    sig = synth.spectrum_pow10(n, 1 / 8)
    A = synth.general(n, n, sig, tag=103)
    r = rsvd(A, k=10, p=20, q=2, seed=2)
    assert (np.abs(r.s - sig[:10]) / sig[:10]).max() <= 1e-12
    from oracle.philox import gaussian_omega
    Q = orsvd.orth(A @ gaussian_omega(n, 30, 2))
    for _ in range(2):
        Q = orsvd.orth(A @ Q)  # wrong operand on purpose
        Q = orsvd.orth(A @ Q)
    s_wrong = np.linalg.svd(Q.T @ A, compute_uv=False)[:10]
    assert (np.abs(s_wrong - sig[:10]) / sig[:10]).max() > 1e-6


def test_exact_low_rank():
    A, s = synth.rank_r(120, 90, 5, tag=104, scale=3.0)
    r = rsvd(A, k=10, p=5, q=1, seed=3)
    assert np.all(np.abs(r.s[:5] - s) <= 1e-14 * s[0] * 10)
    assert np.all(r.s[5:] <= 1e-14 * s[0])
    assert r.residual <= 1e-14


def test_rank_one_like_c_E():
    # one singular value of order ten, all others zero (the c_E topology)
    gold = json.load(open(GOLDEN))["c_E_rank_one"]
    A, s = synth.rank_r(200, 200, 1, tag=105, scale=10.0)
    r = rsvd(A, k=5, p=5, q=0, seed=4)
    assert abs(r.s[0] - 10.0) <= 1e-13 * 10.0
    assert np.all(r.s[1:] < gold["others_below"] * 10.0)


def test_interlacing_and_pythagoras():
    m, n = 250, 180
    sig = synth.spectrum_exp(n, 15.0)
    A = synth.general(m, n, sig, tag=106)
    r = rsvd(A, k=30, p=6, q=0, seed=6, rank_mode="fixed", rank_param=36)
    # singular values of Q^T A never exceed those of A
    assert np.all(r.s_all <= sig[: r.l] * (1 + 10 * U_EPS) + 1e-15)
    # ||A||^2 = ||Q^T A||^2 + ||(I - QQ^T) A||^2, and with rank = l, e^2 = 1 - ||B||^2/||A||^2
    Q = r.Q
    B = Q.T @ A
    nA, nB, nR = (np.sum(X * X) for X in (A, B, A - Q @ B))
    assert abs(nA - nB - nR) <= 1e-13 * nA
    assert abs(r.residual ** 2 - (1 - nB / nA)) <= 1e-12


def test_scaling_has_no_hidden_normalization():
    m, n = 90, 70
    sig = synth.spectrum_pow10(n, 0.1)
    A = synth.general(m, n, sig, tag=107)
    r1 = rsvd(A, k=8, p=8, q=1, seed=7)
    r2 = rsvd(A * 8.0, k=8, p=8, q=1, seed=7)
    np.testing.assert_allclose(r2.s, 8.0 * r1.s, rtol=4 * U_EPS * 8, atol=0)
    np.testing.assert_allclose(r2.U, r1.U, rtol=0, atol=1e-13)
    np.testing.assert_allclose(r2.V, r1.V, rtol=0, atol=1e-13)


def test_orthonormality_and_signs():
    m, n = 200, 160
    sig = synth.spectrum_exp(n, 10.0)
    A = synth.general(m, n, sig, tag=108)
    r = rsvd(A, k=25, p=10, q=2, seed=8)
    l = r.l
    assert _ortho_err(r.Q) <= 10 * l * U_EPS
    assert _ortho_err(r.U_all) <= 10 * l * U_EPS
    assert _ortho_err(r.V_all) <= 10 * l * U_EPS
    assert np.all(np.diff(r.s_all) <= 0)
    idx = np.argmax(np.abs(r.U), axis=0)
    assert np.all(r.U[idx, np.arange(r.rank)] > 0)


def test_sign_rule_ties_lowest_index_wins():
    # constructed ties: column 0 has |entry| 0.5 at rows 0 (negative), 1 and 2;
    # column 1 has 0.6 at row 0 (positive) and -0.6 at row 1. The entry of
    # largest magnitude with the lowest index decides: column 0 flips,
    # column 1 stays; V's columns follow their U column
    from oracle.method import sign_normalize
    U = np.array([[-0.5, 0.6], [0.5, -0.6], [0.5, 0.1], [0.1, 0.2]])
    V = np.array([[1.0, 2.0], [3.0, -4.0], [-5.0, 6.0]])
    U2, V2 = sign_normalize(U, V)
    assert np.array_equal(U2, [[0.5, 0.6], [-0.5, -0.6], [-0.5, 0.1], [-0.1, 0.2]])
    assert np.array_equal(V2, [[-1.0, 2.0], [-3.0, -4.0], [5.0, 6.0]])
    # a zero column keeps its sign
    Z, W = sign_normalize(np.zeros((3, 1)), np.ones((2, 1)))
    assert np.array_equal(Z, np.zeros((3, 1))) and np.array_equal(W, np.ones((2, 1)))


def test_halko_average_error_bound_q0():
    # Halko, Martinsson, Tropp (2011), Thm 10.5: for q = 0 and p >= 2,
    # E ||(I - QQ^T) A||_F <= (1 + k/(p-1))^(1/2) (sum_{j>k} sigma_j^2)^(1/2)
    m, n, k, p = 80, 60, 6, 4
    sig = synth.spectrum_exp(n, 8.0)
    A = synth.general(m, n, sig, tag=109)
    nA = np.linalg.norm(A)
    errs = []
    for seed in range(200):
        r = rsvd(A, k=k, p=p, q=0, seed=seed, rank_mode="fixed", rank_param=k + p)
        errs.append(r.residual * nA)
    bound = math.sqrt(1 + k / (p - 1)) * math.sqrt(np.sum(sig[k:] ** 2))
    assert np.mean(errs) <= bound
    # and no projection of rank l beats the best rank-l approximation
    assert min(errs) >= math.sqrt(np.sum(sig[k + p:] ** 2)) * (1 - 1e-12)


def test_symmetric_flag_equals_general_route():
    n = 150
    sig = synth.spectrum_exp(n, 12.0)
    A = synth.symmetric(n, sig, tag=110)
    assert np.array_equal(A, A.T)
    r1 = rsvd(A, k=20, p=10, q=2, seed=9, symmetric=True)
    r2 = rsvd(A, k=20, p=10, q=2, seed=9, symmetric=False)
    np.testing.assert_allclose(r1.s, r2.s, rtol=1e-12, atol=1e-15)


def test_threshold_rank_rule():
    n = 300
    d = 20.0
    sig = synth.spectrum_exp(n, d)
    A = synth.symmetric(n, sig, tag=111)
    tau = 1e-4
    r = rsvd(A, k=200, p=20, q=3, seed=10, symmetric=True, rank_mode="rel_threshold", rank_param=tau)
    # sigma_j >= tau sigma_0  <=>  j <= d ln(1/tau)
    expect = int(math.floor(d * math.log(1 / tau))) + 1
    assert r.rank == expect
    # cap at l - p binds when tau is below what l can resolve
    r2 = rsvd(A, k=100, p=20, q=3, seed=10, symmetric=True, rank_mode="rel_threshold", rank_param=1e-6)
    assert r2.rank == 100 and r2.flags & orsvd.FLAG_RANK_CAPPED


def test_threshold_rank_uncapped_for_exact_svd():
    # l = min(m, n): every value is exact, so the rule keeps all values above
    # the threshold even beyond l - p
    n = 60
    sig = synth.spectrum_exp(n, 5.0)
    A = synth.symmetric(n, sig, tag=114)
    r = rsvd(A, k=50, p=20, q=0, seed=12, symmetric=True, rank_mode="rel_threshold", rank_param=1e-5)
    expect = int(math.floor(5.0 * math.log(1e5))) + 1  # 58 > l - p = 40
    assert r.l == n and r.rank == expect
    assert r.flags == orsvd.FLAG_FULL_SVD


def test_percent_rank_and_eq2_values():
    gold = json.load(open(GOLDEN))
    N = gold["channel_dims"][1]["N"]
    assert N % 225 == 0 and gold["channel_dims"][0]["N"] % 225 == 0  # 15 x 15 mesh
    assert percent_rank(1.0, N, N) == 401  # ceil(400.5)
    assert percent_rank(0.2, 7650, 7650) == 16  # ceil(15.3)
    assert percent_rank(1.0, 7650, 7650) == 77  # ceil(76.5)
    assert percent_rank(2.0, 100, 100) == 2  # exact integer is not rounded up
    # Eq. 2 as printed gives ~50 at R% = 1 (N^2/(2 N R) -> 100/2); the text says ~100.
    # The form with one stored factor, N^2/(N R + R), reproduces the text's values.
    for row in gold["eq2_text_values"]:
        k = row["rel_percent"] * N / 100.0  # real-valued R_SVD, as in the text's estimate
        c_eq2 = N * N / (2 * N * k + k)
        c_sym = N * N / (N * k + k)
        assert abs(c_eq2 / (row["C_text_approx"] / 2) - 1) < 0.01
        assert abs(c_sym / row["C_text_approx"] - 1) < 0.01
    assert abs(compression_eq2(401, N, N) - N * N / (2 * N * 401 + 401)) < 1e-9
    assert abs(compression_sym(401, N, N) - N * N / (N * 401 + 401)) < 1e-9


def test_frobenius_tail_rank_rule():
    n = 200
    sig = synth.spectrum_exp(n, 10.0)
    A = synth.symmetric(n, sig, tag=112)
    tau = 1e-3
    r = rsvd(A, k=120, p=20, q=2, seed=11, symmetric=True, rank_mode="frob_tail", rank_param=tau)
    # closed form on the constructed spectrum: smallest k with tail energy <= tau^2 ||A||^2
    tot = np.sum(sig ** 2)
    tails = np.array([np.sum(sig[j:] ** 2) for j in range(n + 1)])
    expect = int(np.argmax(np.sqrt(tails) <= tau * np.sqrt(tot)))
    assert r.rank == expect
    assert r.residual <= tau * (1 + 1e-6)


def test_fixed_rank_clamped_by_k_cap():
    A = synth.general(50, 40, synth.spectrum_exp(40, 5.0), tag=113)
    r = rsvd(A, k=10, p=5, q=0, seed=1, k_cap=7)
    assert r.rank == 7 and r.flags & orsvd.FLAG_RANK_CAPPED
