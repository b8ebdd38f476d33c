"""Pins of the symmetric-channel oracle (oracle/symmetric.py) against exact
SVDs of the input, constructed spectra, interlacing theorems and identities
that hold for any orthonormal basis (not against its own library calls)."""

import numpy as np

import synth
from oracle.method import orth, rsvd
from oracle.philox import gaussian_omega
from oracle.symmetric import rsvd_sym

U_EPS = np.finfo(np.float64).eps / 2


def test_full_width_reproduces_exact_svd():
    # l = N: Q is square orthogonal and Q^T A Q is similar to A
    n = 70
    sig = synth.spectrum_pow10(n, 0.2)
    A = synth.symmetric(n, sig, tag=201)
    r = rsvd_sym(A, k=60, p=20, q=0, seed=3)
    exact = np.linalg.svd(A, compute_uv=False)
    assert r.l == n
    assert np.all(np.abs(r.s_all - exact) <= 1e-13 * exact[0])
    recon = (r.U_all * r.s_all) @ r.V_all.T
    assert np.abs(recon - A).max() <= 1e-13 * np.abs(A).max()


def test_constructed_psd_spectrum_converges():
    # (s_{l+1} / s_k)^(4q+2) = exp(-40 * 10 / 10) ~ 4e-18: values exact to 1e-12
    n = 400
    sig = synth.spectrum_exp(n, 10.0)
    A = synth.symmetric(n, sig, tag=202)
    r = rsvd_sym(A, k=30, p=40, q=2, seed=4)
    assert (np.abs(r.s - sig[:30]) / sig[:30]).max() <= 1e-12
    # PSD input: left and right vectors coincide
    assert np.abs(r.U - r.V).max() <= 1e-10


def test_interlacing_and_one_sided_bound():
    # Cauchy interlacing for the compression Q^T A Q of a PSD A:
    # s_j(Q^T A Q) <= s_j(A); and s_j(Q^T A Q) <= s_j(Q^T A) since Q has
    # orthonormal columns: the symmetric form never exceeds the paper's form
    n = 300
    sig = synth.spectrum_exp(n, 30.0)
    A = synth.symmetric(n, sig, tag=203)
    for seed in range(5):
        r = rsvd_sym(A, k=20, p=5, q=0, seed=seed)
        one = rsvd(A, k=20, p=5, q=0, seed=seed, symmetric=True)
        assert np.all(r.s_all <= sig[: r.l] * (1 + 10 * U_EPS))
        assert np.all(r.s_all <= one.s_all * (1 + 100 * U_EPS))
        # and the one-sided projection is strictly larger somewhere (q = 0
        # leaves the basis unconverged, so the two forms differ)
        assert np.max(one.s_all - r.s_all) > 1e-8


def test_exact_low_rank():
    n, rk = 120, 5
    rng = np.random.default_rng(204)
    U = synth.haar_columns(n, rk, rng)
    s = 4.0 * 2.0 ** -np.arange(rk)
    A = (U * s) @ U.T
    A = np.triu(A) + np.triu(A, 1).T
    r = rsvd_sym(A, k=10, p=5, q=1, seed=5)
    assert np.all(np.abs(r.s[:rk] - s) <= 20 * U_EPS * s[0])
    assert np.all(r.s[rk:] <= 20 * U_EPS * s[0])
    assert r.residual <= 1e-14


def test_indefinite_signs():
    # eigenvalues of both signs: the values are |lambda| and R_j = sign(lambda_j) L_j
    n = 150
    rng = np.random.default_rng(205)
    U = synth.haar_columns(n, n, rng)
    mag = 10.0 ** (-np.arange(n) / 15.0)
    sgn = np.where(np.arange(n) % 3 == 1, -1.0, 1.0)
    A = (U * (mag * sgn)) @ U.T
    A = np.triu(A) + np.triu(A, 1).T
    r = rsvd_sym(A, k=12, p=30, q=2, seed=6)
    assert (np.abs(r.s - mag[:12]) / mag[:12]).max() <= 1e-11
    for j in range(12):
        assert np.abs(r.V[:, j] - sgn[j] * r.U[:, j]).max() <= 1e-9


def test_power_of_two_scaling_is_exact():
    n = 200
    A = synth.symmetric(n, synth.spectrum_exp(n, 15.0), tag=206)
    r1 = rsvd_sym(A, k=20, p=10, q=1, seed=7)
    r2 = rsvd_sym(8.0 * A, k=20, p=10, q=1, seed=7)
    assert np.array_equal(r2.s, 8.0 * r1.s)
    assert np.array_equal(r2.U, r1.U) and np.array_equal(r2.V, r1.V)


def test_pythagoras_at_full_sketch_width():
    # ||A - Q B Q^T||_F^2 = ||A||_F^2 - ||B||_F^2 for any orthonormal Q
    # (the cross term <A, Q Q^T A Q Q^T> equals ||Q^T A Q||_F^2)
    n = 250
    A = synth.symmetric(n, synth.spectrum_exp(n, 20.0), tag=207)
    r = rsvd_sym(A, k=40, p=0, q=1, seed=8)
    fro2 = np.sum(A * A)
    e2 = 1.0 - np.sum(r.s_all ** 2) / fro2
    assert abs(r.residual ** 2 - e2) <= 1e-12
    # and the basis is the one the paper's steps build (same P, q, QR schedule)
    P = gaussian_omega(n, 40, 8)
    Q = orth(A @ P)
    Q = orth(A @ orth(A @ Q))
    assert np.abs(Q.T @ Q - np.eye(40)).max() <= 10 * 40 * U_EPS
    assert np.abs(np.abs(r.Q) - np.abs(Q)).max() <= 1e-12


def test_rejects_non_square():
    import pytest
    with pytest.raises(ValueError):
        rsvd_sym(np.zeros((5, 4)), 2, 1, 0)
