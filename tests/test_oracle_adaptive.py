"""Pins of the adaptive range finder oracle (oracle/adaptive.py).

Each check ties the oracle to something other than itself: the fixed-width
method in exact arithmetic (q = 0 spans the same space), the probabilistic
bound of Halko et al. section 4.3, constructed spectra, exact low rank,
Pythagoras for the Frobenius indicator and orthonormality.
"""

import math

import numpy as np
import pytest

import synth
from oracle.adaptive import FLAG_ADAPT_LIMIT, POSTERIOR_FACTOR, rsvd_adaptive
from oracle.method import FLAG_RANK_CAPPED, rsvd
from oracle.philox import gaussian_omega

U64 = np.finfo(np.float64).eps / 2


def test_posterior_factor_value():
    # 10 sqrt(2/pi) (Halko et al. 2011, Eq. (4.3))
    assert POSTERIOR_FACTOR == pytest.approx(7.978845608028654, rel=1e-15)


def test_q0_spans_the_fixed_sketch():
    # With q = 0 the grown basis spans A P[:, :l], exactly the fixed method's
    # sketch for the same l (the columns of P do not depend on l), so both give
    # the same singular values up to rounding.
    sigma = synth.spectrum_exp(600, 12.0)
    A = synth.general(700, 600, sigma, tag=78)
    r = rsvd_adaptive(A, 1e-6, 10, 0, block=48, seed=9)
    f = rsvd(A, r.l - 10, 10, 0, seed=9)
    assert f.l == r.l
    assert np.max(np.abs(r.s_all - f.s_all)) <= 1e-13 * f.s_all[0]
    sel = f.s_all >= 1e-8 * f.s_all[0]
    assert np.max(np.abs(r.s_all[sel] - f.s_all[sel]) / f.s_all[sel]) <= 1e-8


def test_blocks_use_stable_projection_columns():
    # the blocks drawn at col0 = 0, b, 2b, ... tile the l-column projection
    n, b = 37, 8
    whole = gaussian_omega(n, 3 * b, 5, 2)
    parts = np.concatenate([gaussian_omega(n, b, 5, 2, col0=c) for c in (0, b, 2 * b)], axis=1)
    assert np.array_equal(whole, parts)


@pytest.mark.parametrize("seed", range(30))
def test_posterior_estimate_bounds_true_residual(seed):
    # ||(I - QQ^T) A||_2 <= est except with probability 10^-b (b = 16 here)
    sigma = synth.spectrum_exp(160, 6.0)
    A = synth.general(200, 160, sigma, tag=500 + seed)
    r = rsvd_adaptive(A, 1e-5, 6, 0, block=16, seed=seed)
    E = A - r.Q @ (r.Q.T @ A)
    true = np.linalg.norm(E, 2)
    est = r.extra["est"]
    assert true <= est
    # and it is a bound of the right size, not a blow-up (||E||_F / ||E||_2 is small here)
    assert est <= 200 * true


@pytest.mark.parametrize("d,q", [(20.0, 2), (12.0, 1), (8.0, 0)])
def test_threshold_rank_of_constructed_spectrum(d, q):
    n = 700
    tau = 1e-6
    sigma = synth.spectrum_exp(n, d)
    A = synth.symmetric(n, sigma, tag=77, channel=int(d))
    r = rsvd_adaptive(A, tau, 16, q, block=64, seed=5, symmetric=True)
    k_true = int(np.count_nonzero(sigma >= tau))
    # no constructed value sits within 0.5 % of the threshold at these d
    assert np.min(np.abs(sigma / tau - 1.0)) > 5e-3
    assert r.rank == k_true
    assert r.l >= r.rank + 16
    assert r.flags == 0
    rel = np.abs(r.s - sigma[: r.rank]) / sigma[: r.rank]
    assert rel.max() <= 1e-7
    assert r.extra["est"] <= tau * r.s[0]


def test_exact_low_rank_stops_after_first_block():
    A, s = synth.rank_r(300, 200, 5, tag=41)
    r = rsvd_adaptive(A, 1e-8, 8, 1, block=32, seed=3)
    assert r.l == 32 and r.extra["blocks"] == 1
    assert r.rank == 5
    assert np.max(np.abs(r.s - s) / s) <= 1e-13
    assert r.extra["est"] <= 1e-13 * s[0]
    assert r.residual <= 1e-14


def test_frobenius_indicator_and_rule():
    sigma = synth.spectrum_exp(600, 12.0)
    A = synth.general(700, 600, sigma, tag=78)
    tau = 1e-4
    r = rsvd_adaptive(A, tau, 10, 1, block=32, seed=9, rank_mode="frob_tail")
    E = A - r.Q @ r.extra["Y"]
    # Pythagoras: ||A||_F^2 - ||Y||_F^2 = ||A - Q Y||_F^2 (Y = Q^T A)
    assert abs(r.extra["est"] ** 2 - np.sum(E * E)) <= 1e-14 * r.extra["fro2"]
    # the kept rank meets the Frobenius rule, checked on A itself
    assert r.residual <= tau * (1 + 1e-8)
    # and one fewer value would not
    Uk, sk, Vk = r.U_all[:, : r.rank - 1], r.s_all[: r.rank - 1], r.V_all[:, : r.rank - 1]
    e_less = np.linalg.norm(A - (Uk * sk) @ Vk.T) / math.sqrt(r.extra["fro2"])
    assert e_less > tau
    assert r.rank <= r.l - 10


def test_growth_limit_sets_flags():
    sigma = synth.spectrum_exp(600, 12.0)
    A = synth.general(700, 600, sigma, tag=78)
    r = rsvd_adaptive(A, 1e-6, 10, 1, block=32, seed=9, l_max=64)
    assert r.l == 64
    assert r.flags & FLAG_ADAPT_LIMIT
    assert r.flags & FLAG_RANK_CAPPED
    assert r.rank == 54


def test_basis_orthonormal():
    sigma = synth.spectrum_exp(500, 15.0)
    A = synth.general(520, 500, sigma, tag=79)
    r = rsvd_adaptive(A, 1e-7, 8, 1, block=40, seed=2)
    G = r.Q.T @ r.Q
    assert np.max(np.abs(G - np.eye(r.l))) <= 10 * r.l * U64


def test_symmetric_flag_only_substitutes_transpose():
    sigma = synth.spectrum_exp(300, 8.0)
    A = synth.symmetric(300, sigma, tag=80)
    a = rsvd_adaptive(A, 1e-6, 8, 1, block=32, seed=4, symmetric=True)
    b = rsvd_adaptive(A, 1e-6, 8, 1, block=32, seed=4, symmetric=False)
    assert a.l == b.l and a.rank == b.rank
    assert np.max(np.abs(a.s - b.s)) <= 1e-13


def test_zero_matrix():
    r = rsvd_adaptive(np.zeros((50, 40)), 1e-6, 4, 1, block=16, seed=1)
    assert r.l == 16
    assert r.rank == 1
    assert r.s[0] == 0.0


def test_fixed_run_posterior_judge_bounds_the_basis_error():
    # est = 10 sqrt(2/pi) max_j ||(I - QQ^T) A p_j|| over r = 10 fresh columns
    # bounds ||(I - QQ^T) A||_2 (failure probability 1e-10) and stays within
    # a modest factor of it
    from oracle.adaptive import FLAG_POSTERIOR_FAIL, FLAG_UNCONVERGED, posterior_judge
    from oracle.method import rsvd
    m, n = 300, 200
    sig = synth.spectrum_exp(n, 12.0)
    A = synth.general(m, n, sig, tag=131)
    for seed in range(20):
        r = rsvd(A, 30, 10, 1, seed=seed)
        est, flags = posterior_judge(A, r.Q, r.s_all, r.rank, 1, 1e-6, 10, seed=seed)
        true = np.linalg.norm(A - r.Q @ (r.Q.T @ A), 2)
        assert true <= est <= 200 * true
    # flags against their definitions: threshold rank of exp(-i/12) at 1e-3
    # is 83 (> l - p = 30 + 10 - 10 -> capped at 30; s_40/s_30 = e^(-10/12):
    # (0.43)^6 = 6e-3 > 1e-8 -> UNCONVERGED; est ~ s_41 > 1e-3 s_1 -> FAIL)
    r = rsvd(A, 30, 10, 1, seed=1, rank_mode="rel_threshold", rank_param=1e-3)
    est, flags = posterior_judge(A, r.Q, r.s_all, r.rank, 1, 1e-3, 10, seed=1)
    assert flags == FLAG_UNCONVERGED | FLAG_POSTERIOR_FAIL
    # a wide, converged basis passes: l = 150, q = 2, k = 83 (s_150/s_83 = e^(-67/12))
    r = rsvd(A, 100, 50, 2, seed=1, rank_mode="rel_threshold", rank_param=1e-3)
    est, flags = posterior_judge(A, r.Q, r.s_all, r.rank, 2, 1e-3, 10, seed=1)
    assert r.rank == 1 + int(12.0 * math.log(1e3)) and flags == 0
