"""Parity of the HIP adaptive range finder with the CPU FP64 oracle
(oracle/adaptive.py): same projection stream, block size, p and q.

The growth decisions (l_used, blocks) and the rank are integers and must be
equal; the cases keep the posterior estimate well away from its stopping
bound at every step (it falls by more than 10x per block), so rounding
cannot flip a decision. Singular values meet the FP64 gate
|ds_j| <= 1e-10 s_j + 1e-13 s_1. The error estimate is the norm of a deflated
residual W = (I - QQ^T) A P_blk of size ~tau s_1: a perturbation of the basis
by u moves it by ~u ||A P_blk|| / ||W||, so it is compared to 1e-4 relative.
"""

import numpy as np
import pytest

import synth
from oracle.adaptive import FLAG_ADAPT_LIMIT, rsvd_adaptive

from gpu_util import announce, sigma_gate, to_dev

pytestmark = pytest.mark.gpu


def run_both(A, tau, p, q, block, seed, *, symmetric=False, rank_mode="rel_threshold",
             l_max=None, check_vectors=True):
    import paper_2307_15572_amd as rs
    ref = rsvd_adaptive(A, tau, p, q, block=block, seed=seed, symmetric=symmetric,
                        l_max=l_max, rank_mode=rank_mode)
    out = rs.run(to_dev(A), 0, p, q, seed=seed, symmetric=symmetric, rank_mode=rank_mode,
                 rank_param=tau, adaptive=True, block=block, l_max=l_max or 0)
    assert out.l == ref.l, (out.l, ref.l)
    assert out.blocks == ref.extra["blocks"]
    assert out.rank == ref.rank
    # the oracle's LAPACK QR has no fallback path, so QR_FALLBACK is not compared
    assert out.flags & ~rs.FLAG_QR_FALLBACK == ref.flags, (out.flags, ref.flags)
    s = out.S.cpu().numpy()
    ok, worst = sigma_gate(s, ref.s)
    assert ok, f"sigma gate failed: worst ratio {worst:.3g}"
    assert abs(out.residual - ref.residual) <= 1e-10 * ref.residual + 1e-13
    est_ref = ref.extra["est"]
    # estimates at rounding level (exact low rank) only need to stay there
    assert abs(out.err_est - est_ref) <= 1e-4 * est_ref + 1e-12 * ref.s[0], (out.err_est, est_ref)
    if check_vectors:
        U = out.U.cpu().numpy()
        idx = np.argmax(np.abs(U), axis=0)
        assert np.all(U[idx, np.arange(U.shape[1])] > 0)
        # leading, well-separated vectors agree with the oracle's (same sign rule)
        kk = min(8, out.rank)
        assert np.abs(U[:, :kk] - ref.U[:, :kk]).max() <= 1e-9
        V = out.V.cpu().numpy()
        assert np.abs(V[:, :kk] - ref.V[:, :kk]).max() <= 1e-9
    return out, ref


def test_threshold_symmetric_exp_spectrum():
    # a C4-like channel: exp(-i/d) decay, tau = 1e-6
    n, d = 1500, 20.0
    announce(f"adaptive threshold symmetric n={n} d={d}")
    A = synth.symmetric(n, synth.spectrum_exp(n, d), tag=90, channel=1)
    out, ref = run_both(A, 1e-6, 16, 1, 64, 31, symmetric=True)
    assert out.rank == int(np.count_nonzero(synth.spectrum_exp(n, d) >= 1e-6))


def test_threshold_general_q0_ragged_block():
    # block 48, q = 0, tall general matrix
    announce("adaptive threshold general 2200 x 700 q=0 b=48")
    sigma = synth.spectrum_pow10(700, 1.0 / 24.0)
    A = synth.general(2200, 700, sigma, tag=91)
    run_both(A, 1e-7, 10, 0, 48, 32)


def test_frobenius_rule_general():
    announce("adaptive frob_tail general 1800 x 900")
    sigma = synth.spectrum_exp(900, 15.0)
    A = synth.general(1800, 900, sigma, tag=92)
    out, ref = run_both(A, 1e-4, 10, 1, 32, 33, rank_mode="frob_tail")
    assert out.residual <= 1e-4 * (1 + 1e-8)


def test_exact_low_rank_one_block():
    announce("adaptive exact rank 7, 2000 x 900")
    A, s = synth.rank_r(2000, 900, 7, tag=93)
    out, ref = run_both(A, 1e-9, 8, 1, 32, 34)
    assert out.l == 32 and out.blocks == 1 and out.rank == 7


def test_growth_limit():
    announce("adaptive l_max = 128")
    sigma = synth.spectrum_exp(900, 40.0)
    A = synth.general(1000, 900, sigma, tag=94)
    out, ref = run_both(A, 1e-6, 16, 1, 64, 35, l_max=128, check_vectors=False)
    assert out.flags & FLAG_ADAPT_LIMIT
    assert out.l == 128 and out.rank == 112
