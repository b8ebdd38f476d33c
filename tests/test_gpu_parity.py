"""End-to-end parity of the HIP randomized SVD with the CPU FP64 oracle
(same projection P, same p, q and QR-after-every-product schedule).

Gate (FP64): |ds_j| <= 1e-10 s_j + 1e-13 s_1 for every kept j, and
|de| <= 1e-10 e + 1e-13 for the residual e = ||A - U S V^T||_F / ||A||_F.
The absolute floors follow from Weyl's inequality: rounding A's products by
u ||A||_2 poly(n) moves every singular value by at most that much.
Singular vectors are compared up to sign where the gap to the neighbours is
large enough for them to be determined (tolerance ~ u s_1 / gap)."""

import numpy as np
import pytest

import synth
from oracle.method import rsvd as oracle_rsvd

from gpu_util import announce, sigma_gate, to_dev

pytestmark = pytest.mark.gpu


def _vec_tol(s_all, j):
    gaps = []
    if j > 0:
        gaps.append(s_all[j - 1] - s_all[j])
    if j + 1 < len(s_all):
        gaps.append(s_all[j] - s_all[j + 1])
    gap = min(gaps) if gaps else s_all[0]
    return 1e-12 * s_all[0] / max(gap, 1e-300) + 1e-12


def run_both(A, k, p, q, seed, *, symmetric=False, rank_mode="fixed", rank_param=None, omega=None,
             check_vectors=True, **kw):
    import paper_2307_15572_amd as rs
    ref = oracle_rsvd(A, k, p, q, seed=seed, symmetric=symmetric, rank_mode=rank_mode,
                      rank_param=rank_param, omega=omega)
    out = rs.run(to_dev(A), k, p, q, seed=seed, symmetric=symmetric, rank_mode=rank_mode,
                 rank_param=rank_param, omega=to_dev(omega) if omega is not None else None, **kw)
    s = out.S.cpu().numpy()
    kk = min(out.rank, ref.rank)
    ok, worst = sigma_gate(s[:kk], ref.s[:kk])
    assert ok, f"sigma gate failed: worst ratio {worst:.3g}"
    assert abs(out.residual - ref.residual) <= 1e-10 * ref.residual + 1e-13, (out.residual, ref.residual)
    assert out.l == ref.l
    assert abs(out.rel_percent - ref.rel_percent) < 1e-12 * 100 or out.rank != ref.rank
    if check_vectors:
        U = out.U.cpu().numpy()
        V = out.V.cpu().numpy()
        # the sign rule holds on the GPU output itself
        idx = np.argmax(np.abs(U), axis=0)
        assert np.all(U[idx, np.arange(U.shape[1])] > 0)
        for j in range(kk):
            tol = _vec_tol(ref.s_all, j)
            if tol > 1e-6:
                continue  # (nearly) degenerate: the vector is not determined
            du = min(np.abs(U[:, j] - ref.U[:, j]).max(), np.abs(U[:, j] + ref.U[:, j]).max())
            dv = min(np.abs(V[:, j] - ref.V[:, j]).max(), np.abs(V[:, j] + ref.V[:, j]).max())
            assert du <= tol and dv <= tol, (j, du, dv, tol)
    return out, ref


def test_c1_workload():
    A, sigma, w = synth.c1()
    announce(f"pipeline {w.name} k={w.k} p={w.p} q={w.q}")
    out, ref = run_both(A, w.k, w.p, w.q, w.seed)
    assert out.rank == w.k and out.l == w.k + w.p
    # the constructed spectrum is reached where the sketch has converged
    assert abs(out.S.cpu().numpy()[0] - sigma[0]) <= 1e-12


@pytest.mark.parametrize("m,n,k,p,q,decay", [
    (300, 170, 23, 7, 1, 1 / 10),      # ragged tiles in every dimension
    (200, 700, 30, 10, 2, 1 / 20),     # wide
    (3000, 400, 64, 16, 3, 1 / 64),    # tall, C3-like spectrum
    (1000, 1000, 100, 20, 0, 1 / 30),  # q = 0: the paper's method exactly
    (8192, 2048, 128, 16, 2, 1 / 40),  # A^T X as (X^T A)^T on the streaming kernel
])
def test_general_shapes(m, n, k, p, q, decay):
    announce(f"pipeline general {m}x{n} k={k} p={p} q={q}")
    sig = synth.spectrum_pow10(min(m, n), decay)
    A = synth.general(m, n, sig, tag=300 + m + n)
    run_both(A, k, p, q, seed=m * n)


@pytest.mark.parametrize("m,n,k,p,q,sym", [
    (1001, 1001, 41, 8, 2, True),   # odd n and odd l: copies of A and of every panel
    (1201, 777, 50, 13, 1, False),  # general with odd n and l
    (1500, 1500, 63, 16, 2, True),  # even n, odd l: the panel copies alone
])
def test_odd_sizes_through_even_copies(m, n, k, p, q, sym):
    # odd leading dimensions: the run streams an even-leading-dimension copy
    # of A and of each odd-width panel through the LDS-DMA kernel
    announce(f"pipeline odd sizes {m}x{n} k={k} p={p} q={q} symmetric={sym}")
    sig = synth.spectrum_pow10(min(m, n), 1 / 40)
    A = synth.symmetric(n, sig, tag=311 + n) if sym else synth.general(m, n, sig, tag=311 + n)
    run_both(A, k, p, q, seed=m + n, symmetric=sym)


@pytest.mark.parametrize("n,k,p", [(1025, 64, 16), (1500, 63, 16)])
def test_mixed_fp32_odd_sizes(n, k, p):
    # FP32 panels of odd width and an odd n (copy of A) in the FP32 schedule
    announce(f"mixed fp32 symmetric {n} k={k} p={p}")
    sig = synth.spectrum_pow10(n, 1 / 64)
    A = synth.symmetric(n, sig, tag=331 + n, noise=1e-9)
    rel, nrm, out, ref = _mixed_errors(A, k, p, 2, 17, True, "mixed_fp32", 1)
    assert rel <= 1e-6, rel


def test_symmetric_scaled_c2():
    n = 2048
    announce(f"pipeline symmetric {n} (C2 spectrum and noise)")
    A, sigma, w = synth.c2(n=n)
    out, ref = run_both(A, 256, 16, 2, 2002, symmetric=True)
    assert out.l == 272


@pytest.mark.parametrize("m,n,k,p", [(60, 40, 35, 10), (1, 1, 1, 0), (2, 3, 1, 5), (5, 1, 1, 1),
                                     (17, 17, 16, 1)])
def test_full_and_tiny(m, n, k, p):
    import paper_2307_15572_amd as rs
    announce(f"pipeline tiny/full {m}x{n} k={k} p={p}")
    sig = synth.spectrum_pow10(min(m, n), 0.2)
    A = synth.general(m, n, sig, tag=400 + m * 7 + n)
    out, ref = run_both(A, k, p, 1, seed=3)
    if out.l == min(m, n):
        assert out.flags & rs.FLAG_FULL_SVD


def test_threshold_percent_frobtail_rules():
    n, d = 800, 20.0
    sig = synth.spectrum_exp(n, d)
    A = synth.symmetric(n, sig, tag=501)
    announce("rank rule rel_threshold")
    out, ref = run_both(A, 300, 32, 2, 9, symmetric=True, rank_mode="rel_threshold", rank_param=1e-6,
                        check_vectors=False)
    # threshold ties: a value within the sigma gate of tau s_1 may fall either way
    s = ref.s_all
    near = np.abs(s - 1e-6 * s[0]) <= 1e-10 * s + 1e-13 * s[0]
    assert out.rank == ref.rank or near.any()
    announce("rank rule percent")
    run_both(A, 0, 16, 2, 9, symmetric=True, rank_mode="percent", rank_param=5.0, check_vectors=False)
    announce("rank rule frob_tail")
    out, ref = run_both(A, 300, 32, 2, 9, symmetric=True, rank_mode="frob_tail", rank_param=1e-4,
                        check_vectors=False)
    assert out.rank == ref.rank


@pytest.mark.parametrize("form", ["svd", "symmetric"])
def test_values_only_equals_full_run(form):
    # without vectors or residual the small SVD skips its right rotations and
    # the lift is skipped: the values, the rank and the flags are unchanged
    # (the rows of the Jacobi matrix never depend on the rotations kept
    # beside them), bit for bit
    import paper_2307_15572_amd as rs
    n, d = 1400, 25.0
    A = to_dev(synth.symmetric(n, synth.spectrum_exp(n, d), tag=502))
    announce(f"values-only run vs full run, {form} form")
    kw = dict(seed=12, symmetric=True, rank_mode="rel_threshold", rank_param=1e-6, form=form)
    full = rs.run(A, 400, 48, 2, **kw)
    vals = rs.run(A, 400, 48, 2, want_u=False, want_v=False, want_residual=False, **kw)
    assert vals.rank == full.rank and vals.flags == full.flags
    assert vals.sweeps == full.sweeps
    assert np.array_equal(vals.S.cpu().numpy(), full.S.cpu().numpy())
    ref = oracle_rsvd(synth.symmetric(n, synth.spectrum_exp(n, d), tag=502), 400, 48, 2, seed=12,
                      symmetric=True, rank_mode="rel_threshold", rank_param=1e-6,
                      want_residual=False) if form == "svd" else None
    if ref is not None:
        assert vals.rank == ref.rank
        ok, worst = sigma_gate(vals.S.cpu().numpy(), ref.s)
        assert ok, worst


def test_oversampled_past_the_fp64_floor():
    # a steep spectrum sketched with much more than its numerical rank
    # (sigma_l / sigma_1 ~ 1e-14, q = 0): the unshifted Cholesky QR breaks
    # down and the shifted passes build the basis; the kept values and the
    # rank still match the oracle's (LAPACK QR)
    n, d = 2000, 14.7
    A = synth.symmetric(n, synth.spectrum_exp(n, d), tag=505)
    announce(f"pipeline steep spectrum n={n} d={d} k=261 p=192 q=0")
    out, ref = run_both(A, 261, 192, 0, 11, symmetric=True, rank_mode="rel_threshold",
                        rank_param=1e-6, check_vectors=False)
    assert out.rank == ref.rank


def test_exact_low_rank_on_gpu():
    import paper_2307_15572_amd as rs
    announce("pipeline exact rank 5")
    A, s = synth.rank_r(120, 90, 5, tag=104, scale=3.0)
    out = rs.run(to_dev(A), 10, 5, 1, seed=3)
    S = out.S.cpu().numpy()
    assert np.all(np.abs(S[:5] - s) <= 1e-13 * s[0])
    assert np.all(S[5:] <= 1e-13 * s[0])
    assert out.residual <= 1e-13


def test_caller_omega_and_determinism():
    import paper_2307_15572_amd as rs
    from oracle.philox import gaussian_omega
    announce("caller omega / determinism")
    sig = synth.spectrum_exp(400, 12.0)
    A = synth.general(500, 400, sig, tag=601)
    om = np.random.default_rng(1).standard_normal((400, 40))
    run_both(A, 30, 10, 2, seed=0, omega=om)
    o1 = rs.run(to_dev(A), 30, 10, 2, seed=44)
    o2 = rs.run(to_dev(A), 30, 10, 2, seed=44)
    assert np.array_equal(o1.S.cpu().numpy(), o2.S.cpu().numpy())
    assert np.array_equal(o1.U.cpu().numpy(), o2.U.cpu().numpy())
    o3 = rs.run(to_dev(A), 30, 10, 2, omega=to_dev(gaussian_omega(400, 40, 44)))
    assert np.max(np.abs(o3.S.cpu().numpy() - o1.S.cpu().numpy())) <= 1e-13


def test_nonfinite_input_raises():
    import paper_2307_15572_amd as rs
    announce("non-finite input")
    A = np.ones((50, 40))
    A[7, 3] = np.nan
    with pytest.raises(rs.RsvdError, match="NaN"):
        rs.run(to_dev(A), 5, 5, 1)


def _mixed_errors(A, k, p, q, seed, symmetric, precision, trailing_hp):
    import paper_2307_15572_amd as rs
    ref = oracle_rsvd(A, k, p, q, seed=seed, symmetric=symmetric)
    out = rs.run(to_dev(A), k, p, q, seed=seed, symmetric=symmetric, precision=precision,
                 trailing_hp=trailing_hp)
    s = out.S.cpu().numpy()
    kk = min(out.rank, ref.rank)
    rel = np.abs(s[:kk] - ref.s[:kk]) / ref.s[:kk]
    return rel.max(), np.abs(s[:kk] - ref.s[:kk]).max() / ref.s[0], out, ref


@pytest.mark.parametrize("thp", [0, 1])
def test_mixed_fp32_meets_1e6_gate(thp):
    # FP32 early products, FP64 projection / QR / SVD: every kept singular value
    # within 1e-6 relative of the FP64 oracle (same P, p, q)
    n = 2048
    announce(f"mixed fp32 symmetric {n}, trailing_hp={thp}")
    A, sigma, w = synth.c2(n=n)
    rel, nrm, out, ref = _mixed_errors(A, 256, 16, 2, 2002, True, "mixed_fp32", thp)
    assert rel <= 1e-6, rel
    assert abs(out.residual - ref.residual) <= 1e-6 * ref.residual


@pytest.mark.parametrize("n", [2048, 1025])
def test_mixed_fp32_sliced_meets_1e6_gate(n):
    # FP32 early products, the trailing product and the projection as
    # error-free sliced products: every kept value within 1e-6 of the FP64
    # oracle, and within 1e-10 of the schedule with FP64 trailing products
    # (the same FP32 products before them)
    import paper_2307_15572_amd as rs
    announce(f"mixed fp32 + sliced trailing products, symmetric {n}")
    if n == 2048:
        A, sigma, w = synth.c2(n=n)
        k, p, q, seed = 256, 16, 2, 2002
    else:
        A = synth.symmetric(n, synth.spectrum_pow10(n, 1 / 64), tag=341, noise=1e-9)
        k, p, q, seed = 64, 15, 2, 17
    rel, nrm, out, ref = _mixed_errors(A, k, p, q, seed, True, "mixed_fp32_sliced", 1)
    assert rel <= 1e-6, rel
    assert abs(out.residual - ref.residual) <= 1e-6 * ref.residual
    f64t = rs.run(to_dev(A), k, p, q, seed=seed, symmetric=True, precision="mixed_fp32",
                  trailing_hp=1)
    s1, s2 = out.S.cpu().numpy(), f64t.S.cpu().numpy()
    kk = min(len(s1), len(s2))
    assert np.max(np.abs(s1[:kk] - s2[:kk]) / s2[:kk]) <= 1e-10


def test_mixed_fp32_general_tall():
    announce("mixed fp32 general 3000 x 400")
    sig = synth.spectrum_pow10(400, 1 / 64)
    A = synth.general(3000, 400, sig, tag=701, noise=1e-9)
    rel, nrm, out, ref = _mixed_errors(A, 64, 16, 3, 5, False, "mixed_fp32", 1)
    assert rel <= 1e-6, rel


def test_mixed_fp32_general_transposed_stream():
    # FP32 early products, A^T X taken as (X^T A)^T on the streaming kernel
    announce("mixed fp32 general 8192 x 2048")
    sig = synth.spectrum_pow10(2048, 1 / 20)
    A = synth.general(8192, 2048, sig, tag=703, noise=1e-9)
    rel, nrm, out, ref = _mixed_errors(A, 128, 16, 3, 5, False, "mixed_fp32", 1)
    assert rel <= 1e-6, rel


def test_mixed_bf16_error_level():
    # BF16 early products (u = 2^-8) leave the unconverged tail off by ~1e-3
    # relative; the normwise error stays at u_bf16 * sigma-ratio level and the
    # residual within 1e-3 relative. This mode does not meet the 1e-6 gate.
    n = 2048
    announce("mixed bf16 symmetric 2048")
    A, sigma, w = synth.c2(n=n)
    rel, nrm, out, ref = _mixed_errors(A, 256, 16, 2, 2002, True, "mixed_bf16", 2)
    assert nrm <= 1e-5
    assert rel <= 1e-2
    assert abs(out.residual - ref.residual) <= 1e-3 * ref.residual


def test_tall_full_size_properties():
    # the 131072 x 8192 workload at full size, where the oracle cannot run:
    # (i) the leading values (converged: (sigma_528/sigma_255)^7 ~ 1e-19) equal
    #     the constructed spectrum up to the noise floor (Weyl: |ds| <= ||E||_2
    #     ~ 1e-9) and FP64 rounding;
    # (ii) no value exceeds the constructed one by more than that bound
    #     (interlacing: s_j(Q^T A) <= s_j(A) <= sigma_j + ||E||_2);
    # (iii) U and V orthonormal; the residual matches sqrt(1 - sum s^2 / ||A||^2)
    #     to the noise floor's share (Pythagoras with U S V^T = Q Q^T A P_k)
    import torch
    import paper_2307_15572_amd as rs
    announce("tall 131072 x 8192 full size, FP64, properties")
    A, sigma, w = synth.c3_device(device="cuda:0")
    out = rs.run(A, w.k, w.p, w.q, seed=w.seed, want_residual=True)
    s = out.S.cpu().numpy()
    assert out.rank == 512 and out.l == 528
    lead = 256
    assert np.all(np.abs(s[:lead] - sigma[:lead]) <= 2e-9 + 1e-10 * sigma[:lead])
    assert np.all(s <= sigma[: len(s)] + 2e-9 + 1e-13)
    U, V = out.U, out.V
    eye = torch.eye(512, dtype=torch.float64, device=A.device)
    assert (U.T @ U - eye).abs().max().item() <= 1e-12
    assert (V.T @ V - eye).abs().max().item() <= 1e-12
    fro2 = out.fro2
    pyth = np.sqrt(max(1.0 - np.sum(s ** 2) / fro2, 0.0))
    assert abs(out.residual - pyth) <= 1e-6
    del A
    torch.cuda.empty_cache()
