"""Per-kernel parity on the GPU: projection P, FP64 GEMM, QR, small SVD."""

import numpy as np
import pytest

from oracle.philox import gaussian_omega as oracle_omega
from oracle.method import orth as oracle_orth
import synth

from gpu_util import announce, bf16_round, to_dev

pytestmark = pytest.mark.gpu

U_EPS = 2.0 ** -53


@pytest.mark.parametrize("n,l,col0,seed,ch", [(1000, 50, 0, 2001, 0), (37, 13, 5, 7, 3),
                                                (4096, 272, 0, 2002, 0), (1, 1, 0, 0, 0)])
def test_omega_matches_oracle(n, l, col0, seed, ch):
    import paper_2307_15572_amd as rs
    announce(f"omega n={n} l={l} col0={col0}")
    g = rs.gaussian_omega(n, l, seed, ch, col0=col0).cpu().numpy()
    ref = oracle_omega(n, l, seed, ch, col0=col0)
    # same Philox words; transcendental functions may differ by an ulp or two
    assert np.all(np.abs(g - ref) <= 8 * U_EPS * (np.abs(ref) + 1.0))


GEMM_CASES = [
    (False, 64, 16, 16), (False, 1, 1, 1), (False, 130, 50, 77), (False, 517, 272, 1000),
    (False, 300, 528, 257), (False, 2048, 272, 8192), (False, 64, 300, 20000),
    (True, 50, 50, 512), (True, 272, 272, 16384), (True, 1000, 33, 999), (True, 40, 7, 3),
    # A^T B on the LDS-DMA kernel with A in its stored orientation: ragged
    # row tiles (columns of A clamped), the smallest even M, several column
    # blocks, split K; odd M takes the register-staged kernel
    (True, 130, 50, 4096), (True, 2, 20, 64), (True, 600, 600, 2048), (True, 3000, 528, 16384),
    (True, 131, 40, 256),
]


@pytest.mark.parametrize("ta,m,n,k", GEMM_CASES)
def test_dgemm_matches_numpy(ta, m, n, k):
    import paper_2307_15572_amd as rs
    announce(f"dgemm ta={ta} m={m} n={n} k={k}")
    rng = np.random.default_rng(m * 7 + n * 3 + k)
    A = rng.standard_normal((k, m) if ta else (m, k))
    B = rng.standard_normal((k, n))
    C0 = rng.standard_normal((m, n))
    ref = (A.T if ta else A) @ B
    got = rs.dgemm(to_dev(A), to_dev(B), trans_a=ta).cpu().numpy()
    # componentwise FP64 error bound for a k-term dot product
    scale = (np.abs(A.T if ta else A) @ np.abs(B))
    assert np.all(np.abs(got - ref) <= 2 * k * U_EPS * scale + 1e-300)
    got2 = rs.dgemm(to_dev(A), to_dev(B), trans_a=ta, alpha=-0.5, beta=2.0, C=to_dev(C0)).cpu().numpy()
    ref2 = -0.5 * ref + 2.0 * C0
    assert np.all(np.abs(got2 - ref2) <= 2 * k * U_EPS * (0.5 * scale + 2 * np.abs(C0)) + 1e-300)


@pytest.mark.parametrize("m,l,decay", [(500, 50, 1 / 16), (4096, 272, 1 / 40), (3000, 100, 1 / 8),
                                       (200, 200, 1 / 64), (20, 1, 0.1), (2000, 528, 1 / 64),
                                       (1500, 33, 0.05), (2600, 1250, 1 / 200), (3000, 257, 1 / 40),
                                       (700, 16, 0.1), (900, 17, 0.05), (5000, 271, 1 / 50),
                                       # 273..320: grid Cholesky with diagonal-tile inverses
                                       # only, then the block triangular solve
                                       (4096, 288, 1 / 40), (6000, 320, 1 / 50),
                                       # 321..608: the wide substitution kernel; 609: the
                                       # full inverse and a product
                                       (5000, 400, 1 / 80), (4000, 608, 1 / 150),
                                       (3000, 609, 1 / 150)])
def test_orth_matches_oracle(m, l, decay):
    import paper_2307_15572_amd as rs
    announce(f"orth m={m} l={l} decay={decay}")
    rng = np.random.default_rng(m + l)
    # panel with graded columns: condition number about 10^(decay * l)
    U = synth.haar_columns(m, l, rng)
    V = synth.haar_columns(l, l, rng)
    Y = (U * (10.0 ** (-decay * np.arange(l)))) @ V.T
    Q, X, flags = rs.orth(to_dev(Y))
    Q = Q.cpu().numpy()
    X = X.cpu().numpy()
    assert np.abs(Q.T @ Q - np.eye(l)).max() <= 20 * l * U_EPS
    assert np.abs(Q @ X - Y).max() <= 50 * l * U_EPS * np.abs(Y).max()
    assert np.all(np.diag(X) > 0) and np.allclose(np.tril(X, -1), 0)
    # diag(R) > 0 makes Q unique: compare with the oracle's Householder Q
    Qref = oracle_orth(Y)
    kappa = 10.0 ** (decay * (l - 1))
    assert np.abs(Q - Qref).max() <= 1e3 * kappa * U_EPS + 1e-12


@pytest.mark.parametrize("m,l,scale", [(4000, 272, 1.0), (3000, 130, 1e-3), (2000, 17, 1.0),
                                         (5000, 400, 1.0), (3000, 609, 1e2)])
def test_orth_of_orthonormal_panel(m, l, scale):
    # a panel with orthonormal columns times a diagonal close to one: the
    # second Cholesky pass sees a Gram within 2^-33 of the identity and takes
    # the first-order factor (one workgroup up to l = 272, the predicated
    # grid path beyond); Q, X must still meet the same bounds
    import paper_2307_15572_amd as rs
    announce(f"orth of a near-orthonormal panel m={m} l={l} scale={scale}")
    rng = np.random.default_rng(m + 7 * l)
    U = synth.haar_columns(m, l, rng)
    d = 1.0 + 1e-3 * rng.uniform(-1.0, 1.0, l)
    Y = scale * U * d
    Q, X, flags = rs.orth(to_dev(Y))
    Q = Q.cpu().numpy()
    X = X.cpu().numpy()
    assert np.abs(Q.T @ Q - np.eye(l)).max() <= 20 * l * U_EPS
    assert np.abs(Q @ X - Y).max() <= 50 * l * U_EPS * np.abs(Y).max()
    assert np.all(np.diag(X) > 0) and np.allclose(np.tril(X, -1), 0)
    # Q is unique (diag(X) > 0): the oracle's Householder Q
    assert np.abs(Q - oracle_orth(Y)).max() <= 1e-12


def test_orth_numerically_rank_deficient():
    # rank-6 product: the shifted three-pass Cholesky QR still returns an
    # orthonormal Q whose span contains the panel (noise directions complete it)
    import paper_2307_15572_amd as rs
    announce("orth numerically rank-deficient 300 x 40 (rank 6)")
    rng = np.random.default_rng(5)
    Y = rng.standard_normal((300, 6)) @ rng.standard_normal((6, 40))
    Q, X, flags = rs.orth(to_dev(Y))
    Q = Q.cpu().numpy()
    X = X.cpu().numpy()
    assert np.abs(Q.T @ Q - np.eye(40)).max() <= 1e-12
    assert np.abs(Q @ X - Y).max() <= 1e-12 * np.abs(Y).max()


def test_orth_exactly_rank_deficient_uses_householder():
    # exactly zero columns make every Cholesky pass break down: Householder QR
    import paper_2307_15572_amd as rs
    announce("orth exact zero columns 300 x 40")
    rng = np.random.default_rng(6)
    Y = rng.standard_normal((300, 40))
    Y[:, 25:] = 0.0
    Q, X, flags = rs.orth(to_dev(Y))
    Q = Q.cpu().numpy()
    X = X.cpu().numpy()
    assert flags & rs.FLAG_QR_FALLBACK
    assert np.abs(Q.T @ Q - np.eye(40)).max() <= 1e-13
    assert np.abs(Q @ X - Y).max() <= 1e-13 * np.abs(Y).max()
    assert np.all(np.diag(X) >= 0) and np.allclose(np.tril(X, -1), 0)
    # the first 25 columns are the unique QR of the nonzero part
    assert np.abs(Q[:, :25] - oracle_orth(Y[:, :25])).max() <= 1e-12


@pytest.mark.parametrize("rows,l,rank", [(3000, 300, 8), (1500, 96, 40), (700, 128, 0), (16384, 272, 100),
                                         (5000, 304, 50)])
def test_orth_rank_deficient_large_panel_grid_householder(rows, l, rank):
    # panels past the one-workgroup size take the fallback on a grid of
    # workgroups: same contract (orthonormal Q, Q X = Y, diag(X) >= 0)
    import paper_2307_15572_amd as rs
    announce(f"orth rank-deficient {rows} x {l} (rank {rank}), grid Householder")
    rng = np.random.default_rng(rows + l)
    if rank:
        Y = rng.standard_normal((rows, rank)) @ rng.standard_normal((rank, l))
        Y[:, l - 5:] = 0.0
    else:
        Y = np.zeros((rows, l))
        Y[:, 3] = rng.standard_normal(rows)
    Q, X, flags = rs.orth(to_dev(Y))
    Q = Q.cpu().numpy()
    X = X.cpu().numpy()
    assert flags & rs.FLAG_QR_FALLBACK
    assert np.abs(Q.T @ Q - np.eye(l)).max() <= 1e-12
    assert np.abs(Q @ X - Y).max() <= 1e-12 * max(np.abs(Y).max(), 1.0)
    assert np.all(np.diag(X) >= 0) and np.allclose(np.tril(X, -1), 0)


@pytest.mark.parametrize("l,decay", [(50, 1 / 16), (272, 1 / 40), (17, 0.5), (1, 0.0), (128, 1 / 20),
                                     (528, 1 / 64), (300, 1 / 30), (1250, 1 / 200)])
def test_small_svd_matches_lapack(l, decay):
    import paper_2307_15572_amd as rs
    announce(f"small_svd l={l}")
    rng = np.random.default_rng(l)
    U = synth.haar_columns(l, l, rng)
    V = synth.haar_columns(l, l, rng)
    sig = 10.0 ** (-decay * np.arange(l))
    R = np.triu(np.linalg.qr((U * sig) @ V.T)[1])
    s, Us, W, sweeps, flags = rs.small_svd(to_dev(R))
    s = s.cpu().numpy()
    Us = Us.cpu().numpy()
    W = W.cpu().numpy()
    assert not (flags & rs.FLAG_JACOBI_MAXSWEEP)
    ref = np.linalg.svd(R, compute_uv=False)
    assert np.all(np.abs(s - ref) <= 1e-13 * ref[0] + 1e-12 * ref)
    assert np.all(np.diff(s) <= 0)
    # R^T = Us diag(s) W^T with orthonormal Us, W
    assert np.abs(R.T - (Us * s) @ W.T).max() <= 1e-13 * ref[0] * max(1, l / 10)
    # orthonormality to 10 l u (accumulated rotations), at least 1e-12
    orth_tol = max(1e-12, 10 * l * 1.1102230246251565e-16)
    assert np.abs(Us.T @ Us - np.eye(l)).max() <= orth_tol
    assert np.abs(W.T @ W - np.eye(l)).max() <= orth_tol


@pytest.mark.parametrize("scale", [1e150, 1e-140])
def test_small_svd_extreme_scale(scale):
    # Gram entries from 1e300 down to 1e-290: the rotations are formed from
    # (d, e) scaled by a power of two, so no square or product over- or
    # underflows (the row Grams themselves must stay in the normal range: the
    # smallest singular value here is 1e-5 of the largest)
    import paper_2307_15572_amd as rs
    announce(f"small_svd extreme scale {scale:g}")
    l = 100
    rng = np.random.default_rng(7)
    U = synth.haar_columns(l, l, rng)
    V = synth.haar_columns(l, l, rng)
    R = np.triu(np.linalg.qr((U * 10.0 ** (-np.arange(l) / 20)) @ V.T)[1]) * scale
    s, Us, W, sweeps, flags = rs.small_svd(to_dev(R))
    s = s.cpu().numpy()
    assert not (flags & rs.FLAG_JACOBI_MAXSWEEP)
    ref = np.linalg.svd(R, compute_uv=False)
    assert np.all(np.isfinite(s))
    assert np.all(np.abs(s - ref) <= 1e-13 * ref[0] + 1e-12 * ref)


def test_small_svd_equal_row_norms():
    # blocks [[3, 4], [0, 5]]: rows of equal norm, so h_qq - h_pp is exactly
    # zero for those pairs (a 45-degree rotation); singular values sqrt(45),
    # sqrt(5) per block, times the block's scale
    import paper_2307_15572_amd as rs
    announce("small_svd equal row norms")
    nb = 17
    l = 2 * nb
    R = np.zeros((l, l))
    scales = 2.0 ** np.arange(nb)
    for i in range(nb):
        R[2 * i:2 * i + 2, 2 * i:2 * i + 2] = scales[i] * np.array([[3.0, 4.0], [0.0, 5.0]])
    s, Us, W, sweeps, flags = rs.small_svd(to_dev(R))
    s = s.cpu().numpy()
    assert not (flags & rs.FLAG_JACOBI_MAXSWEEP)
    ref = np.sort(np.concatenate([scales * np.sqrt(45.0), scales * np.sqrt(5.0)]))[::-1]
    assert np.all(np.abs(s - ref) <= 1e-14 * ref)


LOWP_CASES = [("mixed_fp32", False, 517, 272, 1000), ("mixed_fp32", False, 2048, 272, 8192),
              ("mixed_fp32", True, 272, 272, 4096), ("mixed_fp32", False, 100, 50, 77),
              ("mixed_bf16", False, 517, 272, 1000), ("mixed_bf16", False, 2048, 272, 8192),
              ("mixed_bf16", True, 300, 100, 2000), ("mixed_bf16", False, 33, 18, 16),
              ("mixed_bf16_split", False, 517, 272, 1000), ("mixed_bf16_split", False, 2048, 272, 8192),
              ("mixed_bf16_split", True, 300, 100, 2000), ("mixed_bf16_split", False, 33, 18, 16)]


@pytest.mark.parametrize("prec,ta,m,n,k", LOWP_CASES)
def test_lowp_gemm_error_bound(prec, ta, m, n, k):
    # operands rounded to the format (unit roundoff u_in) and products summed in
    # FP32 (u32): |C - C_ref| <= (2 u_in + (k + 2) u32) (|A| |B|) componentwise
    import paper_2307_15572_amd as rs
    announce(f"gemm {prec} ta={ta} m={m} n={n} k={k}")
    rng = np.random.default_rng(m + 3 * n + 7 * k)
    A = rng.standard_normal((k, m) if ta else (m, k))
    B = rng.standard_normal((k, n))
    opA = A.T if ta else A
    ref = opA @ B
    got = rs.dgemm(to_dev(A), to_dev(B), trans_a=ta, precision=prec).cpu().numpy()
    u32 = 2.0 ** -24
    if prec == "mixed_bf16_split":
        # x = hi + lo to 2^-17 |x|, the dropped lo*lo term 2^-16 |a b|, and three
        # products summed in FP32 per term
        bound = (2.0 ** -15 + (3 * k + 2) * u32) * (np.abs(opA) @ np.abs(B))
    else:
        u_in = 2.0 ** -24 if prec == "mixed_fp32" else 2.0 ** -8
        bound = (2 * u_in + (k + 2) * u32) * (np.abs(opA) @ np.abs(B))
    assert np.all(np.abs(got - ref) <= bound)
    # and it is not secretly FP64: the error is at the format's level
    if prec == "mixed_bf16" and k >= 1000:
        assert np.abs(got - ref).max() > 1e3 * 2.0 ** -53 * np.abs(ref).max()


# (trans_a, m, n, k): row tiles of 128 and 256 rows with ragged tails, one and
# several column groups, k padded to 64, split K with FP32 partials
BF16_PLANE_CASES = [
    (False, 517, 272, 1000), (False, 2048, 272, 8192), (True, 300, 100, 2000), (False, 33, 18, 16),
    (False, 1, 1, 1), (False, 129, 17, 65), (False, 5000, 528, 3000), (True, 2048, 8, 20000),
    (False, 2600, 300, 700), (True, 1000, 33, 999),
]


@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("ta,m,n,k", BF16_PLANE_CASES)
def test_bf16_planes_gemm(split, ta, m, n, k):
    # the rounded operands multiply exactly in FP32; the only error left is
    # the FP32 accumulation: |C - P X| <= (k + 2) u32 (|P| |X|) per entry,
    # P, X the BF16 operands (split: hi hi + hi lo + lo hi, lo lo dropped)
    import paper_2307_15572_amd as rs
    announce(f"bf16 planes gemm split={split} ta={ta} m={m} n={n} k={k}")
    rng = np.random.default_rng(11 * m + 5 * n + k + split)
    A = rng.standard_normal((k, m) if ta else (m, k))
    B = rng.standard_normal((k, n))
    opA = A.T if ta else A
    got = rs.bf16_gemm(to_dev(A), to_dev(B), trans_a=ta, split=split).cpu().numpy()
    ah, bh = bf16_round(opA), bf16_round(B)
    if split:
        al, bl = bf16_round(opA - ah), bf16_round(B - bh)
        ref = ah @ bh + ah @ bl + al @ bh
        mag = np.abs(ah) @ np.abs(bh) + np.abs(ah) @ np.abs(bl) + np.abs(al) @ np.abs(bh)
        terms = 3 * k
    else:
        ref = ah @ bh
        mag = np.abs(ah) @ np.abs(bh)
        terms = k
    u32 = 2.0 ** -24
    assert np.all(np.abs(got - ref) <= (terms + 2) * u32 * mag)
    # and the operand rounding is the format's: against the FP64 product
    exact = opA @ B
    u_in = 2.0 ** -15 if split else 2.0 ** -8
    assert np.all(np.abs(got - exact) <= (2 * u_in + (terms + 2) * u32) * (np.abs(opA) @ np.abs(B)))


def test_sliced_product_exact_on_small_integers():
    # integers of at most 7 bits fit one slice each: the slice product is the
    # exact product, so C equals A B (exact in FP64 here) bitwise
    import torch
    import paper_2307_15572_amd as rs
    announce("sliced product, integer inputs, 333 x 1001 x 70")
    g = torch.Generator().manual_seed(21)
    A = torch.randint(-100, 101, (333, 1001), generator=g).double()
    B = torch.randint(-100, 101, (1001, 70), generator=g).double()
    C = rs.dgemm(to_dev(A.numpy()), to_dev(B.numpy()), precision="mixed_fp32_sliced")
    assert torch.equal(C.cpu(), A @ B)


@pytest.mark.parametrize("m,n,k", [(700, 130, 1001), (1024, 272, 4096), (65, 17, 33)])
def test_sliced_product_error_bound(m, n, k):
    # random FP64 operands whose rows and columns span many binades: every
    # entry within 4e-14 k max_k |a_ik| max_k |b_kj| of the exact product
    # (numpy FP64 products differ from it by far less), and far closer than
    # an FP32 product would be
    import paper_2307_15572_amd as rs
    announce(f"sliced product error bound {m} x {n} x {k}")
    rng = np.random.default_rng(m + n + k)
    A = rng.standard_normal((m, k)) * np.exp2(rng.integers(-30, 30, size=(m, 1)))
    B = rng.standard_normal((k, n)) * np.exp2(rng.integers(-30, 30, size=(1, n)))
    C = rs.dgemm(to_dev(A), to_dev(B), precision="mixed_fp32_sliced").cpu().numpy()
    ref = A @ B
    scale = k * np.abs(A).max(axis=1)[:, None] * np.abs(B).max(axis=0)[None, :]
    err = np.abs(C - ref) / scale
    assert err.max() <= 4e-14, err.max()
    C32 = rs.dgemm(to_dev(A), to_dev(B), precision="mixed_fp32").cpu().numpy()
    assert err.max() < 1e-5 * (np.abs(C32 - ref) / scale).max()


@pytest.mark.parametrize("m,n,k", [(1000, 777, 272), (300, 5000, 259), (129, 17, 16), (5000, 40, 1),
                                   (600, 2000, 300), (4096, 4096, 256), (700, 900, 190)])
def test_residual_pass_matches_numpy(m, n, k):
    # ||A - U_k S_k V_k^T||_F / ||A||_F against the same sums in numpy; inner
    # sizes up to 272 (k padded to 16) keep U diag(s) in registers, wider
    # ones take the streaming kernel; ragged row strips and column slices
    import paper_2307_15572_amd as rs
    announce(f"residual pass m={m} n={n} k={k}")
    rng = np.random.default_rng(m * 7 + n * 3 + k)
    U = np.linalg.qr(rng.standard_normal((m, k)))[0] if k <= m else rng.standard_normal((m, k))
    V = np.linalg.qr(rng.standard_normal((n, k)))[0] if k <= n else rng.standard_normal((n, k))
    S = np.sort(rng.uniform(0.5, 2.0, k))[::-1].copy()
    A = (U * S) @ V.T + 1e-3 * rng.standard_normal((m, n))
    out = rs.residual(to_dev(A), to_dev(S), to_dev(U), to_dev(V), k)
    ref = np.linalg.norm(A - (U * S) @ V.T) / np.linalg.norm(A)
    assert abs(out.residual - ref) <= 1e-9 * ref


@pytest.mark.parametrize("m,n,k", [(700, 1002, 190), (130, 18, 16), (1000, 4098, 272), (65, 2000, 64)])
def test_residual_register_kernel_ragged(m, n, k):
    # the register-resident residual kernel pinned on shapes it would not
    # take by default: a ragged last 16-column stage (n even, not a multiple
    # of 16), row strips past m, inner sizes of every instance
    import paper_2307_15572_amd as rs
    announce(f"residual register kernel m={m} n={n} k={k}")
    rng = np.random.default_rng(m + 3 * n + 5 * k)
    U = np.linalg.qr(rng.standard_normal((m, k)))[0]
    V = np.linalg.qr(rng.standard_normal((n, k)))[0]
    S = np.sort(rng.uniform(0.5, 2.0, k))[::-1].copy()
    A = (U * S) @ V.T + 1e-3 * rng.standard_normal((m, n))
    kcp = (k + 15) // 16 * 16
    try:
        rs.tune_set("residual", m, n, kcp, waves=8, registers=1)
        out = rs.residual(to_dev(A), to_dev(S), to_dev(U), to_dev(V), k)
    finally:
        rs.tune_clear()
    ref = np.linalg.norm(A - (U * S) @ V.T) / np.linalg.norm(A)
    assert abs(out.residual - ref) <= 1e-9 * ref
