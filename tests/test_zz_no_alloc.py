"""rsvd_run_noalloc (the workspace in the library's static device array)
against rsvd_run with a caller workspace: the same plan, the same inputs, the
FP64 gate on the singular values and the residual, and the vectors up to
rounding; two calls in a row, the second on a smaller problem, so the second
run finds the first one's contents in the array."""

import ctypes

import numpy as np
import pytest

import synth

from gpu_util import announce, sigma_gate, to_dev

pytestmark = pytest.mark.gpu


def _compare(rs, plan, A, k):
    ref_bufs = plan.allocate("cuda:0")
    plan.run_into(A, ref_bufs)
    r_ref = plan.result(ref_bufs)
    na_bufs = {kk: v for kk, v in plan.allocate("cuda:0").items()
               if kk not in ("work_buf", "work", "work_bytes")}
    # poison the outputs so that a run that wrote nothing cannot pass
    na_bufs["S"].fill_(float("nan"))
    if na_bufs["U"] is not None:
        na_bufs["U"].fill_(float("nan"))
    if na_bufs["V"] is not None:
        na_bufs["V"].fill_(float("nan"))
    plan.run_into_noalloc(A, na_bufs)
    r = plan.result(na_bufs)
    rs.check_flags(r.flags, "rsvd_run_noalloc")
    assert r.rank == r_ref.rank == k and r.l_used == r_ref.l_used and r.flags == r_ref.flags
    s = na_bufs["S"][: r.rank].cpu().numpy()
    s_ref = ref_bufs["S"][: r.rank].cpu().numpy()
    ok, worst = sigma_gate(s, s_ref)
    assert ok, worst
    assert abs(r.residual - r_ref.residual) <= 1e-10 * r_ref.residual + 1e-13
    U = na_bufs["U"][:, : r.rank].cpu().numpy()
    U_ref = ref_bufs["U"][:, : r.rank].cpu().numpy()
    V = na_bufs["V"][:, : r.rank].cpu().numpy()
    V_ref = ref_bufs["V"][:, : r.rank].cpu().numpy()
    # same kernels on the same data: the vectors agree to rounding
    assert np.abs(U - U_ref).max() <= 1e-10 and np.abs(V - V_ref).max() <= 1e-10


def test_noalloc_matches_rsvd_run_two_calls():
    import paper_2307_15572_amd as rs
    assert rs.lib().rsvd_noalloc_max_bytes() == 64 << 20
    cases = [(3000, 2000, 60, 16, 2, False), (700, 700, 30, 10, 1, True)]
    for m, n, k, p, q, sym in cases:
        announce(f"noalloc {m}x{n} k={k} p={p} q={q} symmetric={sym}")
        sig = synth.spectrum_pow10(min(m, n), 1.0 / 20)
        A_np = synth.symmetric(n, sig, tag=m) if sym else synth.general(m, n, sig, tag=m)
        plan = rs.Plan(m, n, k, p, q, symmetric=sym, seed=5 + m, want_residual=True)
        assert plan.workspace_bytes <= 64 << 20
        _compare(rs, plan, to_dev(A_np), k)


def test_noalloc_rejects_plans_beyond_the_array():
    # refused on the host before anything is enqueued
    import paper_2307_15572_amd as rs
    import torch
    announce("noalloc size limit")
    plan = rs.Plan(16384, 16384, 256, 16, 2, symmetric=True, want_residual=True)
    assert plan.workspace_bytes > 64 << 20
    A = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    st = rs.lib().rsvd_run_noalloc(plan._h, ctypes.c_void_p(A.data_ptr()), 16384, None, 0,
                                   ctypes.c_void_p(A.data_ptr()), None, 0, None, 0,
                                   ctypes.c_void_p(A.data_ptr()), None)
    assert st == rs.RSVD_ENOMEM
