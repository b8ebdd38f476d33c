"""Batched channels on concurrent streams (and replayed from a hipGraph):
each channel must equal the single-run result bitwise (the same kernels on
the same data), and the single runs meet the FP64 gate against the oracle.
Graph replays are interleaved with other eager work and compared each time."""

import numpy as np
import pytest

import synth
from oracle.method import rsvd as oracle_rsvd

from gpu_util import announce, sigma_gate, to_dev

pytestmark = pytest.mark.gpu


def _channels(count, lo, hi, tag):
    dims, dec = synth.channel_dims(count, lo, hi, tag=tag)
    mats, probs = [], []
    for c, (n, d) in enumerate(zip(dims, dec)):
        n = int(n)
        A, sigma = synth.channel(c, n, float(d), tag=tag)
        k = min(max(8, int(3 * d)), n - 8)
        mats.append(A)
        probs.append(dict(m=n, n=n, k=k, p=8, q=1, symmetric=True, seed=7, channel=c))
    return mats, probs


def _single(A, pr):
    import paper_2307_15572_amd as rs
    kw = dict(pr)
    m, n, k, p, q = (kw.pop(x) for x in ("m", "n", "k", "p", "q"))
    return rs.run(A, k, p, q, **kw)


def _check_against_single(bp, bufs, dev_mats, probs, res):
    for c, (A, pr) in enumerate(zip(dev_mats, probs)):
        one = _single(A, pr)
        r = res[c]
        assert r.rank == one.rank and r.l_used == one.l and r.flags == one.flags
        assert r.residual == one.residual
        k = one.rank
        assert np.array_equal(bufs["S"][c][:k].cpu().numpy(), one.S.cpu().numpy())
        assert np.array_equal(bufs["U"][c][:, :k].cpu().numpy(), one.U.cpu().numpy())
        assert np.array_equal(bufs["V"][c][:, :k].cpu().numpy(), one.V.cpu().numpy())


def test_batch_equals_single_runs_eager():
    import paper_2307_15572_amd as rs
    announce("batch of 10 channels, eager lanes")
    mats, probs = _channels(10, 120, 1400, tag=601)
    dev = [to_dev(A) for A in mats]
    bp = rs.BatchPlan(probs, lanes=4, use_graph=False)
    bufs = bp.allocate("cuda:0")
    bp.run_into(dev, bufs)
    res = bp.results(bufs)
    assert not bp.graph_used()
    _check_against_single(bp, bufs, dev, probs, res)
    # two channels against the oracle
    for c in (0, 3):
        pr = probs[c]
        ref = oracle_rsvd(mats[c], pr["k"], pr["p"], pr["q"], seed=7, channel=c, symmetric=True)
        s = bufs["S"][c][: res[c].rank].cpu().numpy()
        ok, worst = sigma_gate(s, ref.s[: res[c].rank])
        assert ok, (c, worst)


def test_batch_graph_replays_match_eager():
    import torch
    import paper_2307_15572_amd as rs
    announce("batch of 12 channels, graph capture + 3 replays")
    mats, probs = _channels(12, 100, 900, tag=602)
    dev = [to_dev(A) for A in mats]
    eager = rs.BatchPlan(probs, lanes=4, use_graph=False)
    eb = eager.allocate("cuda:0")
    eager.run_into(dev, eb)
    eager.results(eb)
    gp = rs.BatchPlan(probs, lanes=4, use_graph=True)
    gb = gp.allocate("cuda:0")
    for rep in range(3):
        for c in range(len(probs)):
            gb["S"][c].fill_(-1.0)
        gp.run_into(dev, gb)
        assert gp.graph_used()
        res = gp.results(gb)
        # unrelated eager work and a synchronization between replays
        x = torch.randn(512, 512, dtype=torch.float64, device="cuda:0")
        (x @ x).sum().item()
        for c in range(len(probs)):
            assert res[c].flags == 0 or res[c].flags == rs.FLAG_FULL_SVD
            assert np.array_equal(gb["S"][c].cpu().numpy(), eb["S"][c].cpu().numpy()), (rep, c)
            assert np.array_equal(gb["U"][c].cpu().numpy(), eb["U"][c].cpu().numpy()), (rep, c)
    # new output buffers: captured again, same results
    gb2 = gp.allocate("cuda:0")
    gp.run_into(dev, gb2)
    gp.results(gb2)
    for c in range(len(probs)):
        assert np.array_equal(gb2["V"][c].cpu().numpy(), eb["V"][c].cpu().numpy())


def test_batch_mixed_precision_and_threshold_rule():
    import paper_2307_15572_amd as rs
    announce("batch, mixed fp32 + rel_threshold channels")
    mats, probs = _channels(6, 200, 1200, tag=603)
    for pr in probs:
        pr.update(precision="mixed_fp32", rank_mode="rel_threshold", rank_param=1e-6,
                  k=min(pr["m"] - 24, 3 * pr["k"]), p=16, q=2)
    dev = [to_dev(A) for A in mats]
    bp = rs.BatchPlan(probs, lanes=3, use_graph=True)
    bufs = bp.allocate("cuda:0")
    bp.run_into(dev, bufs)
    res = bp.results(bufs)
    _check_against_single(bp, bufs, dev, probs, res)


def test_grouped_small_svd_values_only_channels():
    # values-only channels stop before their small SVD; one launch sweeps all
    # of them (lockstep rounds, per-channel sweep counters) and each channel
    # is finished afterwards. Every channel must equal its single run bitwise
    # (values, rank, flags, sweep count), beside two channels that want
    # vectors and run whole; graph replays with eager work between them
    import torch
    import paper_2307_15572_amd as rs
    announce("batch of 14 channels: 12 values-only (grouped small SVD) + 2 with vectors")
    mats, probs = _channels(14, 150, 1500, tag=604)
    for c, pr in enumerate(probs):
        pr.update(rank_mode="rel_threshold", rank_param=1e-6, k=min(pr["m"] - 40, 3 * pr["k"]),
                  p=16, q=2)
        if c not in (2, 9):
            pr.update(want_u=False, want_v=False, want_residual=False)
        if c == 4:
            pr.update(posterior=16)
        if c == 5:
            pr.update(form="symmetric")
        if c == 6:
            pr.update(precision="mixed_fp32", trailing_hp=1)
    dev = [to_dev(A) for A in mats]
    bp = rs.BatchPlan(probs, lanes=4, use_graph=True)
    bufs = bp.allocate("cuda:0")
    singles = [_single(A, pr) for A, pr in zip(dev, probs)]
    for rep in range(2):
        for c in range(len(probs)):
            bufs["S"][c].fill_(-1.0)
        bp.run_into(dev, bufs)
        res = bp.results(bufs)
        x = torch.randn(256, 256, dtype=torch.float64, device="cuda:0")
        (x @ x).sum().item()
        for c, one in enumerate(singles):
            r = res[c]
            assert (r.rank, r.flags, r.sweeps) == (one.rank, one.flags, one.sweeps), (rep, c)
            k = one.rank
            assert np.array_equal(bufs["S"][c][:k].cpu().numpy(), one.S.cpu().numpy()), (rep, c)
            if c in (2, 9):
                assert np.array_equal(bufs["U"][c][:, :k].cpu().numpy(), one.U.cpu().numpy())
                assert np.array_equal(bufs["V"][c][:, :k].cpu().numpy(), one.V.cpu().numpy())
    for c in (0, 7):
        pr = probs[c]
        ref = oracle_rsvd(mats[c], pr["k"], pr["p"], pr["q"], seed=7, channel=c, symmetric=True,
                          rank_mode="rel_threshold", rank_param=1e-6, want_residual=False)
        assert res[c].rank == ref.rank
        ok, worst = sigma_gate(bufs["S"][c][: res[c].rank].cpu().numpy(), ref.s)
        assert ok, (c, worst)


def test_wide_and_shifted_channels_graph():
    # panels wider than 272 (the multi-workgroup Cholesky, here with the
    # batch's share of the device) and steep spectra (the shifted passes):
    # every channel equals its single run bitwise (values, vectors, rank,
    # flags, sweeps), over graph replays with eager work between them
    import torch
    import paper_2307_15572_amd as rs
    announce("batch of 7 channels, l 120..704, graph replays")
    spec = [(700, 320, 4.0), (1100, 400, 4.0), (1500, 560, 4.0), (2000, 704, 4.0),
            (900, 200, 4.0), (1300, 480, 40.0), (600, 120, 40.0)]
    mats, probs = [], []
    for c, (n, l, r) in enumerate(spec):
        A, _ = synth.channel(c, n, l / r, tag=605)
        mats.append(A)
        probs.append(dict(m=n, n=n, k=l - 16, p=16, q=1, symmetric=True, seed=9, channel=c))
    probs[1].update(want_u=False, want_v=False, want_residual=False,
                    rank_mode="rel_threshold", rank_param=1e-6)
    probs[3].update(precision="mixed_fp32", trailing_hp=1)
    probs[6].update(want_u=False, want_v=False, want_residual=False)
    dev = [to_dev(A) for A in mats]
    singles = [_single(A, pr) for A, pr in zip(dev, probs)]
    bp = rs.BatchPlan(probs, lanes=4, use_graph=True)
    bufs = bp.allocate("cuda:0")
    for rep in range(2):
        for c in range(len(probs)):
            bufs["S"][c].fill_(-1.0)
        bp.run_into(dev, bufs)
        assert bp.graph_used()
        res = bp.results(bufs)
        x = torch.randn(256, 256, dtype=torch.float64, device="cuda:0")
        (x @ x).sum().item()
        for c, one in enumerate(singles):
            r = res[c]
            assert (r.rank, r.flags, r.sweeps) == (one.rank, one.flags, one.sweeps), (rep, c)
            k = one.rank
            assert np.array_equal(bufs["S"][c][:k].cpu().numpy(), one.S.cpu().numpy()), (rep, c)
            if probs[c].get("want_u", True):
                assert r.residual == one.residual, (rep, c)
                assert np.array_equal(bufs["U"][c][:, :k].cpu().numpy(), one.U.cpu().numpy())
                assert np.array_equal(bufs["V"][c][:, :k].cpu().numpy(), one.V.cpu().numpy())
    pr = probs[2]
    ref = oracle_rsvd(mats[2], pr["k"], pr["p"], pr["q"], seed=9, channel=2, symmetric=True)
    ok, worst = sigma_gate(bufs["S"][2][: res[2].rank].cpu().numpy(), ref.s[: res[2].rank])
    assert ok, worst


def test_grouped_small_svd_four_wave_launch_equals_single_runs():
    # more first-round block pairs than CUs: the grouped launch runs 4-wave
    # workgroups (two per CU) while the single runs use 8 waves per pair; the
    # Gram of a pair sums the same partials in the same order either way, so
    # values, ranks, flags and sweep counts agree bitwise
    import paper_2307_15572_amd as rs
    announce("batch of 16 values-only channels, l ~ 560: 4-wave grouped small SVDs")
    mats, probs = [], []
    for c in range(16):
        n = 1100 + 37 * c
        A, _ = synth.channel(c, n, 140.0, tag=606)
        mats.append(A)
        probs.append(dict(m=n, n=n, k=540 + c, p=16, q=1, symmetric=True, seed=13, channel=c,
                          want_u=False, want_v=False, want_residual=False))
    pairs = sum((-(-(pr["k"] + pr["p"]) // 16) + 1) // 2 * 2 // 2 for pr in probs)
    assert pairs > 256
    dev = [to_dev(A) for A in mats]
    singles = [_single(A, pr) for A, pr in zip(dev, probs)]
    bp = rs.BatchPlan(probs, lanes=4, use_graph=True)
    bufs = bp.allocate("cuda:0")
    bp.run_into(dev, bufs)
    res = bp.results(bufs)
    for c, one in enumerate(singles):
        r = res[c]
        assert (r.rank, r.flags, r.sweeps) == (one.rank, one.flags, one.sweeps), c
        k = one.rank
        assert np.array_equal(bufs["S"][c][:k].cpu().numpy(), one.S.cpu().numpy()), c
